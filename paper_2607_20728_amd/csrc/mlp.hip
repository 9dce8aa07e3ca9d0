// The learned preconditioner's network on gfx950: three dense layers of width
// 128 with SiLU between them, BF16 operands on the MFMA units (FP32
// accumulation), FP32 master weights and Adam.  Forward and backward are
// hand-written: one small GEMM kernel (one wave per 16 x 16 output tile of
// v_mfma_f32_16x16x16_bf16) with fused epilogues, a loss kernel, column sums
// and the optimizer step.  Every reduction runs in a fixed order, so a step is
// deterministic.
//
//   xh = (x - mu_x)/s_x,  h1 = silu(xh W1^T + b1),  h2 = silu(h1 W2^T + b2),
//   yh = h2 W3^T + b3,    y = yh s_y + mu_y
//   L  = sum w (yh - (t - mu_y)/s_y)^2 / max(sum w, 1)
//
// Parameters are one flat FP32 vector: W1 [128][n_in], b1 [128],
// W2 [128][128], b2 [128], W3 [n_out][128], b3 [n_out].
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "context.h"

struct bse_mlp {
  int n_in = 0, n_out = 0;
  long np = 0;
  long off[7] = {0};  // W1 b1 W2 b2 W3 b3 end
  hipStream_t st = nullptr;
  float *p = nullptr, *m = nullptr, *v = nullptr, *g = nullptr, *norm = nullptr;
  uint16_t *w1 = nullptr, *w2 = nullptr, *w3 = nullptr;
  int step = 0;
  long cap = 0;
  uint16_t *xh = nullptr, *h1b = nullptr, *h2b = nullptr, *dyb = nullptr, *dz2b = nullptr,
           *dz1b = nullptr;
  float *z1 = nullptr, *z2 = nullptr, *yh = nullptr, *dy = nullptr, *dz2 = nullptr,
        *dz1 = nullptr;
  double* red = nullptr;
  std::vector<void*> allocs;
  bsex::HostStage hs;  // pinned staging of host <-> device copies
};

namespace bsex {
namespace {

constexpr int W = 128;
typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

__host__ __device__ inline uint16_t f2bf(float f) {
  uint32_t u;
  memcpy(&u, &f, 4);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40);  // quiet NaN
  u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even
  return (uint16_t)(u >> 16);
}
__host__ __device__ inline float bf2f(uint16_t b) {
  const uint32_t u = (uint32_t)b << 16;
  float f;
  memcpy(&f, &u, 4);
  return f;
}
__device__ inline float silu(float z) { return z / (1.0f + __expf(-z)); }
__device__ inline float silu_d(float z) {
  const float s = 1.0f / (1.0f + __expf(-z));
  return s * (1.0f + z * (1.0f - s));
}

// C[i][j] = sum_k a(i,k) b(k,j); a(i,k) = TA ? A[k lda + i] : A[i lda + k],
// b(k,j) = TB ? B[j ldb + k] : B[k ldb + j].  Out-of-range operands read as 0,
// so M, N, K need no padding.  One wave per 16 x 16 tile: grid (N/16, M/16).
// Epilogue: z = C + bias[j]; act 0: outf = z (then y = z scale[j] + shift[j]
// when scale is given); act 1: outf = z, outb = bf16(silu(z)); act 2:
// z *= silu'(zin[i][j]), outf = z, outb = bf16(z).
template <bool TA, bool TB>
__global__ __launch_bounds__(64) void k_mm(int M, int N, int K, const uint16_t* __restrict__ A,
                                           int lda, const uint16_t* __restrict__ B, int ldb,
                                           const float* __restrict__ bias, int act,
                                           const float* __restrict__ zin,
                                           const float* __restrict__ scale,
                                           const float* __restrict__ shift, float* outf,
                                           uint16_t* outb, int ldc) {
  const int l = threadIdx.x;
  const int i0 = blockIdx.y * 16, j0 = blockIdx.x * 16;
  const int r = l & 15, q = l >> 4;
  v4f acc = {0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < K; k0 += 16) {
    v4s av, bv;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int k = k0 + 4 * q + t;
      const int i = i0 + r, j = j0 + r;
      uint16_t a = 0, b = 0;
      if (i < M && k < K) a = TA ? A[(long)k * lda + i] : A[(long)i * lda + k];
      if (j < N && k < K) b = TB ? B[(long)j * ldb + k] : B[(long)k * ldb + j];
      av[t] = (short)a;
      bv[t] = (short)b;
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc, 0, 0, 0);
  }
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int i = i0 + 4 * q + t, j = j0 + r;
    if (i >= M || j >= N) continue;
    float z = acc[t] + (bias ? bias[j] : 0.0f);
    const long e = (long)i * ldc + j;
    if (act == 1) {
      outf[e] = z;
      outb[e] = f2bf(silu(z));
    } else if (act == 2) {
      z *= silu_d(zin[e]);
      outf[e] = z;
      outb[e] = f2bf(z);
    } else {
      outf[e] = scale ? z * scale[j] + shift[j] : z;
    }
  }
}

__global__ void k_norm_in(const float* __restrict__ x, const float* __restrict__ mu,
                          const float* __restrict__ s, long n, int nin, uint16_t* xh) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * nin) return;
  const int c = (int)(e % nin);
  xh[e] = f2bf((x[e] - mu[c]) / s[c]);
}

// loss and dL/dyh; one workgroup, fixed-order FP64 sums
__global__ __launch_bounds__(256) void k_loss(const float* __restrict__ yh,
                                              const float* __restrict__ t,
                                              const float* __restrict__ w,
                                              const float* __restrict__ mu,
                                              const float* __restrict__ s, long n, int nout,
                                              float* dy, uint16_t* dyb, double* red) {
  __shared__ double sh[256];
  const long ne = n * nout;
  double ws = 0.0;
  for (long e = threadIdx.x; e < ne; e += 256) ws += w ? (double)w[e] : 1.0;
  sh[threadIdx.x] = ws;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) sh[threadIdx.x] += sh[threadIdx.x + h];
    __syncthreads();
  }
  const double den = sh[0] > 1.0 ? sh[0] : 1.0;
  __syncthreads();
  double ls = 0.0;
  for (long e = threadIdx.x; e < ne; e += 256) {
    const int o = (int)(e % nout);
    const double we = w ? (double)w[e] : 1.0;
    const double err = (double)yh[e] - ((double)t[e] - mu[o]) / s[o];
    ls += we * err * err;
    const float d = (float)(2.0 * we * err / den);
    dy[e] = d;
    dyb[e] = f2bf(d);
  }
  sh[threadIdx.x] = ls;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) sh[threadIdx.x] += sh[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) red[0] = sh[0] / den;
}

// out[j] = sum_i A[i][j] for i < n (one thread per column, fixed order)
__global__ void k_colsum(const float* __restrict__ A, long n, int N, float* out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  double s = 0.0;
  for (long i = 0; i < n; ++i) s += A[i * N + j];
  out[j] = (float)s;
}

__global__ void k_adam(float* p, const float* __restrict__ g, float* m, float* v, long np,
                       float lr, float c1, float c2) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= np) return;
  const float gi = g[e];
  const float mi = 0.9f * m[e] + 0.1f * gi;
  const float vi = 0.999f * v[e] + 0.001f * gi * gi;
  m[e] = mi;
  v[e] = vi;
  p[e] -= lr * (mi / c1) / (sqrtf(vi / c2) + 1e-8f);
}

__global__ void k_to_bf(const float* __restrict__ x, long n, uint16_t* y) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) y[e] = f2bf(x[e]);
}

inline unsigned nb256(long n) { return (unsigned)((n + 255) / 256); }

template <typename T>
int mlp_alloc(bse_mlp* q, T** p, size_t count) {
  void* d = nullptr;
  BSE_HIP(hipMalloc(&d, sizeof(T) * std::max<size_t>(count, 1)));
  q->allocs.push_back(d);
  *p = reinterpret_cast<T*>(d);
  return BSE_OK;
}

int refresh_bf16(bse_mlp* q) {
  hipLaunchKernelGGL(k_to_bf, dim3(nb256(W * q->n_in)), dim3(256), 0, q->st, q->p + q->off[0],
                     (long)W * q->n_in, q->w1);
  hipLaunchKernelGGL(k_to_bf, dim3(nb256(W * W)), dim3(256), 0, q->st, q->p + q->off[2],
                     (long)W * W, q->w2);
  hipLaunchKernelGGL(k_to_bf, dim3(nb256(W * q->n_out)), dim3(256), 0, q->st, q->p + q->off[4],
                     (long)W * q->n_out, q->w3);
  BSE_HIP(hipGetLastError());
  return BSE_OK;
}

int ensure_cap(bse_mlp* q, long n) {
  if (n <= q->cap) return BSE_OK;
  uint16_t** bs[] = {&q->xh, &q->h1b, &q->h2b, &q->dyb, &q->dz2b, &q->dz1b};
  float** fs[] = {&q->z1, &q->z2, &q->yh, &q->dy, &q->dz2, &q->dz1};
  for (auto b : bs) {
    if (*b) {
      (void)hipFree(*b);
      q->allocs.erase(std::find(q->allocs.begin(), q->allocs.end(), (void*)*b));
    }
  }
  for (auto f : fs) {
    if (*f) {
      (void)hipFree(*f);
      q->allocs.erase(std::find(q->allocs.begin(), q->allocs.end(), (void*)*f));
    }
  }
  const long wmax = std::max<long>(W, std::max(q->n_in, q->n_out));
  BSE_TRY(mlp_alloc(q, &q->xh, (size_t)n * q->n_in));
  BSE_TRY(mlp_alloc(q, &q->h1b, (size_t)n * W));
  BSE_TRY(mlp_alloc(q, &q->h2b, (size_t)n * W));
  BSE_TRY(mlp_alloc(q, &q->dyb, (size_t)n * q->n_out));
  BSE_TRY(mlp_alloc(q, &q->dz2b, (size_t)n * W));
  BSE_TRY(mlp_alloc(q, &q->dz1b, (size_t)n * W));
  BSE_TRY(mlp_alloc(q, &q->z1, (size_t)n * W));
  BSE_TRY(mlp_alloc(q, &q->z2, (size_t)n * W));
  BSE_TRY(mlp_alloc(q, &q->yh, (size_t)n * wmax));
  BSE_TRY(mlp_alloc(q, &q->dy, (size_t)n * q->n_out));
  BSE_TRY(mlp_alloc(q, &q->dz2, (size_t)n * W));
  BSE_TRY(mlp_alloc(q, &q->dz1, (size_t)n * W));
  q->cap = n;
  return BSE_OK;
}

template <bool TA, bool TB>
int mm(bse_mlp* q, int M, int N, int K, const uint16_t* A, int lda, const uint16_t* B, int ldb,
       const float* bias, int act, const float* zin, const float* scale, const float* shift,
       float* outf, uint16_t* outb, int ldc) {
  if (M <= 0 || N <= 0) return BSE_OK;
  const dim3 g((unsigned)((N + 15) / 16), (unsigned)((M + 15) / 16));
  hipLaunchKernelGGL((k_mm<TA, TB>), g, dim3(64), 0, q->st, M, N, K, A, lda, B, ldb, bias, act,
                     zin, scale, shift, outf, outb, ldc);
  BSE_HIP(hipGetLastError());
  return BSE_OK;
}

// forward through the hidden layers; yh (normalised output) in q->yh, or the
// de-normalised y in y_out when given
int forward_impl(bse_mlp* q, long n, const float* x, float* y_out) {
  BSE_TRY(ensure_cap(q, n));
  const float* mu_x = q->norm;
  const float* s_x = q->norm + q->n_in;
  const float* mu_y = q->norm + 2 * q->n_in;
  const float* s_y = mu_y + q->n_out;
  hipLaunchKernelGGL(k_norm_in, dim3(nb256(n * q->n_in)), dim3(256), 0, q->st, x, mu_x, s_x, n,
                     q->n_in, q->xh);
  BSE_HIP(hipGetLastError());
  const int ni = (int)n;
  BSE_TRY((mm<false, true>(q, ni, W, q->n_in, q->xh, q->n_in, q->w1, q->n_in, q->p + q->off[1], 1,
                           nullptr, nullptr, nullptr, q->z1, q->h1b, W)));
  BSE_TRY((mm<false, true>(q, ni, W, W, q->h1b, W, q->w2, W, q->p + q->off[3], 1, nullptr, nullptr,
                           nullptr, q->z2, q->h2b, W)));
  if (y_out)
    return mm<false, true>(q, ni, q->n_out, W, q->h2b, W, q->w3, W, q->p + q->off[5], 0, nullptr,
                           s_y, mu_y, y_out, nullptr, q->n_out);
  return mm<false, true>(q, ni, q->n_out, W, q->h2b, W, q->w3, W, q->p + q->off[5], 0, nullptr,
                         nullptr, nullptr, q->yh, nullptr, q->n_out);
}

// splitmix64 (Steele, Lea and Flood 2014) for the initial weights
uint64_t splitmix(uint64_t& s) {
  uint64_t z = (s += 0x9e3779b97f4a7c15ull);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

int create_impl(int n_in, int n_out, uint64_t seed, hipStream_t st, bse_mlp* q) {
  q->n_in = n_in;
  q->n_out = n_out;
  q->st = st;
  const long sz[6] = {(long)W * n_in, W, (long)W * W, W, (long)n_out * W, n_out};
  q->off[0] = 0;
  for (int k = 0; k < 6; ++k) q->off[k + 1] = q->off[k] + sz[k];
  q->np = q->off[6];
  BSE_TRY(mlp_alloc(q, &q->p, q->np));
  BSE_TRY(mlp_alloc(q, &q->m, q->np));
  BSE_TRY(mlp_alloc(q, &q->v, q->np));
  BSE_TRY(mlp_alloc(q, &q->g, q->np));
  BSE_TRY(mlp_alloc(q, &q->norm, 2 * (n_in + n_out)));
  BSE_TRY(mlp_alloc(q, &q->w1, (size_t)W * n_in));
  BSE_TRY(mlp_alloc(q, &q->w2, (size_t)W * W));
  BSE_TRY(mlp_alloc(q, &q->w3, (size_t)W * n_out));
  BSE_TRY(mlp_alloc(q, &q->red, 4));
  // W ~ U(-1/sqrt(fan_in), 1/sqrt(fan_in)), b = 0
  std::vector<float> h(q->np, 0.0f);
  const int fan[3] = {n_in, W, W};
  uint64_t s = seed;
  for (int L = 0; L < 3; ++L) {
    const float a = 1.0f / std::sqrt((float)fan[L]);
    for (long e = q->off[2 * L]; e < q->off[2 * L + 1]; ++e) {
      const double u = (double)(splitmix(s) >> 11) * (1.0 / 9007199254740992.0);
      h[e] = (float)((2.0 * u - 1.0) * a);
    }
  }
  std::vector<float> nrm(2 * (n_in + n_out), 0.0f);
  for (int c = 0; c < n_in; ++c) nrm[n_in + c] = 1.0f;
  for (int o = 0; o < n_out; ++o) nrm[2 * n_in + n_out + o] = 1.0f;
  BSE_TRY(stage_h2d(&q->hs, h.data(), q->p, sizeof(float) * q->np, st));
  BSE_TRY(stage_h2d(&q->hs, nrm.data(), q->norm, sizeof(float) * nrm.size(), st));
  BSE_HIP(hipMemsetAsync(q->m, 0, sizeof(float) * q->np, st));
  BSE_HIP(hipMemsetAsync(q->v, 0, sizeof(float) * q->np, st));
  BSE_TRY(refresh_bf16(q));
  BSE_HIP(hipStreamSynchronize(st));
  return BSE_OK;
}

void destroy(bse_mlp* q) {
  if (!q) return;
  if (q->st) (void)hipStreamSynchronize(q->st);
  for (void* p : q->allocs) (void)hipFree(p);
  stage_free(&q->hs);
  delete q;
}

int train_impl(bse_mlp* q, long n, const float* x, const float* t, const float* w, float lr,
               float* loss_host, float* grad_dev) {
  BSE_TRY(forward_impl(q, n, x, nullptr));
  const int ni = (int)n, no = q->n_out, nin = q->n_in;
  const float* mu_y = q->norm + 2 * nin;
  const float* s_y = mu_y + no;
  hipLaunchKernelGGL(k_loss, dim3(1), dim3(256), 0, q->st, q->yh, t, w, mu_y, s_y, n, no, q->dy,
                     q->dyb, q->red);
  BSE_HIP(hipGetLastError());
  float* g = q->g;
  // layer 3
  BSE_TRY((mm<true, false>(q, no, W, ni, q->dyb, no, q->h2b, W, nullptr, 0, nullptr, nullptr,
                           nullptr, g + q->off[4], nullptr, W)));
  hipLaunchKernelGGL(k_colsum, dim3(1), dim3(128), 0, q->st, q->dy, n, no, g + q->off[5]);
  BSE_TRY((mm<false, false>(q, ni, W, no, q->dyb, no, q->w3, W, nullptr, 2, q->z2, nullptr, nullptr,
                            q->dz2, q->dz2b, W)));
  // layer 2
  BSE_TRY((mm<true, false>(q, W, W, ni, q->dz2b, W, q->h1b, W, nullptr, 0, nullptr, nullptr,
                           nullptr, g + q->off[2], nullptr, W)));
  hipLaunchKernelGGL(k_colsum, dim3(1), dim3(128), 0, q->st, q->dz2, n, W, g + q->off[3]);
  BSE_TRY((mm<false, false>(q, ni, W, W, q->dz2b, W, q->w2, W, nullptr, 2, q->z1, nullptr, nullptr,
                            q->dz1, q->dz1b, W)));
  // layer 1
  BSE_TRY((mm<true, false>(q, W, nin, ni, q->dz1b, W, q->xh, nin, nullptr, 0, nullptr, nullptr,
                           nullptr, g + q->off[0], nullptr, nin)));
  hipLaunchKernelGGL(k_colsum, dim3(1), dim3(128), 0, q->st, q->dz1, n, W, g + q->off[1]);
  BSE_HIP(hipGetLastError());
  if (grad_dev)
    BSE_HIP(hipMemcpyAsync(grad_dev, g, sizeof(float) * q->np, hipMemcpyDeviceToDevice, q->st));
  q->step += 1;
  const float c1 = 1.0f - std::pow(0.9f, (float)q->step);
  const float c2 = 1.0f - std::pow(0.999f, (float)q->step);
  hipLaunchKernelGGL(k_adam, dim3(nb256(q->np)), dim3(256), 0, q->st, q->p, g, q->m, q->v, q->np,
                     lr, c1, c2);
  BSE_HIP(hipGetLastError());
  BSE_TRY(refresh_bf16(q));
  double L = 0.0;
  BSE_TRY(stage_d2h(&q->hs, q->red, &L, sizeof(double), q->st));
  if (loss_host) *loss_host = (float)L;
  return BSE_OK;
}

}  // namespace

// evaluation inside the solvers: y [n][n_out] from x [n][n_in] on `st`
int mlp_eval(bse_mlp* q, long n, const float* x, float* y, hipStream_t st) {
  hipStream_t keep = q->st;
  q->st = st;
  const int rc = forward_impl(q, n, x, y);
  q->st = keep;
  return rc;
}
int mlp_n_in(const bse_mlp* q) { return q->n_in; }
int mlp_n_out(const bse_mlp* q) { return q->n_out; }

}  // namespace bsex

using namespace bsex;

extern "C" {

int bse_mlp_create(int32_t n_in, int32_t n_out, uint64_t seed, void* stream, bse_mlp** out) {
  if (!out) return fail(BSE_EINVAL, "out is NULL");
  *out = nullptr;
  if (n_in < 1 || n_in > 64 || n_out < 1 || n_out > 16)
    return fail(BSE_EINVAL, "n_in must be 1..64 and n_out 1..16");
  bse_mlp* q = nullptr;
  try {
    q = new bse_mlp();
  } catch (...) {
    return fail(BSE_ENOMEM, "host allocation failed");
  }
  const int rc = create_impl(n_in, n_out, seed, (hipStream_t)stream, q);
  if (rc != BSE_OK) {
    destroy(q);
    return rc;
  }
  *out = q;
  return BSE_OK;
}

int bse_mlp_n_params(const bse_mlp* q, int64_t* n) {
  if (!q || !n) return fail(BSE_EINVAL, "NULL argument");
  *n = q->np;
  return BSE_OK;
}

int bse_mlp_set_params(bse_mlp* q, const float* params_host) {
  if (!q || !params_host) return fail(BSE_EINVAL, "NULL argument");
  for (long e = 0; e < q->np; ++e)
    if (!std::isfinite(params_host[e])) return fail(BSE_EINVAL, "non-finite parameter %ld", e);
  BSE_TRY(stage_h2d(&q->hs, params_host, q->p, sizeof(float) * q->np, q->st));
  BSE_HIP(hipMemsetAsync(q->m, 0, sizeof(float) * q->np, q->st));
  BSE_HIP(hipMemsetAsync(q->v, 0, sizeof(float) * q->np, q->st));
  q->step = 0;
  BSE_TRY(refresh_bf16(q));
  BSE_HIP(hipStreamSynchronize(q->st));
  return BSE_OK;
}

int bse_mlp_get_params(bse_mlp* q, float* params_host) {
  if (!q || !params_host) return fail(BSE_EINVAL, "NULL argument");
  return stage_d2h(&q->hs, q->p, params_host, sizeof(float) * q->np, q->st);
}

int bse_mlp_set_norm(bse_mlp* q, const float* mu_x, const float* s_x, const float* mu_y,
                     const float* s_y) {
  if (!q || !mu_x || !s_x || !mu_y || !s_y) return fail(BSE_EINVAL, "NULL argument");
  std::vector<float> h;
  h.insert(h.end(), mu_x, mu_x + q->n_in);
  h.insert(h.end(), s_x, s_x + q->n_in);
  h.insert(h.end(), mu_y, mu_y + q->n_out);
  h.insert(h.end(), s_y, s_y + q->n_out);
  for (size_t e = 0; e < h.size(); ++e)
    if (!std::isfinite(h[e])) return fail(BSE_EINVAL, "non-finite normalisation");
  for (int c = 0; c < q->n_in; ++c)
    if (!(s_x[c] > 0)) return fail(BSE_EINVAL, "s_x[%d] must be positive", c);
  for (int o = 0; o < q->n_out; ++o)
    if (!(s_y[o] > 0)) return fail(BSE_EINVAL, "s_y[%d] must be positive", o);
  return stage_h2d(&q->hs, h.data(), q->norm, sizeof(float) * h.size(), q->st);
}

int bse_mlp_forward(bse_mlp* q, int32_t n, const float* x_dev, float* y_dev) {
  if (!q || (n > 0 && (!x_dev || !y_dev))) return fail(BSE_EINVAL, "NULL argument");
  if (n < 0) return fail(BSE_EINVAL, "n < 0");
  if (n == 0) return BSE_OK;
  BSE_TRY(forward_impl(q, n, x_dev, y_dev));
  BSE_HIP(hipStreamSynchronize(q->st));
  return BSE_OK;
}

int bse_mlp_train_step(bse_mlp* q, int32_t n, const float* x_dev, const float* t_dev,
                       const float* w_dev, float lr, float* loss_host, float* grad_dev) {
  if (!q || !x_dev || !t_dev) return fail(BSE_EINVAL, "NULL argument");
  if (n < 1) return fail(BSE_EINVAL, "n must be >= 1");
  if (!std::isfinite(lr) || lr < 0) return fail(BSE_EINVAL, "lr must be finite and >= 0");
  return train_impl(q, n, x_dev, t_dev, w_dev, lr, loss_host, grad_dev);
}

int bse_mlp_free(bse_mlp* q) {
  destroy(q);
  return BSE_OK;
}

}  // extern "C"
