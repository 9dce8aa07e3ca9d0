// FP64 and FP32 GEMMs on the CDNA matrix cores (v_mfma_f64_16x16x4f64,
// v_mfma_f32_16x16x4f32).
//
// Workgroup tile BM x 64, K step 16 staged through LDS (the next step's
// tiles are held in registers meanwhile), four waves.  BM = 64:
// the waves own 32 x 32 quarters as 2 x 2 MFMA tiles.  BM = 16, for outputs
// of at most 16 rows (the solvers' products of a few vectors with a whole
// subspace): the waves own the four 16 x 16 tiles side by side, so no matrix
// core work or LDS is spent on 48 rows of zeros.  Operand layout of the
// 16x16x4 instructions: A[i][k] and B[k][j] from lane i + 16 k (i, j < 16,
// k < 4); the four accumulator values of lane j + 16 q are C[q + 4 t][j]
// (f64) and C[4 q + t][j] (f32), t < 4 (both checked on the device).
//
// The tall variant splits a long K across workgroups (C = A B^T with small
// M, N) and sums the partial tiles in a fixed order, so results repeat
// bitwise.
#include <algorithm>

#include "common.h"

namespace bsex {

namespace {

typedef double double4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));

constexpr int BN = 64, BK = 16;

// rows of the workgroup tile for an M-row output
inline int bm_for(long M) { return M <= 16 ? 16 : 64; }

template <typename T>
struct MfmaOf;
template <>
struct MfmaOf<double> {
  typedef double4_t acc_t;
  static __device__ __forceinline__ acc_t step(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // row of accumulator value t of lane group q
  static __device__ __forceinline__ int row(int q, int t) { return q + 4 * t; }
};
template <>
struct MfmaOf<float> {
  typedef float4_t acc_t;
  static __device__ __forceinline__ acc_t step(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int q, int t) { return 4 * q + t; }
};

// one workgroup tile of C = alpha op(A) op(B) + beta C (in T, accumulated in T)
template <typename T, int TA, int TB, int BM>
__device__ __forceinline__ void gemm_tile(long M, long N, long K, T alpha,
                                          const T* __restrict__ A, long lda,
                                          const T* __restrict__ B, long ldb, T beta,
                                          const T* Cin, T* __restrict__ C, long ldc,
                                          long k_chunk, long c_split_stride) {
  typedef MfmaOf<T> MF;
  constexpr int WGM = BM == 64 ? 2 : 1;  // waves along M
  constexpr int WGN = 4 / WGM;           // waves along N
  constexpr int TM = BM / (16 * WGM);    // MFMA tiles per wave along M
  constexpr int TN = BN / (16 * WGN);    // and along N
  __shared__ T As[BK][BM + 1];
  __shared__ T Bs[BK][BN + 1];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave / WGN, wn = wave % WGN;
  const long m0 = (long)blockIdx.y * BM;
  const long n0 = (long)blockIdx.x * BN;
  const long kb = (long)blockIdx.z * k_chunk;
  const long ke = min(K, kb + k_chunk);
  typename MF::acc_t acc[TM][TN];
  for (int a = 0; a < TM; ++a)
    for (int b = 0; b < TN; ++b)
      for (int t = 0; t < 4; ++t) acc[a][b][t] = 0;

  // element e of a thread's share of the A tile is (m, k) = a_mk(e), of the
  // B tile (n, k) = b_nk(e); the next K step's tiles are loaded into
  // registers while the matrix cores work on the current one
  constexpr int NA = BM * BK / 256, NB = BN * BK / 256;
  auto a_mk = [&](int e, int& m, int& k) {
    if (TA) {  // A[k][m], m contiguous
      m = e % BM;
      k = e / BM;
    } else {   // A[m][k], k contiguous
      k = e % BK;
      m = e / BK;
    }
  };
  auto b_nk = [&](int e, int& n, int& k) {
    if (TB) {  // B[n][k], k contiguous
      k = e % BK;
      n = e / BK;
    } else {   // B[k][n], n contiguous
      n = e % BN;
      k = e / BN;
    }
  };
  T ra[NA], rb[NB];
  auto fetch = [&](long k0) {
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      int m, k;
      a_mk(tid + 256 * q, m, k);
      const long gm = m0 + m, gk = k0 + k;
      ra[q] = (gm < M && gk < ke) ? (TA ? A[gk * lda + gm] : A[gm * lda + gk]) : (T)0;
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      int n, k;
      b_nk(tid + 256 * q, n, k);
      const long gn = n0 + n, gk = k0 + k;
      rb[q] = (gn < N && gk < ke) ? (TB ? B[gn * ldb + gk] : B[gk * ldb + gn]) : (T)0;
    }
  };
  if (kb < ke) fetch(kb);
  for (long k0 = kb; k0 < ke; k0 += BK) {
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      int m, k;
      a_mk(tid + 256 * q, m, k);
      As[k][m] = ra[q];
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      int n, k;
      b_nk(tid + 256 * q, n, k);
      Bs[k][n] = rb[q];
    }
    __syncthreads();
    if (k0 + BK < ke) fetch(k0 + BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      const int kr = kk + (lane >> 4);
      T a[TM], b[TN];
#pragma unroll
      for (int t = 0; t < TM; ++t) a[t] = As[kr][wm * 16 * TM + t * 16 + (lane & 15)];
#pragma unroll
      for (int t = 0; t < TN; ++t) b[t] = Bs[kr][wn * 16 * TN + t * 16 + (lane & 15)];
#pragma unroll
      for (int ta = 0; ta < TM; ++ta)
#pragma unroll
        for (int tb = 0; tb < TN; ++tb)
          acc[ta][tb] = MF::step(a[ta], b[tb], acc[ta][tb]);
    }
    __syncthreads();
  }
  T* Cz = C + (long)blockIdx.z * c_split_stride;
#pragma unroll
  for (int ta = 0; ta < TM; ++ta)
#pragma unroll
    for (int tb = 0; tb < TN; ++tb)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const long gm = m0 + wm * 16 * TM + ta * 16 + MF::row(lane >> 4, t);
        const long gn = n0 + wn * 16 * TN + tb * 16 + (lane & 15);
        if (gm < M && gn < N) {
          T v = alpha * acc[ta][tb][t];
          if (beta != (T)0) v += beta * (Cin ? Cin[gm * ldc + gn] : Cz[gm * ldc + gn]);
          Cz[gm * ldc + gn] = v;
        }
      }
}

template <int TA, int TB, int BM>
__global__ __launch_bounds__(256) void k_dgemm(long M, long N, long K, double alpha,
                                               const double* __restrict__ A, long lda,
                                               const double* __restrict__ B, long ldb,
                                               double beta, const double* Cin,
                                               double* __restrict__ C, long ldc, long k_chunk,
                                               long c_split_stride) {
  gemm_tile<double, TA, TB, BM>(M, N, K, alpha, A, lda, B, ldb, beta, Cin, C, ldc, k_chunk,
                                c_split_stride);
}

template <int TA, int TB, int BM>
__global__ __launch_bounds__(256) void k_sgemm(long M, long N, long K, float alpha,
                                               const float* __restrict__ A, long lda,
                                               const float* __restrict__ B, long ldb,
                                               float beta, const float* Cin,
                                               float* __restrict__ C, long ldc, long k_chunk,
                                               long c_split_stride) {
  gemm_tile<float, TA, TB, BM>(M, N, K, alpha, A, lda, B, ldb, beta, Cin, C, ldc, k_chunk,
                               c_split_stride);
}

// C = alpha * sum_z P[z] + beta * C, fixed order over z
__global__ void k_reduce_split(long M, long N, int nz, const double* __restrict__ P, long pstride,
                               double alpha, double beta, double* __restrict__ C, long ldc) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= M * N) return;
  const long m = e / N, n = e % N;
  double s = 0.0;
  for (int z = 0; z < nz; ++z) s += P[z * pstride + m * N + n];
  double v = alpha * s;
  if (beta != 0.0) v += beta * C[m * ldc + n];
  C[m * ldc + n] = v;
}

}  // namespace

namespace {

void launch(int ta, int tb, int bm, dim3 grid, hipStream_t st, long M, long N, long K,
            double alpha, const double* A, long lda, const double* B, long ldb, double beta,
            const double* Cin, double* C, long ldc, long kc, long cstride) {
#define L3(TA_, TB_, BM_)                                                                      \
  hipLaunchKernelGGL((k_dgemm<TA_, TB_, BM_>), grid, dim3(256), 0, st, M, N, K, alpha, A, lda, \
                     B, ldb, beta, Cin, C, ldc, kc, cstride)
#define L2(TA_, TB_)    \
  if (bm == 16)         \
    L3(TA_, TB_, 16);   \
  else                  \
    L3(TA_, TB_, 64)
  if (!ta && !tb)
    L2(0, 0);
  else if (!ta && tb)
    L2(0, 1);
  else if (ta && !tb)
    L2(1, 0);
  else
    L2(1, 1);
#undef L2
#undef L3
}

void launch_s(int ta, int tb, int bm, dim3 grid, hipStream_t st, long M, long N, long K,
              float alpha, const float* A, long lda, const float* B, long ldb, float beta,
              float* C, long ldc) {
#define L3(TA_, TB_, BM_)                                                                      \
  hipLaunchKernelGGL((k_sgemm<TA_, TB_, BM_>), grid, dim3(256), 0, st, M, N, K, alpha, A, lda, \
                     B, ldb, beta, (const float*)nullptr, C, ldc, K > 0 ? K : 1, 0L)
#define L2(TA_, TB_)    \
  if (bm == 16)         \
    L3(TA_, TB_, 16);   \
  else                  \
    L3(TA_, TB_, 64)
  if (!ta && !tb)
    L2(0, 0);
  else if (!ta && tb)
    L2(0, 1);
  else if (ta && !tb)
    L2(1, 0);
  else
    L2(1, 1);
#undef L2
#undef L3
}

long tiles_of(long M, long N) {
  const long bm = bm_for(M);
  return ((M + bm - 1) / bm) * ((N + BN - 1) / BN);
}

}  // namespace

int dgemm(int ta, int tb, long M, long N, long K, double alpha, const double* A, long lda,
          const double* B, long ldb, double beta, double* C, long ldc, hipStream_t st) {
  return dgemm_from(ta, tb, M, N, K, alpha, A, lda, B, ldb, beta, nullptr, C, ldc, st);
}

int sgemm(int ta, int tb, long M, long N, long K, float alpha, const float* A, long lda,
          const float* B, long ldb, float beta, float* C, long ldc, hipStream_t st) {
  if (M <= 0 || N <= 0) return BSE_OK;
  const int bm = bm_for(M);
  const dim3 grid((unsigned)((N + BN - 1) / BN), (unsigned)((M + bm - 1) / bm), 1);
  if (grid.y > 65535) return fail(BSE_EINVAL, "sgemm: M too large for the grid");
  if (K <= 0) alpha = 0.0f;
  launch_s(ta, tb, bm, grid, st, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc);
  BSE_HIP(hipGetLastError());
  return BSE_OK;
}

int dgemm_from(int ta, int tb, long M, long N, long K, double alpha, const double* A, long lda,
               const double* B, long ldb, double beta, const double* Cin, double* C, long ldc,
               hipStream_t st) {
  if (M <= 0 || N <= 0) return BSE_OK;
  const int bm = bm_for(M);
  const dim3 grid((unsigned)((N + BN - 1) / BN), (unsigned)((M + bm - 1) / bm), 1);
  if (grid.y > 65535) return fail(BSE_EINVAL, "dgemm: M too large for the grid");
  const long kc = K > 0 ? K : 1;
  if (K <= 0) alpha = 0.0;
  launch(ta, tb, bm, grid, st, M, N, K, alpha, A, lda, B, ldb, beta, Cin, C, ldc, kc, 0L);
  BSE_HIP(hipGetLastError());
  return BSE_OK;
}

// split-K factor for an op(A) op(B) product whose tile grid is small: aim at
// ~4096 workgroups (16 per CU, so global-load latency is hidden by occupancy)
// with K chunks of at least 1024
static long k_splits(long M, long N, long K) {
  const long tiles = tiles_of(M, N);
  if (tiles >= 2048 || K < 2048) return 1;
  long s = std::min((K + 1023) / 1024, std::max(1L, 4096 / tiles));
  return std::max(s, 1L);
}

long dgemm_work(long M, long N, long K) {
  const long s = k_splits(M, N, K);
  return s > 1 ? s * M * N : 0;
}

int dgemm_ws(int ta, int tb, long M, long N, long K, double alpha, const double* A, long lda,
             const double* B, long ldb, double beta, double* C, long ldc, double* work,
             long work_len, hipStream_t st) {
  long s = k_splits(M, N, K);
  if (s <= 1 || !work || s * M * N > work_len)
    return dgemm(ta, tb, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, st);
  long kc = (K + s - 1) / s;
  kc = ((kc + BK - 1) / BK) * BK;
  s = (K + kc - 1) / kc;
  const int bm = bm_for(M);
  const dim3 grid((unsigned)((N + BN - 1) / BN), (unsigned)((M + bm - 1) / bm), (unsigned)s);
  if (grid.y > 65535) return fail(BSE_EINVAL, "dgemm: M too large for the grid");
  launch(ta, tb, bm, grid, st, M, N, K, 1.0, A, lda, B, ldb, 0.0, nullptr, work, N, kc, M * N);
  BSE_HIP(hipGetLastError());
  const long tot = M * N;
  hipLaunchKernelGGL(k_reduce_split, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, M, N,
                     (int)s, work, M * N, alpha, beta, C, ldc);
  BSE_HIP(hipGetLastError());
  return BSE_OK;
}

// K splits of a product with a long K: about TALL_TARGET workgroups in all,
// K chunks of at least 1024
constexpr long TALL_TARGET = 1024;
static long tall_splits(long M, long N, long K) {
  const long tiles = tiles_of(M, N);
  long s = TALL_TARGET / (tiles > 0 ? tiles : 1);
  const long maxs = (K + 1023) / 1024;
  if (s > maxs) s = maxs;
  if (s < 1) s = 1;
  return s;
}

long dgemm_tall_work(long M, long N, long K) { return tall_splits(M, N, K) * M * N; }

int dgemm_tall(long M, long N, long K, double alpha, const double* A, long lda, const double* B,
               long ldb, double beta, double* C, long ldc, double* work, long work_len,
               hipStream_t st) {
  if (M <= 0 || N <= 0) return BSE_OK;
  long s = tall_splits(M, N, K);
  if (s * M * N > work_len) return fail(BSE_EINVAL, "dgemm_tall: work buffer too small");
  long kc = (K + s - 1) / s;
  kc = ((kc + BK - 1) / BK) * BK;
  if (kc < BK) kc = BK;
  s = (K + kc - 1) / kc;
  if (s < 1) s = 1;
  const int bm = bm_for(M);
  const dim3 grid((unsigned)((N + BN - 1) / BN), (unsigned)((M + bm - 1) / bm), (unsigned)s);
  launch(0, 1, bm, grid, st, M, N, K, 1.0, A, lda, B, ldb, 0.0, nullptr, work, N, kc, M * N);
  BSE_HIP(hipGetLastError());
  const long tot = M * N;
  hipLaunchKernelGGL(k_reduce_split, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, M, N,
                     (int)s, work, M * N, alpha, beta, C, ldc);
  BSE_HIP(hipGetLastError());
  return BSE_OK;
}

}  // namespace bsex
