// FP64 GEMM on the CDNA matrix cores (v_mfma_f64_16x16x4f64).
//
// Workgroup tile 64 x 64, K step 16 staged through LDS; four waves each own
// a 32 x 32 quarter as 2 x 2 MFMA tiles.  Operand layout of the 16x16x4 f64
// instruction: A[i][k] and B[k][j] from lane i + 16 k (i, j < 16, k < 4);
// the four accumulator values of lane j + 16 q are C[q + 4 t][j], t < 4.
//
// The tall variant splits a long K across workgroups (C = A B^T with small
// M, N) and sums the partial tiles in a fixed order, so results repeat
// bitwise.
#include <algorithm>

#include "common.h"

namespace bsex {

namespace {

typedef double double4_t __attribute__((ext_vector_type(4)));

constexpr int BM = 64, BN = 64, BK = 16;

template <int TA, int TB>
__global__ __launch_bounds__(256) void k_dgemm(long M, long N, long K, double alpha,
                                               const double* __restrict__ A, long lda,
                                               const double* __restrict__ B, long ldb,
                                               double beta, double* __restrict__ C, long ldc,
                                               long k_chunk, long c_split_stride) {
  __shared__ double As[BK][BM + 1];
  __shared__ double Bs[BK][BN + 1];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const long m0 = (long)blockIdx.y * BM;
  const long n0 = (long)blockIdx.x * BN;
  const long kb = (long)blockIdx.z * k_chunk;
  const long ke = min(K, kb + k_chunk);
  double4_t acc[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) acc[a][b] = (double4_t){0.0, 0.0, 0.0, 0.0};

  for (long k0 = kb; k0 < ke; k0 += BK) {
    // A tile: op(A)[m0 + m][k0 + k]
    for (int e = tid; e < BM * BK; e += 256) {
      int m, k;
      if (TA) {  // A[k][m], m contiguous
        m = e % BM;
        k = e / BM;
      } else {   // A[m][k], k contiguous
        k = e % BK;
        m = e / BK;
      }
      const long gm = m0 + m, gk = k0 + k;
      double v = 0.0;
      if (gm < M && gk < ke) v = TA ? A[gk * lda + gm] : A[gm * lda + gk];
      As[k][m] = v;
    }
    // B tile: op(B)[k0 + k][n0 + n]
    for (int e = tid; e < BN * BK; e += 256) {
      int n, k;
      if (TB) {  // B[n][k], k contiguous
        k = e % BK;
        n = e / BK;
      } else {   // B[k][n], n contiguous
        n = e % BN;
        k = e / BN;
      }
      const long gn = n0 + n, gk = k0 + k;
      double v = 0.0;
      if (gn < N && gk < ke) v = TB ? B[gn * ldb + gk] : B[gk * ldb + gn];
      Bs[k][n] = v;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      const int kr = kk + (lane >> 4);
      double a[2], b[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        a[t] = As[kr][wm * 32 + t * 16 + (lane & 15)];
        b[t] = Bs[kr][wn * 32 + t * 16 + (lane & 15)];
      }
#pragma unroll
      for (int ta = 0; ta < 2; ++ta)
#pragma unroll
        for (int tb = 0; tb < 2; ++tb)
          acc[ta][tb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ta], b[tb], acc[ta][tb], 0, 0, 0);
    }
    __syncthreads();
  }
  double* Cz = C + (long)blockIdx.z * c_split_stride;
#pragma unroll
  for (int ta = 0; ta < 2; ++ta)
#pragma unroll
    for (int tb = 0; tb < 2; ++tb)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const long gm = m0 + wm * 32 + ta * 16 + (lane >> 4) + 4 * t;
        const long gn = n0 + wn * 32 + tb * 16 + (lane & 15);
        if (gm < M && gn < N) {
          double v = alpha * acc[ta][tb][t];
          if (beta != 0.0) v += beta * Cz[gm * ldc + gn];
          Cz[gm * ldc + gn] = v;
        }
      }
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

int dgemm(int ta, int tb, long M, long N, long K, double alpha, const double* A, long lda,
          const double* B, long ldb, double beta, double* C, long ldc, hipStream_t st) {
  if (M <= 0 || N <= 0) return BSE_OK;
  const dim3 grid((unsigned)((N + BN - 1) / BN), (unsigned)((M + BM - 1) / BM), 1);
  if (grid.y > 65535) return fail(BSE_EINVAL, "dgemm: M too large for the grid");
  const long kc = K > 0 ? K : 1;
  if (K <= 0) alpha = 0.0;
#define LAUNCH(TA_, TB_)                                                                    \
  hipLaunchKernelGGL((k_dgemm<TA_, TB_>), grid, dim3(256), 0, st, M, N, K, alpha, A, lda, B, \
                     ldb, beta, C, ldc, kc, 0L)
  if (!ta && !tb)
    LAUNCH(0, 0);
  else if (!ta && tb)
    LAUNCH(0, 1);
  else if (ta && !tb)
    LAUNCH(1, 0);
  else
    LAUNCH(1, 1);
#undef LAUNCH
  BSE_HIP(hipGetLastError());
  return BSE_OK;
}

// split-K factor for an op(A) op(B) product whose tile grid is small: aim at
// ~4096 workgroups (16 per CU, so global-load latency is hidden by occupancy)
// with K chunks of at least 1024
static long k_splits(long M, long N, long K) {
  const long tiles = ((M + BM - 1) / BM) * ((N + BN - 1) / BN);
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
  const dim3 grid((unsigned)((N + BN - 1) / BN), (unsigned)((M + BM - 1) / BM), (unsigned)s);
  if (grid.y > 65535) return fail(BSE_EINVAL, "dgemm: M too large for the grid");
#define LAUNCH(TA_, TB_)                                                                       \
  hipLaunchKernelGGL((k_dgemm<TA_, TB_>), grid, dim3(256), 0, st, M, N, K, 1.0, A, lda, B, ldb, \
                     0.0, work, N, kc, M * N)
  if (!ta && !tb)
    LAUNCH(0, 0);
  else if (!ta && tb)
    LAUNCH(0, 1);
  else if (ta && !tb)
    LAUNCH(1, 0);
  else
    LAUNCH(1, 1);
#undef LAUNCH
  BSE_HIP(hipGetLastError());
  const long tot = M * N;
  hipLaunchKernelGGL(k_reduce_split, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, M, N,
                     (int)s, work, M * N, alpha, beta, C, ldc);
  BSE_HIP(hipGetLastError());
  return BSE_OK;
}

static long tall_splits(long M, long N, long K) {
  const long tiles = ((M + BM - 1) / BM) * ((N + BN - 1) / BN);
  long s = 1024 / (tiles > 0 ? tiles : 1);
  const long maxs = (K + 4095) / 4096;
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
  const dim3 grid((unsigned)((N + BN - 1) / BN), (unsigned)((M + BM - 1) / BM), (unsigned)s);
  hipLaunchKernelGGL((k_dgemm<0, 1>), grid, dim3(256), 0, st, M, N, K, 1.0, A, lda, B, ldb, 0.0,
                     work, N, kc, M * N);
  BSE_HIP(hipGetLastError());
  const long tot = M * N;
  hipLaunchKernelGGL(k_reduce_split, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, M, N,
                     (int)s, work, M * N, alpha, beta, C, ldc);
  BSE_HIP(hipGetLastError());
  return BSE_OK;
}

}  // namespace bsex
