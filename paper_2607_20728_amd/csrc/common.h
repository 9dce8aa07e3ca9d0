// Internal declarations of the bsex library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/bsex.h"

namespace bsex {

// ---- XCD grouping of workgroups ----------------------------------------------
// Workgroup b of a launch runs on XCD b mod 8 (round-robin dispatch), and each
// XCD has its own L2.  For a launch of nsub workgroups per item over items
// rounded up to a multiple of 8 (round8), xcd_item maps b to (item, sub) so
// that every workgroup of one item runs on the same XCD and the item's shared
// inputs are fetched into one L2 only; a bijection of [0, nsub * round8(n)).
// BSEX_XCD_GROUP=0 keeps the plain order (item = b / nsub).
constexpr int kXcds = 8;
inline long round8(long n) { return (n + kXcds - 1) / kXcds * kXcds; }
__device__ __forceinline__ void xcd_item(long b, int nsub, bool group, long& item, int& sub) {
  if (!group) {
    item = b / nsub;
    sub = (int)(b % nsub);
    return;
  }
  const long i = b / kXcds;
  item = (i / nsub) * kXcds + (b % kXcds);
  sub = (int)(i % nsub);
}
bool xcd_group_on();

// ---- error reporting --------------------------------------------------------
void set_error(const char* fmt, ...);
int fail(int code, const char* fmt, ...);

#define BSE_HIP(call)                                                        \
  do {                                                                       \
    hipError_t e_ = (call);                                                  \
    if (e_ != hipSuccess)                                                    \
      return ::bsex::fail(BSE_EHIP, "%s failed: %s (%s:%d)", #call,          \
                          hipGetErrorString(e_), __FILE__, __LINE__);        \
  } while (0)

#define BSE_TRY(call)                 \
  do {                                \
    int rc_ = (call);                 \
    if (rc_ != BSE_OK) return rc_;    \
  } while (0)

// ---- host <-> device copies ------------------------------------------------------
// A pinned host buffer through which every copy between device memory and a
// caller's (pageable) host buffer goes; synchronous on `st` when it returns.
struct HostStage {
  void* p = nullptr;
  size_t bytes = 0;
};
int stage_d2h(HostStage* s, const void* dev, void* host, size_t bytes, hipStream_t st);
int stage_h2d(HostStage* s, const void* host, void* dev, size_t bytes, hipStream_t st);
void stage_free(HostStage* s);

// ---- basis (host) -------------------------------------------------------------
struct Basis {
  double cell[3];
  int grid[3];
  double ecut, omega;
  long nr;
  int npw, nhalf;
  std::vector<int> mill_half;   // [nhalf][3]
  std::vector<int> idx_p, idx_m;  // linear grid index of +G / -G
  std::vector<double> g2;       // |G|^2 per basis function [npw]
};
int basis_build(const double cell[3], const int grid[3], double ecut, Basis* b);

// ---- FFT ------------------------------------------------------------------------
struct FftAxis {
  int n = 0;
  int nrad = 0;
  int rad[8] = {0};
  double2* tw = nullptr;  // device, exp(-2 pi i k / n), k < n
  float2* twf = nullptr;  // the same in FP32
};
struct FftPlan {
  int N[3] = {0, 0, 0};
  long nr = 0;
  size_t max_lds = 65536;
  bool ct_plane[2] = {false, false}, ct_axis[2] = {false, false};  // [FP64, FP32], in use
  bool ct_plane_ok[2] = {false, false}, ct_axis_ok[2] = {false, false};  // available
  bool prune[2] = {false, false};  // pruned sphere-plane kernels [FP64, FP32]
  bool axis_direct[2] = {false, false};  // axis-1 pass with direct first/last pass
  FftAxis ax[3];
};
int fft_plan_init(FftPlan* p, const int grid[3]);
// runtime = true: use the runtime-length kernels even where compile-time ones exist
void fft_plan_set_runtime(FftPlan* p, bool runtime);
void fft_plan_free(FftPlan* p);
// In-place batched 3-D complex transform of [batch][N1][N2][N3] (N3 fastest).
// dir = -1: sum_r f(r) exp(-i G.r); dir = +1: sum_G f(G) exp(+i G.r).  No scaling.
int fft3d(const FftPlan& p, double2* data, long batch, int dir, hipStream_t st);
int fft3d(const FftPlan& p, float2* data, long batch, int dir, hipStream_t st);

// Sphere <-> grid maps of the pruned transforms: the full sphere (+G and -G
// of every half-sphere vector, and G = 0) grouped by plane i1.
struct SpherePlan {
  int nplanes = 0, nent = 0, e_zero = 0, nmax1 = 0;
  int m2 = 0, m3 = 0;  // largest |n2|, |n3| of the sphere's modes
  int *plane_i1 = nullptr, *plane_off = nullptr, *ent_pos = nullptr, *ent_code = nullptr;
  int *e_plus = nullptr, *e_minus = nullptr;  // entry index of +G_k / -G_k
  int* plane_sp = nullptr;  // [N1]: sphere plane of grid plane i1, -1 when it holds no mode
};
int sphere_plan_build(const FftPlan& p, const Basis& b, SpherePlan* sp);
void sphere_plan_free(SpherePlan* sp);
// grid[set][p] = sum_G f(G) e^{iGr} of orbitals 2p, 2p+1 of each set (packed),
// f(0) = x0/sqrt(Omega), f(+-G) = (xc -+ i xs)/sqrt(2 Omega).  Planes that miss
// the sphere are left unwritten by the first kernel and read as zero.
int sphere_to_grid(const FftPlan& p, const SpherePlan& sp, double omega, const double* X, int nv,
                   int nset, double2* grid, hipStream_t st);
int sphere_to_grid(const FftPlan& p, const SpherePlan& sp, double omega, const double* X, int nv,
                   int nset, float2* grid, hipStream_t st);
// compact[g][e] = sum_r grid[g](r) e^{-i G_e.r} for the sphere entries e only
// (the grid is overwritten).
int grid_to_compact(const FftPlan& p, const SpherePlan& sp, double2* grid, long batch,
                    double2* compact, hipStream_t st);
int grid_to_compact(const FftPlan& p, const SpherePlan& sp, float2* grid, long batch,
                    float2* compact, hipStream_t st);
// Forward 3-D FFT of the pair grids of a W build (Eqs. 2c, 3), the pointwise
// work fused into the last (plane) pass: each grid leaves as its transform
// times f(G) * s (zero when f is NULL: no bare Coulomb part) and, when
// compact is set, the transform's sphere entries (unscaled) go to
// compact[g][e] as grid_to_compact writes them (the PDEP projection reads
// them there).
int fft3d_fwd_w(const FftPlan& p, const SpherePlan& sp, double2* data, long batch,
                const double* f, double s, double2* compact, hipStream_t st);
int fft3d_fwd_w(const FftPlan& p, const SpherePlan& sp, float2* data, long batch, const float* f,
                float s, float2* compact, hipStream_t st);
// The same transform with the pair grids formed inside its first pass from
// the packed orbitals orb and the block list IJ (nblk blocks of 32 grids, the
// tile layout of pair_density).  It needs a direct-access pass for the
// axis-1 length in that precision (fwd_pairs_supported(p, f32) tells; the
// call fails otherwise).
bool fwd_pairs_supported(const FftPlan& p, bool f32);
int fft3d_fwd_pairs(const FftPlan& p, const SpherePlan& sp, const double2* orb, int nv,
                    const int2* IJ, long nblk, double2* data, const double* f, double s,
                    double2* compact, hipStream_t st);
int fft3d_fwd_pairs(const FftPlan& p, const SpherePlan& sp, const float2* orb, int nv,
                    const int2* IJ, long nblk, float2* data, const float* f, float s,
                    float2* compact, hipStream_t st);
// ... and with grid q < nm formed as M[q] times the real field x
// (component xc of the packed grid x2), the pair products of the
// exchange-like terms
int fft3d_fwd_times(const FftPlan& p, const SpherePlan& sp, const double2* M, long nm,
                    const double2* x2, int xc, double2* data, const double* f, double s,
                    double2* compact, hipStream_t st);

// ---- GEMM -----------------------------------------------------------------------
// C[M][N] = alpha op(A) op(B) + beta C, row-major, FP64 MFMA.
// op(A) = A[M][K] (ta = 0) or A^T with A[K][M] (ta = 1); op(B) likewise.
int dgemm(int ta, int tb, long M, long N, long K, double alpha, const double* A, long lda,
          const double* B, long ldb, double beta, double* C, long ldc, hipStream_t st);
// the same in FP32 (FP32 MFMA, FP32 accumulation)
int sgemm(int ta, int tb, long M, long N, long K, float alpha, const float* A, long lda,
          const float* B, long ldb, float beta, float* C, long ldc, hipStream_t st);
// the same with the beta term read from Cin (same layout and ldc) instead of
// C: C = alpha op(A) op(B) + beta Cin.  Cin = NULL reads C; otherwise Cin
// must not overlap C.
int dgemm_from(int ta, int tb, long M, long N, long K, double alpha, const double* A, long lda,
               const double* B, long ldb, double beta, const double* Cin, double* C, long ldc,
               hipStream_t st);
// dgemm with K split across workgroups when the output tiles are too few to
// fill the device (partials in `work`, summed in a fixed order)
int dgemm_ws(int ta, int tb, long M, long N, long K, double alpha, const double* A, long lda,
             const double* B, long ldb, double beta, double* C, long ldc, double* work,
             long work_len, hipStream_t st);
long dgemm_work(long M, long N, long K);
// C[M][N] = alpha A[M][K] B[N][K]^T + beta C for small M, N and long K
// (split over K with a fixed-order reduction; work buffer owned by the caller).
int dgemm_tall(long M, long N, long K, double alpha, const double* A, long lda,
               const double* B, long ldb, double beta, double* C, long ldc,
               double* work, long work_len, hipStream_t st);
long dgemm_tall_work(long M, long N, long K);

// ---- host dense linear algebra ------------------------------------------------------
// Symmetric eigen-decomposition: A[n][n] row-major (overwritten by eigenvectors,
// column j = vector j), w ascending.
int host_syev(int n, double* A, double* w);
// Lower Cholesky in place; returns non-zero when not positive definite.
int host_cholesky(int n, double* A);
// in-place inverse of a lower-triangular L (row-major, upper part zero);
// returns nonzero on a zero or non-finite diagonal
int host_trinv_lower(int n, double* L);
}  // namespace bsex
