// Launchers of the element-wise, transform-side and tau kernels.
#pragma once
#include "common.h"

namespace bsex {

// Orbitals are stored as rows of n_pw real coefficients.  A "set" is a block
// of `nv` orbitals; `nset` sets are stored back to back.  Real-space grids
// hold two orbitals of one set per complex grid (packed: x = orbital 2p,
// y = orbital 2p+1), nvh = ceil(nv/2) grids per set.
struct SphereMap {
  const int* idx_p;   // [nhalf] position of +G in a grid (or compact array)
  const int* idx_m;   // [nhalf] position of -G
  int nhalf;
  int npw;
  long nr;            // stride between grids
  double omega;
  long zero = 0;      // position of G = 0
};

// grid[set][p][r] = packed coefficients of X (grid must be zero first unless
// accumulate = 1, in which case the coefficients are added).
int scatter_sets(const SphereMap& m, const double* X, int nv, int nset, double2* grid,
                 int accumulate, hipStream_t st);
int scatter_sets(const SphereMap& m, const double* X, int nv, int nset, float2* grid,
                 int accumulate, hipStream_t st);
int scatter_sets(const SphereMap& m, const float* X, int nv, int nset, float2* grid,
                 int accumulate, hipStream_t st);
// Y[set][v][j] = scale * <e_j | grid>  (+ (T_j + shift - eps_v) * A[set][v][j] if A)
// (+ beta * Y).  The grid holds N_r times the Fourier coefficients when it
// comes straight from a forward transform, so callers pass scale = 1/N_r.
int gather_sets(const SphereMap& m, const double2* grid, int nv, int nset, double scale,
                const double* A, const double* T, const double* eps, double shift, double beta,
                double* Y, hipStream_t st);
int gather_sets(const SphereMap& m, const float2* grid, int nv, int nset, double scale,
                const double* A, const double* T, const double* eps, double shift, double beta,
                double* Y, hipStream_t st);
// the coefficients alone, in FP32: Y[set][v][j] = scale * <e_j | grid>
int gather_sets(const SphereMap& m, const float2* grid, int nv, int nset, double scale, float* Y,
                hipStream_t st);
// grid[g][r] *= f[r] * scale  (real field f of length nr)
int mul_real_field(double2* grid, long ngrid, long nr, const double* f, double scale,
                   hipStream_t st);
int mul_real_field(float2* grid, long ngrid, long nr, const float* f, float scale,
                   hipStream_t st);
// y[i] = (float)x[i]
int to_f32(const double* x, float* y, long n, hipStream_t st);
int to_f64(const float* x, double* y, long n, hipStream_t st);
// X[i][j] = g_ij / (1 + T_j), g_ij standard normal from a counter-based
// generator of the given seed (the same for any launch shape)
int random_smooth(double* X, long rows, long len, const double* T, unsigned long long seed,
                  hipStream_t st);
// out[r] = Re(grid[r]) for one grid
int real_part(const double2* grid, long nr, double* out, hipStream_t st);
// drho[b/2][r] packed over vectors: drho_b(r) = sum_v phi_v(r) a_{b,v}(r)
int transition_density(const double2* phir, const double2* a, int nv, int nb, long nr,
                       double2* drho, hipStream_t st);
int transition_density(const float2* phir, const float2* a, int nv, int nb, long nr, float2* drho,
                       hipStream_t st);
// z = kD * V a + s * Vdrho_b phi - y   (y may be NULL, vdrho may be NULL); in place into y or out
int combine(const double2* a, const double2* phir, const double* V, const double2* vdrho,
            const double2* y, double2* out, int nv, int nb, long nr, double s, int with_v,
            hipStream_t st);
int combine(const float2* a, const float2* phir, const float* V, const float2* vdrho,
            const float2* y, float2* out, int nv, int nb, long nr, double s, int with_v,
            hipStream_t st);
// pair densities of 8x8 blocks [blk0, blk0 + nblk) of the upper triangle
int pair_density(const double2* phir, int nv, const int2* blkIJ, long nblk, long nr,
                 double2* grids, hipStream_t st);
int pair_density(const float2* phir, int nv, const int2* blkIJ, long nblk, long nr,
                 float2* grids, hipStream_t st);
// natural tau tile (packed grids, 64 elements per block) -> blocked stream layout
int tau_store(const double2* grids, const int2* blkIJ, long nblk, long nr, int R, double* dst,
              long dst_nblk, long dst_blk0, hipStream_t st);
int tau_store(const double2* grids, const int2* blkIJ, long nblk, long nr, int R, float* dst,
              long dst_nblk, long dst_blk0, hipStream_t st);
int tau_store(const float2* grids, const int2* blkIJ, long nblk, long nr, int R, float* dst,
              long dst_nblk, long dst_blk0, hipStream_t st);
// optional epilogue of the last stream launch: write z = with_v V a +
// s (v_c*Drho_b) phi - y (vdrho may be NULL) instead of y
struct FuseArgs {
  const double* V;
  const double2* vdrho;
  const double2* phir;
  double s;
  int with_v;
};
struct FuseArgsF {
  const float* V;
  const float2* vdrho;
  const float2* phir;
  double s;
  int with_v;
};
// y[b][v] (+)= sum_v' tau_{vv'} a[b][v'] over the blocks of one buffer; with
// fuse != NULL, y receives z instead and may alias a.  R grid points per
// workgroup (1 or 2, the layout tau was stored in); bl selects the kernel:
// 1 = quad-shared loads (the default: four lanes share a grid point's 8 trial
// vectors, each reads two columns of a block and DPP broadcasts give all four
// lanes the whole block), 4 or 2 = that many lanes share a grid point's
// vectors and each reads the whole block.  rows > 0: the blocks touch only bands
// row0 .. row0 + rows - 1 (multiples of 8), and only those bands of a and y
// are read and written (not with fuse); rows = 0: every band.
int tau_stream(const double* tau, long buf_nblk, long nblk, const int2* blkIJ, int R,
               const double2* a, double2* y, int nb, int nv, long nr, int accumulate,
               size_t max_lds, hipStream_t st, const FuseArgs* fuse = nullptr, int bl = 1,
               int row0 = 0, int rows = 0);
// FP32 variant (tau, a, y in FP32; products in FP32, sums in FP64 LDS)
int tau_stream(const float* tau, long buf_nblk, long nblk, const int2* blkIJ, int R,
               const float2* a, float2* y, int nb, int nv, long nr, int accumulate,
               size_t max_lds, hipStream_t st, const FuseArgsF* fuse = nullptr, int bl = 1,
               int row0 = 0, int rows = 0);
size_t tau_stream_lds(int nv, int R, size_t elem = sizeof(double), int bl = 1);
// raise the dynamic-LDS limit of the stream kernels (bytes <= device maximum)
int tau_stream_set_lds_limit(size_t bytes);

// potential V(G) of Gaussian sites on the full grid (Nyquist zero), complex
int site_potential(const double* xyz, const double* depth, const double* width, int nsites,
                   const int grid[3], const double cell[3], double2* out, hipStream_t st);
// Coulomb kernel 4 pi/|G|^2 on every grid frequency (minimum image), 0 at G = 0
int coulomb_kernel(const int grid[3], const double cell[3], double* out, hipStream_t st);
// rho_t(r) = sum_v a_v^2 - phi_v phit_v + 2 z_v phi_v  (one set of nv orbitals)
int force_density(const double2* a, const double2* phit, const double2* z, const double2* phir,
                  int nv, long nr, double2* rho, hipStream_t st);
// partial sums for dw/dR: out[site][3] (host) from the forward transform of rho
// rho[r] = (sum_v phi_v(r)^2, 0) over the nv orbitals of phir
int occupied_density(const double2* phir, int nv, long nr, double2* rho, hipStream_t st);
// self-consistent KS model: from rho_occ = sum_v phi_v^2 (real part), with
// rho = occ rho_occ: V_xc and f_xc of Slater exchange with the density floor
// floor_ (formulas at the kernel); rho_out (optional) receives rho
int xc_fields(const double2* rho_occ, long nr, double occ, double floor_, double* vxc,
              double* fxc, double* rho_out, hipStream_t st);
// exchange-like terms sum_w L_w (v_c * (M_w x)): pair grids (M_2q x, M_2q+1 x)
// for the real grid function x = component xc of x2 (M holds nv functions
// packed two per complex grid; an odd nv leaves the last .y of M zero), and
// o2.{x|y}(r) += scale sum_w L_w(r) P_w(r)
int pair_times(const double2* M, int nv, const double2* x2, int xc, long nr, double2* out,
               hipStream_t st);
int contract_pairs(const double2* L, const double2* P, int nv, long nr, double2* o2, int oc,
                   double scale, hipStream_t st);
// w <- scale (w + f_xc t) on ngrid complex grids (f_Hxc * t once w = v_c * t)
int hxc_field(double2* w, const double2* t, const double* fxc, long ngrid, long nr, double scale,
              hipStream_t st);
int force_reduce(const double2* rhoG, const double* xyz, const double* depth,
                 const double* width, int nsites, const int grid[3], const double cell[3],
                 double* part, long part_len, double* out_dev, hipStream_t st);
long force_reduce_work(int nsites, long nr);

// ---- vector helpers for the solvers (deterministic reductions) --------------------------
// out[i] = sum_j A[i*len + j] * B[i*len + j], i < rows (fixed-order split
// reduction through `work`, which must hold row_dots_work(rows, len) doubles)
int row_dots(const double* A, const double* B, long rows, long len, double* out, double* work,
             long work_len, hipStream_t st);
long row_dots_work(long rows, long len);
// Y[i][j] = a[i] * X[i][j] + b[i] * Y[i][j]  (a or b NULL means 1)
int row_axpby(const double* a, const double* X, const double* b, double* Y, long rows, long len,
              hipStream_t st);
// Y[i][j] *= s[i]
int row_scale(const double* s, double* Y, long rows, long len, hipStream_t st);
// p[0..n) = 0 by a kernel (safe inside captured graphs, unlike a memset node)
int zero_fill(double* p, long n, hipStream_t st);
// Y = alpha X + beta Y over n elements
int axpby(double alpha, const double* X, double beta, double* Y, long n, hipStream_t st);
// Davidson preconditioner: T[k][v][j] = R[k][v][j] / clamp(Tk_j - eps_v + shift_v - theta_k),
// shift_v = shift + (vshift ? vshift[v] : 0)
int precond_davidson(const double* R, double* T, const double* Tk, const double* eps,
                     const double* theta, double shift, int nk, int nv, int npw, hipStream_t st,
                     const double* vshift = nullptr);
// CG preconditioner: T[v][j] = R[v][j] / max(Tk_j - eps_v + shift_v, 0.1),
// shift_v = vshift ? vshift[v] : shift
int precond_cg(const double* R, double* T, const double* Tk, const double* eps, double shift,
               int nv, int npw, hipStream_t st, const double* vshift = nullptr);
// C[k][v][c] /= clamp(eps[nv + c] - eps[v] + shift - (theta ? theta[k] : 0)), |den| >= dmin
int coarse_scale(double* C, int nk, int nv, int nc, const double* eps, const double* theta,
                 double shift, double dmin, hipStream_t st);
// Per-band sums for the learned preconditioner's features: out[v][0] =
// sum_j Tk_j Phi_vj^2, [1] = sum_j U_vj^2, [2] = sum_j U_vj^2 / max(Tk_j - eps_v
// + shift, 0.1), [3] = sum_r phi_v(r)^4 (phir packs two bands per complex grid).
// U may be NULL (then [1] = [2] = 0).
int band_features(const double* Phi, const double* Tk, const double* eps, const double* U,
                  const double2* phir, double shift, int nv, int npw, long nr, double* out,
                  hipStream_t st);
}  // namespace bsex
