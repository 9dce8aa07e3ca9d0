// The library context: device-resident system data, work buffers, tau cache.
#pragma once
#include <vector>

#include "common.h"
#include "kernels.h"

namespace bsex {

enum Phase {
  PH_PROJ = 0,   // occupied projector (overlap and update GEMMs)
  PH_FFT_INV,    // sphere -> grid scatter and inverse transforms
  PH_K1E,        // transition density and Poisson solve
  PH_TAU_STREAM, // tau contraction over the cached blocks (K1d)
  PH_TAU_TILE,   // tau contraction over blocks rebuilt during the call
  PH_TAU_BUILD,  // tau tiles rebuilt during an apply
  PH_COMBINE,    // V a + s v_c*Drho phi - y
  PH_FFT_FWD,    // forward transforms and gather (with the diagonal term)
  PH_SOLVER,     // Davidson / CG bookkeeping (dots, small GEMMs)
  PH_INIT_TAU,   // tau cache build at init
  PH_GS,         // ground-state eigensolver
  PH_COUNT
};

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};
// process-wide cache of device blocks across contexts (bse_memory_cache)
bool cache_keeps();
void cache_put(const DevBuf& b);
int memory_cache(int on);
// hipMemGetInfo with this device's cached blocks counted as free
int mem_info(size_t* freeb, size_t* totalb);

}  // namespace bsex

struct bse_ctx {
  bsex::Basis basis;
  int nv = 0, nvh = 0, npdep = 0, nsites = 0, kmask = 0, norb = 0, n_extra = 0;
  double scissor = 0, spin = 2, gap_min = 0, gs_tol = 1e-10, gs_resid = -1, ks_gap = -1;
  int gs_sweeps = 0;
  // self-consistent KS model (0: H = T + V_ext fixed)
  int ks = 0, scf_iters = 0, scf_max_iter = 200;
  double rho_floor = 1e-3, scf_tol = 1e-10, scf_resid = -1;
  double* Vext = nullptr;     // [nr] V_ext (Vr holds V_ext + V_H + V_xc)
  double* fxc = nullptr;      // [nr] f_xc at the ground-state density
  double* rho_ks = nullptr;   // [nr] ground-state density 2 sum phi^2
  double alpha = 0.0;         // exact-exchange fraction alpha_EXX of H_KS
  double2* xpair = nullptr;   // [nvh][nr] pair grids of the exchange terms
  // PDEP work of the exchange form of W (coupling beyond the TDA):
  // sphere coefficients [nv][npw], PDEP projections [nv][npdep], result [nv][npw]
  double *wx_RS = nullptr, *wx_T = nullptr, *wx_F = nullptr;
  double2* wx_cmp = nullptr;  // [nvh][npw] sphere entries of the pair transforms
  double2* xgrid = nullptr;   // [xgrid_sets][nvh][nr] -alpha K_x a of an apply block
  int xgrid_sets = 0;
  double t_gs_ms = 0, t_tau_ms = 0, t_tau_alloc_ms = 0, t_init_ms = 0;  // init stages, wall
  hipStream_t st = nullptr;
  int dev = -1;               // device the context was initialised on
  bsex::HostStage hstage;     // pinned staging of every host <-> device copy
  bsex::FftPlan fft;
  bsex::SphereMap map{};     // sphere <-> full grid
  bsex::SpherePlan sp;        // pruned transforms
  bsex::SphereMap cmap{};    // sphere <-> compact transform output
  double2* compact = nullptr;
  long compact_grids = 0;
  std::vector<bsex::DevBuf> allocs;
  std::vector<bsex::DevBuf> pool;  // released blocks kept for reuse
  // device system data
  int *idx_p = nullptr, *idx_m = nullptr;
  double* T = nullptr;        // [npw] |G|^2/2
  double* Vr = nullptr;       // [nr] V(r)
  double* vc = nullptr;       // [nr] 4 pi/|G|^2 (0 at G = 0)
  double* Phi = nullptr;      // [norb][npw]
  double* eps_d = nullptr;    // [norb]
  double2* phir = nullptr;    // [nvh][nr]
  double* Pt = nullptr;       // [npw][npdep] v_c^1/2 P
  double* Ptc = nullptr;      // [npw][npdep] v_c^1/2 P c
  double* sites = nullptr;    // xyz[3n] | depth[n] | width[n]
  int2* blkIJ = nullptr;      // [nblk]
  std::vector<int2> blkIJ_h;  // the same on the host
  std::vector<double> eps_h;  // [norb]
  std::vector<double> site_h; // same layout as sites
  // tau
  int R = 1;
  size_t max_lds = 65536;
  long nblk = 0, nblk_cached = 0, tile_blk = 0;
  int tau_policy = BSE_TAU_AUTO;
  double* tau_cache = nullptr;
  double2* tile_grids = nullptr;
  double *tile_RS = nullptr, *tile_T = nullptr, *tile_F = nullptr;
  double2* tile_cmp = nullptr;  // sphere entries of the tile's transforms [grid][n_pw]
  double* rebuild_buf = nullptr;
  // apply work, chunks of at most nbc vectors
  int nbc = 0;
  double *A_s = nullptr, *Zs = nullptr, *Ov = nullptr;
  double2 *agrid = nullptr, *ygrid = nullptr, *drho = nullptr;
  double* gw = nullptr;
  long gw_len = 0;
  double* rdw = nullptr;  // row_dots partial sums
  long rdw_len = 0;
  // mixed precision (FP32 grids, FFTs and tau; FP64 projector, diagonal, solvers)
  int precision = BSE_FP64;   // capability the context was built with
  int active = BSE_FP64;      // precision of the operator applies
  int Rf = 2;                 // grid points per stream workgroup, FP32 layout
  int tau_bl = 1;             // stream kernel: 1 quad-shared loads, or 4 / 2 lanes per grid
                              // point reading whole blocks
  float2* phir_f = nullptr;   // [nvh][nr]
  float* Vr_f = nullptr;      // [nr]
  float* vc_f = nullptr;      // [nr]
  float *Pt_f = nullptr, *Ptc_f = nullptr;  // FP32 copies of Pt, Ptc (mixed: FP32 PDEP GEMMs)
  float* tau_f = nullptr;     // [nr/Rf][nblk][64 Rf] FP32 cache (always whole)
  float2 *agrid_f = nullptr, *drho_f = nullptr, *compact_f = nullptr;
  int nbc_f = 0;
  long compact_f_grids = 0;
  // Wannier-localised frame (localize = 1): K1d, its tau blocks and U's W
  // term work in it.  phik / phik_f are the orbital grids of those terms:
  // phir_loc (phir_loc_f) when localised, else phir (phir_f).
  int loc = 0;
  double prune_thr = 0.0;
  double* Uloc = nullptr;         // [nv][nv] U[v][j]
  double* Phi_loc = nullptr;      // [nv][npw] U^T Phi
  double2* phir_loc = nullptr;    // [nvh][nr]
  float2* phir_loc_f = nullptr;   // [nvh][nr] (mixed)
  double* A_rot = nullptr;        // [nbc][nv][npw] rotated block, then the rotated-back result
  const double2* phik = nullptr;
  const float2* phik_f = nullptr;
  double loc_spread = -1.0;
  int loc_sweeps = 0;
  long nblk_all = 0;
  std::vector<double> loc_U_h, loc_cen_h;  // [nv][nv], [nv][3]
  // learned preconditioner (not owned)
  bse_mlp* learned = nullptr;
  // HIP graphs of the block apply, one per (block size, precision), replayed
  // on the staging buffers gX -> gY; graph_bufs are the context buffers the
  // graphs reference: releasing any of them destroys every graph first
  bool use_graph = false;
  // the vectors handed to the block apply already lie in the P_c space (the
  // solvers' own subspace vectors): the input projection is skipped
  bool in_pc = false;
  hipStream_t cap_st = nullptr;  // private stream the graphs are captured on
  double *gX = nullptr, *gY = nullptr;
  std::vector<std::pair<int, hipGraphExec_t>> graphs;
  std::vector<void*> graph_bufs;
  // profiling
  bool prof = false;
  double ph_ms[bsex::PH_COUNT] = {0};
  long ph_n[bsex::PH_COUNT] = {0};
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev_open;
  size_t ev_used = 0;
};

namespace bsex {
int ctx_alloc(bse_ctx* c, void** p, size_t bytes);
template <typename T>
int ctx_alloc_t(bse_ctx* c, T** p, size_t count) {
  return ctx_alloc(c, reinterpret_cast<void**>(p), sizeof(T) * count);
}
void ctx_release(bse_ctx* c, void* p);
// return the cached released blocks to the device (before sizing caches)
void ctx_pool_flush(bse_ctx* c);

// profiling
struct PhaseScope {
  bse_ctx* c;
  int ph;
  hipEvent_t e1 = nullptr;
  PhaseScope(bse_ctx* c_, int ph_);
  ~PhaseScope();
};
int prof_collect(bse_ctx* c);

// operator pieces (device, stream ordered)
int proj_c(bse_ctx* c, const double* X, double* Y, int nset);
int gemm(bse_ctx* c, int ta, int tb, long M, long N, long K, double alpha, const double* A,
         long lda, const double* B, long ldb, double beta, double* C, long ldc);
int apply_chunk(bse_ctx* c, int nb, const double* X, double* Y);
int apply_H(bse_ctx* c, int nvs, int nset, const double* X, double* Y, double2* grids,
            double shift, const double* eps, int project);
int to_grid(bse_ctx* c, const double* X, int nvs, int nset, double2* grids);
// forward transform of packed grids and projection onto the sphere rows Y,
// plus (T + shift - eps_v) A when A is given
int from_grid(bse_ctx* c, double2* grids, int nvs, int nset, const double* A, const double* eps,
              double shift, double* Y);
int kernel_part(bse_ctx* c, const double2* agrid, double* Kt);
int sigma_phi(bse_ctx* c, const double2* agrid, double2* y);
int orth_block(bse_ctx* c, const double* V, long m, double* W, long k, long len, double* tmp,
               int passes, double drop);
int ensure_apply_work(bse_ctx* c, int nbc);
int ensure_ygrid(bse_ctx* c);
// tau of blocks [gb0, gb0 + nblk) stored into dst (FP64, R points per row,
// a buffer of dst_nblk blocks from dst_blk0) and/or dstf (the whole FP32
// cache, Rf points per row, at block gb0); either may be null
int tau_build_range_f(bse_ctx* c, const float2* orbr, long gb0, long nblk, float* dst,
                      long dst_nblk, long dst_blk0, int mask);
int tau_build_range(bse_ctx* c, const double2* orbr, long gb0, long nblk, double* dst,
                    long dst_nblk, long dst_blk0, int mask, float* dstf = nullptr);
// learned preconditioner network (mlp.hip): y [n][n_out] from x [n][n_in]
int mlp_eval(bse_mlp* q, long n, const float* x, float* y, hipStream_t st);
int mlp_n_in(const bse_mlp* q);
int mlp_n_out(const bse_mlp* q);
int learned_targets(bse_ctx* c, const double* Xs, const double* Zref, bool two_level, float* feat,
                    double* gamma);
int apply_chunk_mixed(bse_ctx* c, int nb, const double* X, double* Y);
// block apply through a captured HIP graph (captured on first use per block size)
int graph_apply(bse_ctx* c, int nb, const double* X, double* Y);
void graphs_destroy(bse_ctx* c);
int apply_any(bse_ctx* c, int nb, const double* X, double* Y);
int apply_H_f(bse_ctx* c, int nvs, int nset, const double* X, double* Y, double shift,
              const double* eps, int project);
int ensure_mixed_work(bse_ctx* c, int nbc);
int ground_state(bse_ctx* c, int n_want, double tol, bool warm = false);
// self-consistent KS model: SCF ground state, or the potential of given orbitals
int ks_ground_state(bse_ctx* c, int n_want);
int ks_potential_from_orbitals(bse_ctx* c);
// out_v += scale sum_w L_w (v_c * (M_w x_v)), v < nx (packed grids)
int exchange_like(bse_ctx* c, const double2* L, const double2* M, const double2* x, int nx,
                  double2* out, double scale);
int gram_tall(bse_ctx* c, const double* A, long m, const double* B, long n, long len, double* C);
// device address of the allocation-free scratch on `dev` (called once per
// context initialisation, with that device current)
int noalloc_setup(int dev);
// Wannier frame and kept blocks of a context built with localize = 1
int localize(bse_ctx* c, const bse_system_desc* d);
int rotate_bands(bse_ctx* c, int nb, const double* A, double* out, bool back);
// beyond the TDA: Y = P_c (s K2e - K2d) P_c X (FP64), and the lowest roots of
// the coupled problem
int apply_coupling(bse_ctx* c, int nb, const double* X, double* Y);
int full_bse(bse_ctx* c, int ns, const bse_solver_opts* o, double* omega, double* Xout,
             double* Yout, bse_solver_stats* stats);
int diag_axpy(const double* A, const double* Tk, const double* eps, double shift, int nv,
              long npw, int nb, double* Y, hipStream_t st);
long noalloc_scratch_doubles();
}  // namespace bsex
