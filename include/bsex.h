/*
 * bsex.h -- C ABI of the MI355X (gfx950) library for plane-wave analytical
 * excited-state forces from the Bethe-Salpeter equation (Tamm-Dancoff
 * approximation, density-matrix perturbation theory, no empty states).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Return value: 0 (BSE_OK) or a positive bse_status code.  Nothing throws or
 * aborts across the ABI; bse_last_error() returns a thread-local message for
 * the last non-zero return of the calling thread.
 *
 * Basis: the real orthonormal plane-wave basis of the Gamma-point sphere
 * S = {G : |G|^2/2 <= ecut} of an orthorhombic cell (lengths L, volume
 * Omega): e_0 = Omega^-1/2, then for every G of the half sphere (first
 * non-zero Miller index positive) c_G = sqrt(2/Omega) cos(G.r) followed by
 * s_G = sqrt(2/Omega) sin(G.r).  The half sphere is ordered by
 * (|n|^2, n1, n2, n3).  The FFT grid N1 x N2 x N3 must hold the sphere
 * strictly (every |n_i| < N_i/2).  Inner products are plain dot products of
 * coefficient vectors.  n_pw = 1 + 2 * (half-sphere size).
 *
 * Layout: row-major, plane-wave index fastest.  An orbital block is
 * [n_val][n_pw]; a block of trial vectors is [n_b][n_val][n_pw].  All double.
 *
 * Pointers: arguments named *_dev are device pointers (hipMalloc or a torch
 * CUDA tensor on the context's device); *_host are host pointers.  The
 * caller owns every buffer it passes; the library copies host inputs during
 * bse_init_system and never frees caller memory.  A context owns its device
 * allocations until bse_free.
 *
 * Streams: every call is ordered on desc.stream and returns after its work
 * on that stream has finished.  A context is not thread-safe.
 *
 * Units: Hartree and bohr.
 */
#ifndef BSEX_H
#define BSEX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BSEX_ABI_VERSION 4

typedef enum {
  BSE_OK = 0,
  BSE_EINVAL = 1,   /* bad argument, descriptor, shape or non-finite input     */
  BSE_ENOMEM = 2,   /* device allocation failed or tau cache over its budget  */
  BSE_EHIP = 3,     /* a HIP runtime call failed                             */
  BSE_ENOCONV = 4,  /* iteration limit reached; outputs hold the last iterate */
  BSE_EGAP = 5,     /* Kohn-Sham gap eps_{n_val+1} - eps_{n_val} below gap_min */
  BSE_EABI = 6,     /* desc.abi_version differs from BSEX_ABI_VERSION          */
  BSE_ESTATE = 7    /* call not valid in the context's current state          */
} bse_status;

/* which terms of M = D + s K1e - K1d the operator applies (test hook) */
enum {
  BSE_K_D = 1,         /* D: P_c (H - eps_v + scissor)                        */
  BSE_K_1E = 2,        /* K1e: bare-Coulomb exchange-like term (Eq. 2b)         */
  BSE_K_1D_BARE = 4,   /* K1d, bare v_c part of W                             */
  BSE_K_1D_PDEP = 8,   /* K1d, low-rank PDEP part of W (Eq. 3)                 */
  BSE_K_ALL = 15
};

/* Precision of the operator apply (SM Sec. IV discusses single precision for
 * the kernel terms).  BSE_FP64: every step in FP64.  BSE_MIXED: the grids,
 * FFTs, pair potentials tau (cached in FP32) and the kernel terms K1e, K1d in
 * FP32 with FP32 accumulation of the tau contraction; the projector P_c,
 * the diagonal term D, the Davidson Rayleigh-Ritz and every reduction of the
 * solvers stay in FP64.  A BSE_MIXED context also holds the FP64 operator
 * (tau rebuilt on the fly); bse_davidson confirms its result with it and
 * bse_zvector_solve uses it for the outer residual of iterative refinement. */
enum { BSE_FP64 = 0, BSE_MIXED = 1 };
enum { BSE_TAU_AUTO = 0, BSE_TAU_CACHE = 1, BSE_TAU_REBUILD = 2 };

typedef struct bse_ctx bse_ctx;

/*
 * System description.  Defines the synthetic Kohn-Sham Hamiltonian
 * H = |G|^2/2 + V(r), V a sum of Gaussian wells
 *   V_I(r) = -depth_I exp(-|r - R_I|^2 / (2 width_I^2)),
 * periodised in G space on every grid frequency with the Nyquist planes set
 * to zero, and the screened interaction of Eq. 3,
 *   W = v_c + v_c^1/2 [sum_a phi_a lambda_a/(1-lambda_a) phi_a^T] v_c^1/2,
 * v_c(G) = 4 pi/|G|^2 on every grid frequency (minimum image), v_c(0) = 0.
 */
typedef struct {
  int32_t abi_version;        /* BSEX_ABI_VERSION                                 */
  double cell[3];             /* orthorhombic cell lengths (bohr), > 0            */
  int32_t grid[3];            /* FFT grid; each a product of 2, 3 and 5, 4..512   */
  double ecut;                /* Ha                                               */
  int32_t n_sites;            /* >= 0                                             */
  const double *site_xyz;     /* host [n_sites][3] bohr                          */
  const double *site_depth;   /* host [n_sites] Ha                               */
  const double *site_width;   /* host [n_sites] bohr, > 0                         */
  int32_t n_val;              /* occupied orbitals N_v, 1 <= n_val < n_pw          */
  int32_t n_pdep;             /* PDEP rank, 0 <= n_pdep < n_pw                     */
  const double *pdep;         /* host [n_pw][n_pdep], orthonormal columns, row 0 zero */
  const double *lambda;       /* host [n_pdep], each < 1                           */
  double scissor;             /* Delta (Ha); shifts omega only                    */
  double spin_factor;         /* s in D + s K1e - K1d; 2 for a singlet            */
  int32_t precision;          /* BSE_FP64 or BSE_MIXED                            */
  int32_t tau_policy;         /* BSE_TAU_*: cache W(phi_v phi_v') or rebuild it   */
  int64_t tau_budget_bytes;   /* cap on tau cache bytes (FP32 and FP64 caches together);
                                 0 = auto, keeping 4 GB + 330 trial vectors (at most
                                 12% of the device) for solver work (28 GB at
                                 N_v 432, N_pw 21,079); > 0 also drops
                                 that reserve to 1 GB (apply-only use).  BSE_MIXED needs
                                 the whole FP32 cache (ENOMEM otherwise) and gives the
                                 FP64 cache what is left. */
  double gap_min;             /* Ha; EGAP below it (<= 0 disables the check)      */
  int32_t kernel_mask;        /* BSE_K_*; 0 means BSE_K_ALL                        */
  int32_t n_orb;              /* orbitals supplied (>= n_val), or 0 to solve H    */
  const double *orbitals;     /* host [n_orb][n_pw] orthonormal eigenvectors      */
  const double *eps;          /* host [n_orb] eigenvalues, ascending              */
  int32_t n_extra;            /* extra (conduction) states the solver computes    */
  double gs_tol;              /* eigen-residual target of the solver for the n_val
                                 occupied states (0: 1e-10); the n_extra states
                                 above them stop at max(gs_tol, 1e-6)           */
  void *stream;               /* hipStream_t, NULL for the null stream            */
  /* Ground-state model.  0 = the fixed local potential above (default).
   * 1 = self-consistent Kohn-Sham Hamiltonian (the paper's DFT starting
   * point, reduced to a synthetic functional; SM Sec. I):
   *   H_KS = |G|^2/2 + V(r) + V_H[rho] + V_xc[rho],  rho = 2 sum_v phi_v^2,
   *   V_H = v_c * rho,  V_xc = -(3/pi)^(1/3) [(rho + rho_floor)^(1/3) - rho_floor^(1/3)].
   * The ground state is then solved to self-consistency (or, with orbitals
   * supplied, H_KS is built from their density); D uses H_KS, U gains its D
   * part 2 P_c [f_Hxc * Drho_x] phi_v and the Z-vector operator the kernels
   * 2 K^1e,KS + 2 K^2e,KS = 4 P_c [f_Hxc * sum_v' phi_v' Z_v'] phi_v of Eq. 7,
   * f_Hxc * g = v_c * g + (dV_xc/drho) g.
   * alpha_exx > 0 (a hybrid starting point) adds -alpha K_x to H_KS,
   * (K_x psi)(r) = sum_w phi_w(r) [v_c * (phi_w psi)](r), and with it the
   * exact-exchange terms of U's D part and the kernels -K^1d,KS - K^2d,KS of
   * Eq. 7; each costs one Poisson solve per occupied pair and vector, so it
   * is meant for small systems, and it needs the orbitals supplied
   * (n_orb > 0, eigenvectors of that H_KS) and BSE_FP64. */
  int32_t ks_model;
  double rho_floor;           /* density floor of V_xc (0: 1e-3)                  */
  double scf_tol;             /* RMS change of V_H + V_xc ending the SCF (0: 1e-10) */
  double alpha_exx;           /* exact-exchange fraction, 0 <= alpha_exx <= 1      */
  /* Wannier-localised pair pruning (the paper's Wannier-localised W
   * integrals, main text, computational-cost paragraph after Eq. 7).
   * localize = 1 rotates the occupied orbitals into maximally localised
   * Wannier functions w_j = sum_v U[v][j] phi_v: simultaneous
   * diagonalisation of the six matrices <phi|cos, sin(2 pi x_k/L_k)|phi>
   * (Gygi, Fattebert and Schwegler 2003) by Jacobi rounds of a round-robin
   * tournament, the w_j then put in Morton order of their centres.  The
   * pair measure s_jj' = ||w_j w_j'|| / (||w_j^2|| ||w_j'^2||)^(1/2) (L2
   * norms, in [0, 1]) decides which 8x8 blocks of occupied pairs keep their
   * W integrals: block (I, J) is kept when its largest s_jj' is
   * >= prune_threshold (diagonal blocks always are).  In
   * bse_apply the K1d term becomes
   *   (K1d A)_v = P_c sum_j U[v][j] sum_{j' kept with j} W(w_j' w_j) a~_j',
   *   a~_j = sum_v U[v][j] a_v,
   * and the W term of U (bse_u_vector) is restricted to the same pairs in
   * the same frame; D, K1e, the Z-vector and the force contraction are
   * unchanged, and every input and output stays in the canonical frame.
   * With prune_threshold 0 every block is kept and the results equal the
   * canonical ones.  Needs ks_model 0 (EINVAL otherwise). */
  int32_t localize;           /* 0: canonical (default), 1: localised and pruned  */
  double prune_threshold;     /* in [0, 1]                                        */
  const double *loc_rotation; /* host [n_val][n_val] U[v][j], orthogonal to 1e-8, in the
                                 order wanted; NULL: the library localises      */
  int32_t loc_max_sweeps;     /* Jacobi sweep cap (0: 100)                        */
  double loc_tol;             /* sweeps stop when one lowers the spread by less than
                                 loc_tol x spread (0: 1e-9)                     */
} bse_system_desc;

/* Library ABI version (BSEX_ABI_VERSION of the build). */
int32_t bse_abi_version(void);

/* Thread-local message of the last failing call ("" when none). */
const char *bse_last_error(void);

/* Optional: start the HIP runtime on the current device and load the
 * library's device code there (one tiny kernel launch, 256 bytes allocated
 * and freed), so that this one-time cost stays out of later timed calls.
 * EHIP on a runtime error. */
int bse_warm_up(void);

/* Host-only basis queries (no device needed).  n_pw of the sphere; EINVAL if
 * the sphere does not fit the grid. */
int bse_basis_size(const double cell[3], const int32_t grid[3], double ecut,
                   int32_t *n_pw);

/* Miller indices [n_pw][3] and kind [n_pw] (0 = G0, 1 = cos, 2 = sin) of the
 * basis functions in library order.  Either output may be NULL. */
int bse_basis_gvectors(const double cell[3], const int32_t grid[3], double ecut,
                       int32_t *miller_host, int8_t *kind_host);

/* Build a context: copy inputs to the device, take or compute the occupied
 * orbitals (lowest eigenpairs of H), check the Kohn-Sham gap, cache phi(r)
 * and build (or plan) the pair potentials tau_{v'v} = W(phi_v' phi_v) of
 * Eq. 2c.  On failure *out is NULL and nothing leaks. */
int bse_init_system(const bse_system_desc *desc, bse_ctx **out);

typedef struct {
  int32_t n_pw, n_val, n_pdep, n_orb;
  int32_t grid[3];
  int32_t tau_policy;         /* policy in effect                                */
  int64_t tau_blocks;         /* 8x8 pair blocks of the upper triangle            */
  int64_t tau_blocks_cached;  /* blocks held in the FP64 cache                   */
  int64_t tau_bytes;          /* bytes of the FP64 cache                         */
  double gs_resid;            /* max eigen-residual of the solved occupied orbitals (-1 if supplied) */
  double ks_gap;              /* eps_{n_val+1} - eps_{n_val} when known, else -1  */
  int32_t precision;          /* precision the context was built with            */
  int32_t active_precision;   /* precision bse_apply uses now                    */
  int64_t tau_bytes_f32;      /* bytes of the FP32 tau cache (BSE_MIXED), else 0 */
  int32_t gs_sweeps;          /* filter sweeps of the ground-state solve (0: orbitals supplied) */
  double t_ground_state_ms;   /* wall time of bse_init_system: ground-state solve */
  double t_tau_ms;            /*   sizing, allocation and build of the tau caches */
  double t_tau_alloc_ms;      /*     of which the allocation of the caches      */
  double t_init_ms;           /*   the whole call                                 */
  int32_t scf_iters;          /* self-consistent cycles of the KS model (0 if none) */
  double scf_resid;           /* their final RMS potential change (-1 if none)    */
  int64_t tau_blocks_all;     /* 8x8 pair blocks before pruning                   */
  double loc_spread;          /* spread (bohr^2) of the localised frame (-1: canonical) */
  int32_t loc_sweeps;         /* Jacobi sweeps run (0 with loc_rotation or canonical) */
} bse_info;

int bse_get_info(bse_ctx *ctx, bse_info *info);

/* Copy the occupied orbitals [n_val][n_pw] (device) and eigenvalues [n_val]
 * (host).  Either pointer may be NULL.  With orbitals solved by the library,
 * extra conduction states are returned when n > n_val: orbitals_dev must
 * then hold [n][n_pw] and eps_host [n], n <= n_orb. */
int bse_get_orbitals(bse_ctx *ctx, int32_t n, double *orbitals_dev, double *eps_host);

/* The localised frame of a context built with localize = 1: U_host
 * [n_val][n_val] (U[v][j], row-major; columns in the library's order) and
 * centres_host [n_val][3] (bohr, in [0, L_k)).  Either may be NULL.
 * ESTATE for a canonical context. */
int bse_get_frame(bse_ctx *ctx, double *U_host, double *centres_host);

/* The operator of Eqs. 1-2 (scissor form of Table S-I):
 *   Y = P_c (D + s K1e - K1d) P_c X   for n_b trial vectors
 *   (D A)_v   = P_c (H - eps_v + scissor) a_v
 *   (K1e A)_v = P_c (v_c * Drho) phi_v,     Drho = sum_v phi_v a_v
 *   (K1d A)_v = P_c sum_v' tau_{v'v} a_v'
 * X_dev, Y_dev: device [n_b][n_val][n_pw], must not overlap.  n_b >= 0
 * (0 is a no-op).  The input is projected first, so the operator is
 * symmetric on the whole space and maps occupied directions to zero. */
int bse_apply(bse_ctx *ctx, int32_t n_b, const double *X_dev, double *Y_dev);

typedef struct {
  double tol;                 /* residual target; 0 -> 1e-8                        */
  int32_t max_iter;           /* 0 -> 300 (Davidson) / 5000 (CG)                   */
  int32_t block;              /* Davidson block; 0 -> n_states + 4                 */
  int32_t max_subspace;       /* 0 -> 16 * block, or less if device memory is short */
  const double *x0_dev;       /* optional initial guess, [k][n_val][n_pw]         */
  int32_t n_x0;               /* vectors in x0_dev                                 */
  const double *z0_dev;       /* optional Z-vector initial guess [n_val][n_pw]    */
  int32_t use_learned;        /* 1: take the per-band preconditioner shifts and the
                                 Z initial guess from the network attached with
                                 bse_set_learned (ignored when none is attached)  */
  const double *precond_shift_host; /* optional [n_val] per-band shift sigma_v of the
                                 kinetic preconditioner (default 0.25 Ha); overrides
                                 the network's shifts                              */
  int32_t *band_iters_host;   /* optional out [n_val] (Z-vector): iteration at which
                                 band v's own relative residual first reached tol;
                                 when given, the solve runs until every band has  */
  int32_t two_level;          /* 1: correct the kinetic preconditioner on the span
                                 of the conduction states the context holds (n_orb
                                 > n_val): there it is 1/(eps_c - eps_v + Delta -
                                 theta) (Davidson; |.| >= 1e-3 Ha) or
                                 1/(eps_c - eps_v) (Z-vector), applied as
                                 Q K^-1 Q + Psi D^-1 Psi^T, Q = 1 - Psi Psi^T      */
} bse_solver_opts;

typedef struct {
  int32_t iters;              /* iterations performed                             */
  int32_t applies;            /* operator applications (vectors)                  */
  double resid[16];           /* final residual norms (first 16 states)           */
  double t_ms;                /* wall time of the call                            */
  int32_t applies_fp64;       /* of `applies`, those made with the FP64 operator  */
  int32_t learned;            /* 1 when the network's outputs were used           */
  int32_t fallback;           /* 1 when the solve dropped them for the diagonal
                                 preconditioner (residual grew twice in a row, or
                                 a non-finite output)                             */
  double t_u_ms;              /* Z-vector: wall time of its right-hand side U (SM
                                 Sec. I), included in t_ms; 0 otherwise           */
} bse_solver_stats;

/* Lowest n_states eigenpairs of P_c M P_c (Eq. 1) by block Davidson with a
 * shifted kinetic preconditioner.  Residual ||M x - omega x||_2 with
 * ||x||_2 = 1 must reach opts->tol for every requested state.
 * omega_host [n_states]; X_dev [n_states][n_val][n_pw]; stats may be NULL.
 * ENOCONV after max_iter with the last Ritz pairs in the outputs. */
int bse_davidson(bse_ctx *ctx, int32_t n_states, const bse_solver_opts *opts,
                 double *omega_host, double *X_dev, bse_solver_stats *stats);

/* Beyond the Tamm-Dancoff approximation (SM Sec. I, the coupled form with
 * the A_s and B_s blocks; the paper itself works in the TDA).  For real
 * Gamma-point orbitals the coupling operators are
 *   (K2e A)_v = P_c [v_c * sum_v' a_v' phi_v'] phi_v,
 *   (K2d A)_v = P_c sum_v' [W (a_v' phi_v)] phi_v',
 * and bse_apply_coupling returns Y = P_c (s K2e - K2d) P_c X (FP64, the
 * canonical frame, every kernel term switched by kernel_mask like bse_apply;
 * about N_v^2 Poisson and PDEP solves per vector).  X_dev, Y_dev: device
 * [n_b][n_val][n_pw], not overlapping.  EINVAL with ks_model 1. */
int bse_apply_coupling(bse_ctx *ctx, int32_t n_b, const double *X_dev, double *Y_dev);

/* Lowest n_states roots of [[A, B], [B, A]] (X; Y) = omega (X; -Y),
 * A = P_c M P_c (Eq. 1), B the coupling above, by the subspace method of
 * Stratmann, Scuseria and Frisch on (A - B)(A + B) in FP64 (the paper gives
 * no solver for this form).  Converged when ||r+||^2 + ||r-||^2 <= tol^2 with
 * r+ = (A + B)(X + Y) - omega (X - Y), r- = (A - B)(X - Y) - omega (X + Y)
 * and X.X - Y.Y = 1.  omega_host [n_states]; X_dev, Y_dev
 * [n_states][n_val][n_pw] (either may be NULL); stats may be NULL (applies
 * counts each vector once; each costs one A and one B apply).  EINVAL when
 * A - B or A + B is not positive definite on the subspace (an unstable
 * ground state); ENOCONV after max_iter with the last roots in the outputs. */
int bse_full_bse(bse_ctx *ctx, int32_t n_states, const bse_solver_opts *opts,
                 double *omega_host, double *X_dev, double *Y_dev, bse_solver_stats *stats);

/* U vector of SM Sec. I for one normalised exciton A (Xs_dev [n_val][n_pw]):
 *   u_v = P_c[ s (v_c*Drho) a_v - sum_v' W(a_v' a_v) phi_v' ] - sum_v' S_vv' a_v'
 *   S_vv' = <phi_v | [(s K1e - K1d) A]_v'>   (kernel part before P_c).
 * U_dev [n_val][n_pw]. */
int bse_u_vector(bse_ctx *ctx, const double *Xs_dev, double *U_dev);

/* Z-vector equation (Eq. 7) for the synthetic Hamiltonian, whose KS response
 * kernels vanish:  P_c (H - eps_v) P_c Z_v = -u_v  for every band, by block
 * PCG with per-band steps, until ||D Z + U||_F / ||U||_F <= opts->tol.
 * Computes U from Xs_dev first.  Z_dev [n_val][n_pw]. */
int bse_zvector_solve(bse_ctx *ctx, const double *Xs_dev, const bse_solver_opts *opts,
                      double *Z_dev, bse_solver_stats *stats);

/* d omega / d R of Eq. 4 with the densities of Eqs. 5-6:
 *   dw/dR_{I,a} = Omega sum_G Re[ conj(-i G_a V_I(G)) rho_t(G) ],
 *   rho_t = sum_v a_v^2 - sum_vv' phi_v phi_v' <a_v'|a_v> + 2 sum_v Z_v phi_v.
 * dwdR_host [n_sites][3].  The excitation-energy force is -dwdR. */
int bse_forces(bse_ctx *ctx, const double *Xs_dev, const double *Z_dev, double *dwdR_host);

/* bse_forces for callers that cannot allocate memory (code under HIP graph
 * capture, tight serving loops): the same d omega / d R, written to device
 * memory, with no allocation of any kind.  Xs_dev, Z_dev [N_v][N_pw] and
 * dwdR_dev [n_sites][3] are device buffers owned by the caller (dwdR_dev may
 * be NULL when n_sites = 0).  Stream ordered on the context's stream: the
 * call returns once the work is queued, without synchronising.
 * The work buffers are the context's apply buffers (present after
 * bse_init_system) and one static device scratch array of 64 MiB per device,
 * whose address is resolved when a context is initialised on that device
 * and which stays allocated until the process ends.  Calls on one device
 * share that array: calls that overlap on one device race, so serialise
 * them (one stream, or events).  EINVAL when the system needs more scratch
 * (2 N_v^2 doubles plus the per-site partial sums) than the array holds;
 * ESTATE when the context has no apply buffers for 3 vector sets. */
int bse_forces_noalloc(bse_ctx *ctx, const double *Xs_dev, const double *Z_dev,
                       double *dwdR_dev);

/* The ground-state part of the excited-state force: the paper writes the
 * excited-state force as the ground-state force minus d omega / d R (the
 * sentence introducing Eq. 4).  For the synthetic Hamiltonian H = T + V,
 * whose ground-state energy is the occupied eigenvalue sum, that part is the
 * Hellmann-Feynman derivative
 *   dE/dR_{I,a} = sum_v <phi_v| dV/dR_{I,a} |phi_v>
 *              = Omega sum_G Re[ conj(-i G_a V_I(G)) rho(G) ],  rho = sum_v phi_v^2,
 * per unit occupation (multiply by the spin factor for a spin-degenerate
 * ground state).  Uses the context's occupied orbitals; no other input.
 * dEdR_host [n_sites][3] (may be NULL when n_sites = 0).  The excited-state
 * force on the surface E + omega is -(dEdR + dwdR). */
int bse_ground_state_forces(bse_ctx *ctx, double *dEdR_host);

/* Per-phase device time of the calls since the last reset, measured with HIP
 * events on the context's stream while enabled (off by default). */
typedef struct {
  int32_t n_phase;
  const char *name[16];
  double ms[16];
  int64_t count[16];
} bse_phase_times;

/* Select the precision of bse_apply on a context built with BSE_MIXED
 * (BSE_FP64 or BSE_MIXED).  ESTATE on an FP64 context asked for BSE_MIXED. */
int bse_set_precision(bse_ctx *ctx, int32_t precision);

/* Route the block applies of bse_apply and bse_davidson through HIP graphs
 * (on = 1): the first call for each block size (and precision) runs eagerly,
 * then captures the apply on fixed staging buffers; later calls copy the block
 * in, replay the graph and copy the result out.  Results are those of the
 * eager path up to the order of the LDS atomic sums in the tau stream.  Graphs are dropped when a buffer they use is released, when
 * turned off, and by bse_free.  Ignored while profiling is on. */
int bse_set_graphs(bse_ctx *ctx, int32_t on);

int bse_set_profiling(bse_ctx *ctx, int32_t on);
int bse_get_phase_times(bse_ctx *ctx, bse_phase_times *out, int32_t reset);

/*
 * Learned preconditioner (no counterpart in the paper; this project's form).
 * A network maps 8 per-band features to (o_0, o_1):
 *   sigma_v = 0.25 Ha * exp(clamp(o_0, -3, 3))   shift of the kinetic
 *             preconditioner 1/max(|G|^2/2 - eps_v + sigma_v, 0.1) of the
 *             Z-vector PCG and (with the scissor and the Ritz value) of Davidson;
 *   gamma_v = exp(clamp(o_1, -6, 8))             Z initial guess
 *             Z_v^0 = gamma_v P_c Prec_v(-u_v) with the default shift 0.25 Ha
 *             (Prec in its two-level form when the solve uses it).
 * Features of band v (BSE_LEARN_NFEAT = 8):
 *   0 eps_v - eps_{N_v}          1 eps_{N_v+1} - eps_v   (Ha; eps ascending, 1-based)
 *   2 <phi_v|T|phi_v>            3 <phi_v|V|phi_v> = eps_v - feature 2
 *   4 log(Omega int phi_v^4)     5 log ||u_v||           6 <Prec u_v, u_v>/||u_v||^2
 *   7 1 when features 5 and 6 are present (Z-vector), 0 for Davidson (5, 6 = 0).
 * Every solve that uses it is still judged by the plain operator's residual.
 */
#define BSE_LEARN_NFEAT 8
#define BSE_LEARN_NOUT 2

typedef struct bse_mlp bse_mlp;

/* Three dense layers n_in -> 128 -> 128 -> n_out with SiLU between them, BF16
 * operands on the matrix cores with FP32 accumulation, FP32 master weights,
 * Adam (0.9, 0.999, 1e-8).  Inputs are standardised and outputs de-standardised
 * inside with the statistics of bse_mlp_set_norm (default 0 and 1).  Weights
 * W ~ U(+-1/sqrt(fan_in)) from a splitmix64 stream of `seed`, biases 0.
 * n_in 1..64, n_out 1..16.  Calls are ordered on `stream` and synchronous. */
int bse_mlp_create(int32_t n_in, int32_t n_out, uint64_t seed, void *stream, bse_mlp **out);
/* Flat FP32 parameter vector: W1 [128][n_in], b1 [128], W2 [128][128], b2 [128],
 * W3 [n_out][128], b3 [n_out] (row-major).  set resets the Adam state. */
int bse_mlp_n_params(const bse_mlp *mlp, int64_t *n);
int bse_mlp_set_params(bse_mlp *mlp, const float *params_host);
int bse_mlp_get_params(bse_mlp *mlp, float *params_host);
int bse_mlp_set_norm(bse_mlp *mlp, const float *mu_x, const float *s_x, const float *mu_y,
                     const float *s_y);
/* y_dev [n][n_out] from x_dev [n][n_in] (FP32, device). */
int bse_mlp_forward(bse_mlp *mlp, int32_t n, const float *x_dev, float *y_dev);
/* One Adam step on L = sum w (yh - (t - mu_y)/s_y)^2 / max(sum w, 1), yh the
 * normalised output.  t_dev [n][n_out]; w_dev [n][n_out] or NULL (all 1);
 * loss_host (before the step) and grad_dev (flat dL/dparams, FP32) optional. */
int bse_mlp_train_step(bse_mlp *mlp, int32_t n, const float *x_dev, const float *t_dev,
                       const float *w_dev, float lr, float *loss_host, float *grad_dev);
int bse_mlp_free(bse_mlp *mlp);

/* Attach a network (n_in = BSE_LEARN_NFEAT, n_out = BSE_LEARN_NOUT) to a
 * context; NULL detaches.  The context does not own it: keep it alive while
 * attached. */
int bse_set_learned(bse_ctx *ctx, bse_mlp *mlp);

/* Features [n_val][BSE_LEARN_NFEAT] of the Z-vector solve for exciton Xs_dev
 * (feature 7 = 1), and, when Zref_dev (a converged Z) is given, the
 * least-squares initial-guess coefficient per band,
 *   gamma_v* = <p_v, Z_v> / <p_v, p_v>,  p_v = P_c Prec_v(-u_v), shift 0.25 Ha,
 * Prec the kinetic diagonal, or its two-level form when two_level = 1 (the
 * Z-vector solve builds its learned initial guess with the preconditioner it
 * runs with).  Needs the first conduction eigenvalue (n_orb > n_val):
 * ESTATE otherwise. */
int bse_learned_features(bse_ctx *ctx, const double *Xs_dev, const double *Zref_dev,
                         int32_t two_level, float *feat_host, double *gamma_host);

/*
 * Uneven batches of independent systems (each solved as by bse_init_system,
 * bse_davidson for the lowest exciton, bse_zvector_solve and bse_forces).
 * Up to n_streams systems run at once, each on its own HIP stream (default
 * priority) and host thread, largest first, a system being admitted while its
 * device-memory estimate fits mem_budget (a system that fits nothing runs
 * alone).  Each system's tau cache is capped at its own size.  With autotune,
 * the Davidson block apply of each shape class (grid, N_v in buckets of 64,
 * precision) that occurs more than once in the batch is timed under each
 * kernel variant (compile-time or runtime FFT kernels; 4 or 2 lanes per grid
 * point in the tau stream; one warm-up, two timed applies each) and the
 * fastest is cached for the process; a class met once keeps the defaults.
 * desc.stream and desc.precision are ignored (the batch's are used).
 */
typedef struct {
  double tol;                 /* Davidson and Z-vector residual target (0: 1e-6)   */
  int32_t precision;          /* BSE_FP64 or BSE_MIXED                             */
  int32_t n_streams;          /* systems in flight, 1..8 (0: 4)                    */
  int64_t mem_budget;         /* device bytes the batch may hold (0: 85% of free)  */
  int32_t autotune;           /* 1: tune kernel variants per shape                 */
  int32_t use_graph;          /* 1: Davidson applies replay captured HIP graphs    */
} bse_batch_opts;

typedef struct {
  int32_t status;             /* BSE_* of this system                              */
  double omega;               /* lowest excitation energy (Ha)                     */
  double *dwdR_host;          /* caller's [n_sites][3] output, or NULL             */
  int32_t davidson_iters, z_iters;
  double t_init_ms, t_davidson_ms, t_z_ms, t_force_ms;
  int32_t variant;            /* autotuned variant (bit 0: runtime FFT kernels,
                                 bit 1: 2 lanes per point), -1 when not tuned     */
  int32_t stream_slot;        /* stream (worker) that ran it                       */
  char message[160];          /* error text when status != BSE_OK                  */
} bse_batch_result;

/* Returns BSE_OK when every system succeeded, else the first failing status
 * (every result holds its own status and message). */
int bse_batch_run(const bse_system_desc *descs, int32_t n, const bse_batch_opts *opts,
                  bse_batch_result *results);
/* Forget the autotuner's cached choices. */
int bse_tune_cache_clear(void);

int bse_free(bse_ctx *ctx);

/* Device memory across contexts (this library's own; for callers that build
 * one context per geometry, such as a relaxation).  on = 1: bse_free hands
 * a context's device blocks, once its stream has drained, to a process-wide
 * cache, and later contexts on the same device take their blocks from it
 * (best fit, at most twice the size asked) before allocating; an allocation
 * that fails returns the device's cached blocks and tries again.  on = 0:
 * frees every cached block and stops caching.  The cached memory stays
 * held (unavailable to other allocators) until then.  Default off. */
int bse_memory_cache(int32_t on);

#ifdef __cplusplus
}
#endif
#endif /* BSEX_H */
