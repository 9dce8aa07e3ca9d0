// Solvers driving the operator: block Davidson for the excitons (Eq. 1),
// the U vector (SM Sec. I), the Z-vector CG (Eq. 7 with the KS kernels of
// the local synthetic Hamiltonian zero), the force contraction (Eqs. 4-6)
// and a Chebyshev-filtered subspace eigensolver for the ground state.
//
// All long vectors stay on the device; only small projected matrices and
// per-band scalars cross to the host.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <numeric>
#include <random>
#include <vector>

#include "context.h"

namespace bsex {

constexpr double kPrecondShift = 0.25;  // Ha, kinetic preconditioner shift
// The FP32-kernel Davidson stops at half the requested residual, but not below
// kMixedFloor: the FP32 apply differs from the FP64 one by ~1e-8 of |Y|, a few
// 1e-7 in the residual of a normalised vector, so the FP64 check then passes
// without FP64 iterations unless tol is below that floor.
constexpr double kMixedFloor = 3e-7;
// smallest |eps_c - eps_v + Delta - theta| the two-level Davidson
// preconditioner divides by on the conduction states it holds
constexpr double kDavidsonMinDen = 1e-3;
// relative residual of each inner FP32 PCG solve of the Z-vector refinement
constexpr double kMixedInnerTol = 1e-4;
// eigen-residual the ground state asks of the states above the occupied ones
// (they serve the preconditioners and the gap check only), unless gs_tol is
// looser
constexpr double kExtraStateTol = 1e-6;

int learned_features(bse_ctx* c, const double* U, std::vector<float>& F);
int learned_eval(bse_ctx* c, const std::vector<float>& F, std::vector<double>& sigma,
                 std::vector<double>& gamma, bool* ok);

int gram_tall(bse_ctx* c, const double* A, long m, const double* B, long n, long len, double* C) {
  const long need = dgemm_tall_work(m, n, len);
  if (need > c->gw_len) {
    ctx_release(c, c->gw);
    c->gw = nullptr;
    c->gw_len = 0;
    BSE_TRY(ctx_alloc_t(c, &c->gw, (size_t)need));
    c->gw_len = need;
  }
  return dgemm_tall(m, n, len, 1.0, A, len, B, len, 0.0, C, n, c->gw, c->gw_len, c->st);
}

namespace {

struct DVec {  // scoped device scratch owned by the context
  bse_ctx* c;
  double* p = nullptr;
  explicit DVec(bse_ctx* c_) : c(c_) {}
  int alloc(size_t n) { return ctx_alloc_t(c, &p, n); }
  ~DVec() { ctx_release(c, p); }
  DVec(const DVec&) = delete;
  DVec& operator=(const DVec&) = delete;
};

// host copies go through the context's pinned staging buffer; the vector
// forms check that the host buffer holds the n elements copied
int to_host(bse_ctx* c, const double* d, double* h, size_t n) {
  return stage_d2h(&c->hstage, d, h, sizeof(double) * n, c->st);
}

int to_dev(bse_ctx* c, const double* h, double* d, size_t n) {
  return stage_h2d(&c->hstage, h, d, sizeof(double) * n, c->st);
}

int to_host(bse_ctx* c, const double* d, std::vector<double>& h, size_t n) {
  if (n > h.size()) return fail(BSE_EINVAL, "copy of %zu values into a host buffer of %zu", n, h.size());
  return to_host(c, d, h.data(), n);
}

int to_dev(bse_ctx* c, const std::vector<double>& h, double* d, size_t n) {
  if (n > h.size()) return fail(BSE_EINVAL, "copy of %zu values from a host buffer of %zu", n, h.size());
  return to_dev(c, h.data(), d, n);
}

int copy_dev(bse_ctx* c, const double* s, double* d, size_t n) {
  if (n == 0 || s == d) return BSE_OK;
  BSE_HIP(hipMemcpyAsync(d, s, sizeof(double) * n, hipMemcpyDeviceToDevice, c->st));
  return BSE_OK;
}

int dots_host(bse_ctx* c, const double* A, const double* B, long rows, long len, double* scratch,
              std::vector<double>& out) {
  const long need = row_dots_work(rows, len);
  if (need > c->rdw_len) {
    ctx_release(c, c->rdw);
    c->rdw = nullptr;
    c->rdw_len = 0;
    BSE_TRY(ctx_alloc_t(c, &c->rdw, (size_t)need));
    c->rdw_len = need;
  }
  BSE_TRY(row_dots(A, B, rows, len, scratch, c->rdw, c->rdw_len, c->st));
  out.resize(rows);
  return to_host(c, scratch, out, rows);
}

double elapsed_ms(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

// apply the operator to n vectors in chunks of at most c->nbc; in_pc: the
// vectors already lie in the P_c space
int apply_n(bse_ctx* c, long n, const double* X, double* Y, bool in_pc = false) {
  const long L = (long)c->nv * c->basis.npw;
  struct Flag {
    bse_ctx* c;
    bool keep;
    ~Flag() { c->in_pc = keep; }
  } flag{c, c->in_pc};
  c->in_pc = in_pc;
  for (long i = 0; i < n; i += c->nbc) {
    const int k = (int)std::min<long>(c->nbc, n - i);
    if (c->use_graph && !c->prof)
      BSE_TRY(graph_apply(c, k, X + i * L, Y + i * L));
    else
      BSE_TRY(apply_any(c, k, X + i * L, Y + i * L));
  }
  return BSE_OK;
}

// Two-level preconditioner on the rows W[k][v][:] (in place):
//   W <- Q K^-1 Q W + Psi diag(1/(eps_c - eps_v + shift - theta_k)) Psi^T W,
// Psi the conduction states the context holds, Q = 1 - Psi Psi^T, K^-1 the
// kinetic diagonal (kin: the caller's kernel applied in place).  Symmetric
// positive definite when K^-1 is and the denominators are positive (Z-vector);
// in Davidson it is the transition-space diagonal of M on span(Psi).
template <typename Kin>
int precond_two_level(bse_ctx* c, double* W, int nk, const double* theta, double shift,
                      double dmin, Kin kin) {
  const int nv = c->nv, npw = c->basis.npw, nc = c->norb - c->nv;
  if (nc <= 0) return kin(W);
  const long M = (long)nk * nv;
  const double* Psi = c->Phi + (long)nv * npw;
  double *C1 = nullptr, *C2 = nullptr;
  BSE_TRY(ctx_alloc_t(c, &C1, (size_t)M * nc));
  int rc = ctx_alloc_t(c, &C2, (size_t)M * nc);
  auto run = [&]() -> int {
    BSE_TRY(gemm(c, 0, 1, M, nc, npw, 1.0, W, npw, Psi, npw, 0.0, C1, nc));    // Psi^T R
    BSE_TRY(dgemm(0, 0, M, npw, nc, -1.0, C1, nc, Psi, npw, 1.0, W, npw, c->st));  // Q R
    BSE_TRY(kin(W));                                                            // K^-1 Q R
    BSE_TRY(gemm(c, 0, 1, M, nc, npw, 1.0, W, npw, Psi, npw, 0.0, C2, nc));
    BSE_TRY(dgemm(0, 0, M, npw, nc, -1.0, C2, nc, Psi, npw, 1.0, W, npw, c->st));  // Q K^-1 Q R
    BSE_TRY(coarse_scale(C1, nk, nv, nc, c->eps_d, theta, shift, dmin, c->st));
    return dgemm(0, 0, M, npw, nc, 1.0, C1, nc, Psi, npw, 1.0, W, npw, c->st);
  };
  if (rc == BSE_OK) rc = run();
  ctx_release(c, C1);
  ctx_release(c, C2);
  return rc;
}

}  // namespace

// Orthonormalise the rows of W[k][len] against V[m][len] and among
// themselves.  Rows are normalised first; up to two rounds of (project out
// V, then orthonormalise through the eigen-decomposition of the Gram
// matrix) follow.  Directions with Gram eigenvalue below drop^2 are dropped
// in the first round.  The second round is skipped when the first lost at
// most half of the squared norm in every direction (smallest Gram
// eigenvalue >= 1/2): one classical Gram-Schmidt pass is then accurate to
// rounding (the criterion of Daniel, Gragg, Kaufman and Stewart, Math.
// Comp. 30, 772 (1976)).  Surviving rows are compacted to the front of W;
// returns their number, or a negative status.
int orth_block(bse_ctx* c, const double* V, long m, double* W, long k, long len, double* tmp,
               int passes, double drop) {
  if (k <= 0) return 0;
  PhaseScope ps(c, PH_SOLVER);
  DVec sm(c);
  const size_t smn = (size_t)k * (size_t)std::max(m, k) + (size_t)k * k + 2 * (size_t)k + 16;
  if (sm.alloc(smn) != BSE_OK) return -BSE_ENOMEM;
  double* Cm = sm.p;                                     // [k][m]
  double* Bm = sm.p + (size_t)k * std::max(m, k);        // [k][k]
  double* vec = Bm + (size_t)k * k;                      // [2k]
  std::vector<double> nrm;
  if (dots_host(c, W, W, k, len, vec, nrm) != BSE_OK) return -BSE_EHIP;
  std::vector<double> sc(k);
  for (long i = 0; i < k; ++i) sc[i] = nrm[i] > 0 ? 1.0 / std::sqrt(nrm[i]) : 0.0;
  if (to_dev(c, sc, vec, k) != BSE_OK) return -BSE_EHIP;
  if (row_scale(vec, W, k, len, c->st) != BSE_OK) return -BSE_EHIP;
  long kk = k;
  for (int pass = 0; pass < passes; ++pass) {
    if (m > 0) {
      if (gram_tall(c, W, kk, V, m, len, Cm) != BSE_OK) return -BSE_EHIP;
      if (dgemm(0, 0, kk, len, m, -1.0, Cm, m, V, len, 1.0, W, len, c->st) != BSE_OK)
        return -BSE_EHIP;
    }
    if (gram_tall(c, W, kk, W, kk, len, Bm) != BSE_OK) return -BSE_EHIP;
    std::vector<double> G((size_t)kk * kk), lam(kk);
    if (to_host(c, Bm, G, (size_t)kk * kk) != BSE_OK) return -BSE_EHIP;
    if (host_syev((int)kk, G.data(), lam.data())) return -fail(BSE_EINVAL, "Gram eigensolver failed");
    const bool enough = pass == 0 && lam[0] >= 0.5;
    const double thr = (pass == 0) ? drop * drop : 1e-300;
    std::vector<double> Bh;
    long knew = 0;
    for (long j = kk - 1; j >= 0; --j) {  // largest first
      if (!(lam[j] > thr)) continue;
      const double s = 1.0 / std::sqrt(lam[j]);
      for (long i = 0; i < kk; ++i) Bh.push_back(s * G[(size_t)i * kk + j]);
      ++knew;
    }
    if (knew == 0) return 0;
    if (to_dev(c, Bh, Bm, Bh.size()) != BSE_OK) return -BSE_EHIP;
    if (dgemm(0, 0, knew, len, kk, 1.0, Bm, kk, W, len, 0.0, tmp, len, c->st) != BSE_OK)
      return -BSE_EHIP;
    if (copy_dev(c, tmp, W, (size_t)knew * len) != BSE_OK) return -BSE_EHIP;
    kk = knew;
    if (enough) break;
  }
  return (int)kk;
}

// Orthonormalise the k rows of W[k][len] in place by Cholesky QR, done twice:
// rows normalised, then W <- L^{-1} W with W W^T = L L^T.  Returns k; returns
// 0, with W still spanning the same space, when the normalised Gram matrix is
// too ill-conditioned for it (smallest Cholesky pivot below 1e-6 of the
// largest, the loss of orthogonality of one pass then being ~1e-4 or worse),
// so that the caller can fall back to orth_block; negative on error.
static int chol_orth(bse_ctx* c, double* W, long k, long len, double* tmp) {
  if (k <= 0) return 0;
  PhaseScope ps(c, PH_SOLVER);
  DVec sm(c);
  if (sm.alloc((size_t)k * k + 2 * (size_t)k + 16) != BSE_OK) return -BSE_ENOMEM;
  double* Gd = sm.p;
  double* vec = sm.p + (size_t)k * k;
  std::vector<double> nrm;
  if (dots_host(c, W, W, k, len, vec, nrm) != BSE_OK) return -BSE_EHIP;
  std::vector<double> sc(k);
  for (long i = 0; i < k; ++i) {
    if (!(nrm[i] > 0.0)) return 0;
    sc[i] = 1.0 / std::sqrt(nrm[i]);
  }
  if (to_dev(c, sc, vec, k) != BSE_OK) return -BSE_EHIP;
  if (row_scale(vec, W, k, len, c->st) != BSE_OK) return -BSE_EHIP;
  std::vector<double> G((size_t)k * k);
  for (int pass = 0; pass < 2; ++pass) {
    if (gram_tall(c, W, k, W, k, len, Gd) != BSE_OK) return -BSE_EHIP;
    if (to_host(c, Gd, G, G.size()) != BSE_OK) return -BSE_EHIP;
    if (host_cholesky((int)k, G.data())) return 0;
    double lmin = G[0], lmax = G[0];
    for (long i = 0; i < k; ++i) {
      lmin = std::min(lmin, G[(size_t)i * k + i]);
      lmax = std::max(lmax, G[(size_t)i * k + i]);
    }
    if (lmin < 1e-6 * lmax) return 0;
    if (host_trinv_lower((int)k, G.data())) return 0;
    if (to_dev(c, G, Gd, G.size()) != BSE_OK) return -BSE_EHIP;
    if (dgemm(0, 0, k, len, k, 1.0, Gd, k, W, len, 0.0, tmp, len, c->st) != BSE_OK)
      return -BSE_EHIP;
    if (copy_dev(c, tmp, W, (size_t)k * len) != BSE_OK) return -BSE_EHIP;
  }
  return (int)k;
}

// ---------------------------------------------------------------------------
// Davidson (the paper names no eigensolver; its target is the lowest
// eigenpairs of P_c M P_c)
// ---------------------------------------------------------------------------
static int davidson_core(bse_ctx* c, int ns, const bse_solver_opts* o, double* omega,
                         double* Xout, bse_solver_stats* stats) {
  const auto t0 = std::chrono::steady_clock::now();
  const double tol = (o && o->tol > 0) ? o->tol : 1e-8;
  const int maxit = (o && o->max_iter > 0) ? o->max_iter : 300;
  int nb = (o && o->block > 0) ? o->block : ns + 4;
  if (nb < ns) nb = ns;
  // default subspace: 16 blocks (at the defect-supercell size it needs about
  // 60% of the iterations of an 8-block one), smaller if memory runs short
  const bool fixed_sub = o && o->max_subspace > 0;
  int maxsub = fixed_sub ? o->max_subspace : 16 * nb;
  if (maxsub < 3 * nb) maxsub = 3 * nb;
  const long npw = c->basis.npw, nv = c->nv, L = nv * npw;
  BSE_TRY(ensure_apply_work(c, std::min(nb, 8)));
  DVec V(c), AV(c), W(c), AW(c), X(c), AX(c), sm(c);
  BSE_TRY(W.alloc((size_t)2 * nb * L));
  BSE_TRY(AW.alloc((size_t)2 * nb * L));
  BSE_TRY(X.alloc((size_t)nb * L));
  BSE_TRY(AX.alloc((size_t)nb * L));
  for (;;) {
    int rc = V.alloc((size_t)maxsub * L);
    if (rc == BSE_OK) rc = AV.alloc((size_t)maxsub * L);
    if (rc == BSE_OK) break;
    ctx_release(c, V.p);
    ctx_release(c, AV.p);
    V.p = AV.p = nullptr;
    if (fixed_sub || maxsub <= 3 * nb) return rc;
    maxsub = std::max(3 * nb, maxsub * 3 / 4);
    set_error("%s", "");
  }
  BSE_TRY(sm.alloc((size_t)maxsub * maxsub + 4 * (size_t)maxsub + 64));
  double* Cd = sm.p;                              // [m][k] coefficients
  double* vecd = sm.p + (size_t)maxsub * maxsub;  // small vectors
  int applies = 0;
  // preconditioner shifts: the default, the caller's per-band values, or the
  // network's (dropped for the default if the residual grows twice in a row)
  DVec vs(c);
  BSE_TRY(vs.alloc((size_t)nv));
  const double* vshift = nullptr;
  double pshift = c->scissor + kPrecondShift;
  bool learned = false, fallback = false;
  if (o && o->precond_shift_host) {
    BSE_TRY(to_dev(c, o->precond_shift_host, vs.p, nv));
    vshift = vs.p;
    pshift = c->scissor;
  } else if (o && o->use_learned && c->learned) {
    std::vector<float> F;
    std::vector<double> sig, gam;
    bool ok = false;
    BSE_TRY(learned_features(c, nullptr, F));
    BSE_TRY(learned_eval(c, F, sig, gam, &ok));
    if (ok) {
      BSE_TRY(to_dev(c, sig, vs.p, nv));
      vshift = vs.p;
      pshift = c->scissor;
      learned = true;
    } else {
      fallback = true;
    }
  }
  double prev_res = 1e300;
  int grew = 0;
  const bool two_level = o && o->two_level && c->norb > c->nv;

  // ---- initial block: user vectors, then lowest bare transitions ----------
  BSE_HIP(hipMemsetAsync(W.p, 0, sizeof(double) * (size_t)nb * L, c->st));
  int k = 0;
  if (o && o->x0_dev && o->n_x0 > 0) {
    k = std::min(o->n_x0, nb);
    BSE_TRY(copy_dev(c, o->x0_dev, W.p, (size_t)k * L));
  }
  const int nc = c->norb - c->nv;
  if (k < nb && nc > 0) {
    std::vector<std::pair<double, long>> tr;
    for (long v = 0; v < nv; ++v)
      for (long cc = 0; cc < nc; ++cc) tr.push_back({c->eps_h[nv + cc] - c->eps_h[v], v * nc + cc});
    std::stable_sort(tr.begin(), tr.end(),
                     [](const auto& a, const auto& b) { return a.first < b.first; });
    for (size_t q = 0; q < tr.size() && k < nb; ++q, ++k) {
      const long v = tr[q].second / nc, cc = tr[q].second % nc;
      BSE_TRY(copy_dev(c, c->Phi + (nv + cc) * npw, W.p + (size_t)k * L + v * npw, npw));
    }
  }
  if (k < nb) {  // plane waves of lowest kinetic model, kept if they survive P_c
    std::vector<std::pair<double, long>> d;
    for (long v = 0; v < nv; ++v)
      for (long j = 0; j < npw; ++j)
        d.push_back({0.5 * c->basis.g2[j] - c->eps_h[v] + c->scissor + kPrecondShift, v * npw + j});
    std::stable_sort(d.begin(), d.end(), [](const auto& a, const auto& b) { return a.first < b.first; });
    size_t q = 0;
    std::vector<double> one(1, 1.0), nrm;
    while (k < nb && q < d.size()) {
      double* w = W.p + (size_t)k * L;
      BSE_HIP(hipMemsetAsync(w, 0, sizeof(double) * L, c->st));
      BSE_TRY(to_dev(c, one, w + d[q].second, 1));
      ++q;
      BSE_TRY(proj_c(c, w, w, 1));
      BSE_TRY(dots_host(c, w, w, 1, L, vecd, nrm));
      if (std::sqrt(nrm[0]) > 0.3) ++k;
    }
  }
  BSE_TRY(proj_c(c, W.p, W.p, k));
  int m = orth_block(c, V.p, 0, W.p, k, L, AW.p, 2, 1e-8);
  if (m <= 0) return m < 0 ? -m : fail(BSE_EINVAL, "Davidson: empty initial block");
  BSE_TRY(copy_dev(c, W.p, V.p, (size_t)m * L));
  BSE_TRY(apply_n(c, m, V.p, AV.p, true));
  applies += m;
  std::vector<double> Hs((size_t)maxsub * maxsub, 0.0);
  auto refresh_rows = [&](long r0, long r1) -> int {  // Hs rows/cols r0..r1-1 against 0..r1-1
    const long nr_ = r1 - r0;
    BSE_TRY(gram_tall(c, V.p + (size_t)r0 * L, nr_, AV.p, r1, L, Cd));
    std::vector<double> blk((size_t)nr_ * r1);
    BSE_TRY(to_host(c, Cd, blk, blk.size()));
    for (long i = 0; i < nr_; ++i)
      for (long j = 0; j < r1; ++j) {
        Hs[(size_t)(r0 + i) * maxsub + j] = blk[(size_t)i * r1 + j];
        if (j < r0) Hs[(size_t)j * maxsub + r0 + i] = blk[(size_t)i * r1 + j];
      }
    return BSE_OK;
  };
  BSE_TRY(refresh_rows(0, m));

  std::vector<double> theta, rn(nb, 0.0);
  int it = 0;
  bool conv = false;
  for (it = 0; it < maxit; ++it) {
    std::vector<double> A((size_t)m * m), w(m);
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j)
        A[(size_t)i * m + j] = 0.5 * (Hs[(size_t)i * maxsub + j] + Hs[(size_t)j * maxsub + i]);
    if (host_syev(m, A.data(), w.data())) return fail(BSE_EINVAL, "Davidson: small eigensolver failed");
    const int kr = std::min(nb, m);
    std::vector<double> Ck((size_t)m * kr);
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < kr; ++j) Ck[(size_t)i * kr + j] = A[(size_t)i * m + j];
    BSE_TRY(to_dev(c, Ck, Cd, Ck.size()));
    {
      PhaseScope ps(c, PH_SOLVER);
      BSE_TRY(dgemm(1, 0, kr, L, m, 1.0, Cd, kr, V.p, L, 0.0, X.p, L, c->st));
      BSE_TRY(dgemm(1, 0, kr, L, m, 1.0, Cd, kr, AV.p, L, 0.0, AX.p, L, c->st));
    }
    std::vector<double> negth(kr);
    for (int i = 0; i < kr; ++i) negth[i] = -w[i];
    BSE_TRY(to_dev(c, negth, vecd, kr));
    BSE_TRY(copy_dev(c, AX.p, W.p, (size_t)kr * L));           // R = AX - theta X
    BSE_TRY(row_axpby(vecd, X.p, nullptr, W.p, kr, L, c->st));
    std::vector<double> r2;
    BSE_TRY(dots_host(c, W.p, W.p, kr, L, vecd + maxsub, r2));
    for (int i = 0; i < kr; ++i) rn[i] = std::sqrt(std::max(0.0, r2[i]));
    theta.assign(w.begin(), w.begin() + std::min(ns, m));
    bool all = (m >= ns);
    double rmax = 0.0;
    for (int i = 0; i < ns && i < kr; ++i) {
      all = all && (rn[i] <= tol);
      rmax = std::max(rmax, rn[i]);
    }
    if (all) {
      conv = true;
      break;
    }
    if (learned && vshift) {
      grew = rmax > prev_res ? grew + 1 : 0;
      if (grew >= 2 || !std::isfinite(rmax)) {
        vshift = nullptr;
        pshift = c->scissor + kPrecondShift;
        fallback = true;
      }
    }
    prev_res = rmax;
    // preconditioned residuals of the unconverged Ritz vectors
    std::vector<int> todo;
    for (int i = 0; i < kr; ++i)
      if (rn[i] > tol) todo.push_back(i);
    const int nt = (int)todo.size();
    for (int q = 0; q < nt; ++q)
      if (todo[q] != q) BSE_TRY(copy_dev(c, W.p + (size_t)todo[q] * L, W.p + (size_t)q * L, L));
    std::vector<double> th(nt);
    for (int q = 0; q < nt; ++q) th[q] = w[todo[q]];
    BSE_TRY(to_dev(c, th, vecd, nt));
    auto kin = [&](double* w) {
      return precond_davidson(w, w, c->T, c->eps_d, vecd, pshift, nt, (int)nv, (int)npw, c->st,
                              vshift);
    };
    if (two_level)
      BSE_TRY(precond_two_level(c, W.p, nt, vecd, c->scissor, kDavidsonMinDen, kin));
    else
      BSE_TRY(kin(W.p));
    BSE_TRY(proj_c(c, W.p, W.p, nt));
    if (m + nt > maxsub) {  // thick restart on the lowest 2 nb Ritz vectors
      const int keep = std::min(2 * nb, m);
      std::vector<double> Ckeep((size_t)m * keep);
      for (int i = 0; i < m; ++i)
        for (int j = 0; j < keep; ++j) Ckeep[(size_t)i * keep + j] = A[(size_t)i * m + j];
      BSE_TRY(to_dev(c, Ckeep, Cd, Ckeep.size()));
      PhaseScope ps(c, PH_SOLVER);
      // AW holds 2 nb rows: use it as the staging buffer
      BSE_TRY(dgemm(1, 0, keep, L, m, 1.0, Cd, keep, V.p, L, 0.0, AW.p, L, c->st));
      BSE_TRY(copy_dev(c, AW.p, V.p, (size_t)keep * L));
      BSE_TRY(dgemm(1, 0, keep, L, m, 1.0, Cd, keep, AV.p, L, 0.0, AW.p, L, c->st));
      BSE_TRY(copy_dev(c, AW.p, AV.p, (size_t)keep * L));
      m = keep;
      std::fill(Hs.begin(), Hs.end(), 0.0);
      BSE_TRY(refresh_rows(0, m));
    }
    const int kn = orth_block(c, V.p, m, W.p, nt, L, AW.p, 2, 1e-8);
    if (kn < 0) return -kn;
    if (kn == 0) break;
    BSE_TRY(apply_n(c, kn, W.p, AW.p, true));
    applies += kn;
    BSE_TRY(copy_dev(c, W.p, V.p + (size_t)m * L, (size_t)kn * L));
    BSE_TRY(copy_dev(c, AW.p, AV.p + (size_t)m * L, (size_t)kn * L));
    BSE_TRY(refresh_rows(m, m + kn));
    m += kn;
  }
  for (int i = 0; i < ns; ++i) omega[i] = i < (int)theta.size() ? theta[i] : NAN;
  if (Xout) BSE_TRY(copy_dev(c, X.p, Xout, (size_t)ns * L));
  BSE_HIP(hipStreamSynchronize(c->st));
  if (stats) {
    stats->iters = it;
    stats->applies = applies;
    stats->applies_fp64 = c->active == BSE_MIXED ? 0 : applies;
    stats->learned = learned ? 1 : 0;
    stats->fallback = fallback ? 1 : 0;
    for (int i = 0; i < 16; ++i) stats->resid[i] = i < nb ? rn[i] : 0.0;
    stats->t_ms = elapsed_ms(t0);
    stats->t_u_ms = 0.0;
  }
  if (!conv) return fail(BSE_ENOCONV, "Davidson: no convergence in %d iterations", it);
  return BSE_OK;
}

// ---------------------------------------------------------------------------
// Beyond the TDA (SM Sec. I): lowest roots of
//   [[A, B], [B, A]] (X; Y) = omega (X; -Y),  A = D + s K1e - K1d,
//   B = s K2e - K2d,
// i.e. of (A - B)(A + B) on X + Y, by the subspace method of Stratmann,
// Scuseria and Frisch (J. Chem. Phys. 109, 8218 (1998)); the paper gives
// no solver for this form.  With an orthonormal basis b of the P_c space,
// P = b^T (A + B) b and Q = b^T (A - B) b, Q = L L^T: L^T P L u = omega^2 u,
// X + Y = b L u, X - Y = b P L u / omega, scaled to X.X - Y.Y = 1.  The
// residuals r+ = (A + B)(X + Y) - omega (X - Y) and
// r- = (A - B)(X - Y) - omega (X + Y) of each unconverged root, through the
// kinetic preconditioner at theta = omega, extend the basis; the basis
// restarts from the current X + Y and X - Y when full.  FP64 throughout.
// ---------------------------------------------------------------------------
int full_bse(bse_ctx* c, int ns, const bse_solver_opts* o, double* omega, double* Xout,
             double* Yout, bse_solver_stats* stats) {
  const auto t0 = std::chrono::steady_clock::now();
  const double tol = (o && o->tol > 0) ? o->tol : 1e-8;
  const int maxit = (o && o->max_iter > 0) ? o->max_iter : 300;
  int nb = (o && o->block > 0) ? o->block : ns + 4;
  if (nb < ns) nb = ns;
  int maxsub = (o && o->max_subspace > 0) ? o->max_subspace : 12 * nb;
  if (maxsub < 4 * nb) maxsub = 4 * nb;
  const long npw = c->basis.npw, nv = c->nv, L = nv * npw;
  const int keep_active = c->active;
  c->active = BSE_FP64;
  struct Back {
    bse_ctx* c;
    int a;
    ~Back() { c->active = a; }
  } back{c, keep_active};
  BSE_TRY(ensure_apply_work(c, std::min(2 * nb, 8)));
  DVec V(c), ApB(c), AmB(c), W(c), AW(c), BW(c), Xp(c), Xm(c), sm(c);
  BSE_TRY(V.alloc((size_t)maxsub * L));
  BSE_TRY(ApB.alloc((size_t)maxsub * L));
  BSE_TRY(AmB.alloc((size_t)maxsub * L));
  BSE_TRY(W.alloc((size_t)2 * nb * L));
  BSE_TRY(AW.alloc((size_t)2 * nb * L));
  BSE_TRY(BW.alloc((size_t)2 * nb * L));
  BSE_TRY(Xp.alloc((size_t)nb * L));
  BSE_TRY(Xm.alloc((size_t)nb * L));
  BSE_TRY(sm.alloc(2 * (size_t)maxsub * maxsub + 8 * (size_t)maxsub + 64));
  double* Cd = sm.p;                                   // coefficient matrices
  double* vecd = sm.p + 2 * (size_t)maxsub * maxsub;  // small vectors
  int applies = 0;
  // initial block: the lowest bare transitions (conduction states held),
  // then plane waves of lowest kinetic model
  BSE_HIP(hipMemsetAsync(W.p, 0, sizeof(double) * (size_t)nb * L, c->st));
  int k = 0;
  const int nc = c->norb - c->nv;
  if (nc > 0) {
    std::vector<std::pair<double, long>> tr;
    for (long v = 0; v < nv; ++v)
      for (long cc = 0; cc < nc; ++cc) tr.push_back({c->eps_h[nv + cc] - c->eps_h[v], v * nc + cc});
    std::stable_sort(tr.begin(), tr.end(),
                     [](const auto& a, const auto& b) { return a.first < b.first; });
    for (size_t q = 0; q < tr.size() && k < nb; ++q, ++k) {
      const long v = tr[q].second / nc, cc = tr[q].second % nc;
      BSE_TRY(copy_dev(c, c->Phi + (nv + cc) * npw, W.p + (size_t)k * L + v * npw, npw));
    }
  }
  if (k < nb) {
    std::vector<std::pair<double, long>> d;
    for (long v = 0; v < nv; ++v)
      for (long j = 0; j < npw; ++j)
        d.push_back({0.5 * c->basis.g2[j] - c->eps_h[v], v * npw + j});
    std::stable_sort(d.begin(), d.end(), [](const auto& a, const auto& b) { return a.first < b.first; });
    size_t q = 0;
    std::vector<double> one(1, 1.0), nrm;
    while (k < nb && q < d.size()) {
      double* w = W.p + (size_t)k * L;
      BSE_HIP(hipMemsetAsync(w, 0, sizeof(double) * L, c->st));
      BSE_TRY(to_dev(c, one, w + d[q].second, 1));
      ++q;
      BSE_TRY(proj_c(c, w, w, 1));
      BSE_TRY(dots_host(c, w, w, 1, L, vecd, nrm));
      if (std::sqrt(nrm[0]) > 0.3) ++k;
    }
  }
  BSE_TRY(proj_c(c, W.p, W.p, k));
  int m = 0;
  // orthonormalise kn new rows of W against the basis, apply A and B, append
  auto extend = [&](int kn) -> int {
    const int kk = orth_block(c, V.p, m, W.p, kn, L, AW.p, 2, 1e-8);
    if (kk < 0) return -kk;
    if (kk == 0) return BSE_OK;
    BSE_TRY(apply_n(c, kk, W.p, AW.p, true));
    BSE_TRY(apply_coupling(c, kk, W.p, BW.p));
    applies += kk;
    BSE_TRY(copy_dev(c, W.p, V.p + (size_t)m * L, (size_t)kk * L));
    BSE_TRY(copy_dev(c, AW.p, ApB.p + (size_t)m * L, (size_t)kk * L));
    BSE_TRY(axpby(1.0, BW.p, 1.0, ApB.p + (size_t)m * L, (long)kk * L, c->st));
    BSE_TRY(copy_dev(c, AW.p, AmB.p + (size_t)m * L, (size_t)kk * L));
    BSE_TRY(axpby(-1.0, BW.p, 1.0, AmB.p + (size_t)m * L, (long)kk * L, c->st));
    m += kk;
    return BSE_OK;
  };
  BSE_TRY(extend(k));
  if (m == 0) return fail(BSE_EINVAL, "full BSE: empty initial block");
  std::vector<double> om(ns, NAN), rn(nb, 0.0);
  int it = 0;
  bool conv = false;
  for (it = 0; it < maxit; ++it) {
    std::vector<double> Ph((size_t)m * m), Qh((size_t)m * m);
    BSE_TRY(gram_tall(c, V.p, m, ApB.p, m, L, Cd));
    BSE_TRY(to_host(c, Cd, Ph, Ph.size()));
    BSE_TRY(gram_tall(c, V.p, m, AmB.p, m, L, Cd));
    BSE_TRY(to_host(c, Cd, Qh, Qh.size()));
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < i; ++j) {
        const double a = 0.5 * (Ph[(size_t)i * m + j] + Ph[(size_t)j * m + i]);
        const double b = 0.5 * (Qh[(size_t)i * m + j] + Qh[(size_t)j * m + i]);
        Ph[(size_t)i * m + j] = Ph[(size_t)j * m + i] = a;
        Qh[(size_t)i * m + j] = Qh[(size_t)j * m + i] = b;
      }
    // Q = L L^T (lower, row-major), then K = L^T P L
    std::vector<double> Lq = Qh;
    if (host_cholesky(m, Lq.data()))
      return fail(BSE_EINVAL, "full BSE: A - B is not positive definite on the subspace");
    for (int i = 0; i < m; ++i)
      for (int j = i + 1; j < m; ++j) Lq[(size_t)i * m + j] = 0.0;
    std::vector<double> PL((size_t)m * m, 0.0), K((size_t)m * m, 0.0), lam(m);
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j) {
        double t = 0.0;
        for (int q = j; q < m; ++q) t += Ph[(size_t)i * m + q] * Lq[(size_t)q * m + j];
        PL[(size_t)i * m + j] = t;
      }
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j) {
        double t = 0.0;
        for (int q = i; q < m; ++q) t += Lq[(size_t)q * m + i] * PL[(size_t)q * m + j];
        K[(size_t)i * m + j] = t;
      }
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < i; ++j)
        K[(size_t)i * m + j] = K[(size_t)j * m + i] = 0.5 * (K[(size_t)i * m + j] + K[(size_t)j * m + i]);
    if (host_syev(m, K.data(), lam.data())) return fail(BSE_EINVAL, "full BSE: small eigensolver failed");
    const int kr = std::min(nb, m);
    // c+ = L u, c- = P c+ / omega, scaled to c+ . c- = 1; layout [m][kr]
    std::vector<double> cp((size_t)m * kr), cm((size_t)m * kr), w(kr);
    for (int j = 0; j < kr; ++j) {
      if (!(lam[j] > 0)) return fail(BSE_EINVAL, "full BSE: A + B is not positive definite");
      w[j] = std::sqrt(lam[j]);
    }
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < kr; ++j) {
        double t = 0.0;
        for (int q = 0; q <= i; ++q) t += Lq[(size_t)i * m + q] * K[(size_t)q * m + j];
        cp[(size_t)i * kr + j] = t;
      }
    for (int j = 0; j < kr; ++j) {
      double dot = 0.0;
      for (int i = 0; i < m; ++i) {
        double t = 0.0;
        for (int q = 0; q < m; ++q) t += Ph[(size_t)i * m + q] * cp[(size_t)q * kr + j];
        cm[(size_t)i * kr + j] = t / w[j];
        dot += cp[(size_t)i * kr + j] * cm[(size_t)i * kr + j];
      }
      const double sc = 1.0 / std::sqrt(dot);
      for (int i = 0; i < m; ++i) {
        cp[(size_t)i * kr + j] *= sc;
        cm[(size_t)i * kr + j] *= sc;
      }
    }
    double* Cp = Cd;
    double* Cm = Cd + (size_t)m * kr;
    BSE_TRY(to_dev(c, cp, Cp, cp.size()));
    BSE_TRY(to_dev(c, cm, Cm, cm.size()));
    {
      PhaseScope ps(c, PH_SOLVER);
      BSE_TRY(dgemm(1, 0, kr, L, m, 1.0, Cp, kr, V.p, L, 0.0, Xp.p, L, c->st));    // X + Y
      BSE_TRY(dgemm(1, 0, kr, L, m, 1.0, Cm, kr, V.p, L, 0.0, Xm.p, L, c->st));    // X - Y
      // r+ into W[0..kr), r- into W[kr..2 kr)
      BSE_TRY(dgemm(1, 0, kr, L, m, 1.0, Cp, kr, ApB.p, L, 0.0, W.p, L, c->st));
      BSE_TRY(dgemm(1, 0, kr, L, m, 1.0, Cm, kr, AmB.p, L, 0.0, W.p + (size_t)kr * L, L, c->st));
    }
    std::vector<double> negw(2 * kr);
    for (int j = 0; j < kr; ++j) negw[j] = negw[kr + j] = -w[j];
    BSE_TRY(to_dev(c, negw, vecd, 2 * kr));
    BSE_TRY(row_axpby(vecd, Xm.p, nullptr, W.p, kr, L, c->st));
    BSE_TRY(row_axpby(vecd + kr, Xp.p, nullptr, W.p + (size_t)kr * L, kr, L, c->st));
    std::vector<double> r2;
    BSE_TRY(dots_host(c, W.p, W.p, 2 * kr, L, vecd + 2 * maxsub, r2));
    for (int j = 0; j < kr; ++j) rn[j] = std::sqrt(std::max(0.0, r2[j] + r2[kr + j]));
    for (int i = 0; i < ns && i < kr; ++i) om[i] = w[i];
    bool all = m >= ns;
    for (int i = 0; i < ns && i < kr; ++i) all = all && rn[i] <= tol;
    if (all) {
      conv = true;
      break;
    }
    // preconditioned residuals of the unconverged roots (both r+ and r-)
    std::vector<int> todo;
    for (int j = 0; j < kr; ++j)
      if (rn[j] > tol) {
        todo.push_back(j);
        todo.push_back(kr + j);
      }
    const int nt = (int)todo.size();
    for (int q = 0; q < nt; ++q)
      if (todo[q] != q) BSE_TRY(copy_dev(c, W.p + (size_t)todo[q] * L, W.p + (size_t)q * L, L));
    std::vector<double> th(nt);
    for (int q = 0; q < nt; ++q) th[q] = w[todo[q] % kr];
    BSE_TRY(to_dev(c, th, vecd, nt));
    BSE_TRY(precond_davidson(W.p, W.p, c->T, c->eps_d, vecd, c->scissor + kPrecondShift, nt,
                             (int)nv, (int)npw, c->st));
    BSE_TRY(proj_c(c, W.p, W.p, nt));
    if (m + nt > maxsub) {
      // restart from the current X + Y and X - Y of the kr lowest roots
      BSE_TRY(copy_dev(c, Xp.p, W.p, (size_t)kr * L));
      BSE_TRY(copy_dev(c, Xm.p, W.p + (size_t)kr * L, (size_t)kr * L));
      m = 0;
      BSE_TRY(extend(2 * kr));
      continue;
    }
    const int m0 = m;
    BSE_TRY(extend(nt));
    if (m == m0) break;
  }
  for (int i = 0; i < ns; ++i) omega[i] = om[i];
  // X = (X+Y + X-Y)/2, Y = (X+Y - X-Y)/2
  if (Xout) {
    BSE_TRY(copy_dev(c, Xp.p, Xout, (size_t)ns * L));
    BSE_TRY(axpby(0.5, Xm.p, 0.5, Xout, (long)ns * L, c->st));
  }
  if (Yout) {
    BSE_TRY(copy_dev(c, Xp.p, Yout, (size_t)ns * L));
    BSE_TRY(axpby(-0.5, Xm.p, 0.5, Yout, (long)ns * L, c->st));
  }
  BSE_HIP(hipStreamSynchronize(c->st));
  if (stats) {
    stats->iters = it;
    stats->applies = applies;
    stats->applies_fp64 = applies;
    for (int i = 0; i < 16; ++i) stats->resid[i] = i < nb ? rn[i] : 0.0;
    stats->t_ms = elapsed_ms(t0);
    stats->t_u_ms = 0.0;
  }
  if (!conv) return fail(BSE_ENOCONV, "full BSE: no convergence in %d iterations", it);
  return BSE_OK;
}

// Davidson on the operator of the context's precision.  In mixed precision
// the FP32-kernel operator drives the iteration; the Ritz vectors are then
// checked with the FP64 operator (tau rebuilt in FP64) and, if the FP64
// residual is above tol, the FP64 Davidson continues from them.
int davidson(bse_ctx* c, int ns, const bse_solver_opts* o, double* omega, double* Xout,
             bse_solver_stats* stats) {
  if (c->active != BSE_MIXED) return davidson_core(c, ns, o, omega, Xout, stats);
  const auto t0 = std::chrono::steady_clock::now();
  const double tol = (o && o->tol > 0) ? o->tol : 1e-8;
  const long L = (long)c->nv * c->basis.npw;
  DVec X(c), Y(c), sv(c);
  BSE_TRY(X.alloc((size_t)ns * L));
  BSE_TRY(Y.alloc((size_t)ns * L));
  BSE_TRY(sv.alloc(64));
  bse_solver_stats s1{}, s2{};
  bse_solver_opts o1{};
  if (o) o1 = *o;
  o1.tol = std::max(0.5 * tol, kMixedFloor);
  int rc = davidson_core(c, ns, &o1, omega, X.p, &s1);
  if (rc != BSE_OK && rc != BSE_ENOCONV) return rc;
  c->active = BSE_FP64;
  struct Back {
    bse_ctx* c;
    ~Back() { c->active = BSE_MIXED; }
  } back{c};
  BSE_TRY(apply_n(c, ns, X.p, Y.p));
  std::vector<double> th, r2, xx;
  BSE_TRY(dots_host(c, X.p, Y.p, ns, L, sv.p, th));
  BSE_TRY(dots_host(c, X.p, X.p, ns, L, sv.p, xx));
  std::vector<double> nt(ns);
  for (int i = 0; i < ns; ++i) {
    th[i] /= xx[i];
    nt[i] = -th[i];
  }
  BSE_TRY(to_dev(c, nt, sv.p + 32, ns));
  BSE_TRY(row_axpby(sv.p + 32, X.p, nullptr, Y.p, ns, L, c->st));
  BSE_TRY(dots_host(c, Y.p, Y.p, ns, L, sv.p, r2));
  double worst = 0;
  for (int i = 0; i < ns; ++i) worst = std::max(worst, std::sqrt(r2[i] / xx[i]));
  int applies = s1.applies + ns, applies64 = ns;
  int iters = s1.iters;
  if (worst <= tol) {
    for (int i = 0; i < ns; ++i) {
      omega[i] = th[i];
      s2.resid[i] = std::sqrt(r2[i] / xx[i]);
    }
    if (Xout) BSE_TRY(copy_dev(c, X.p, Xout, (size_t)ns * L));
  } else {
    bse_solver_opts o2{};
    if (o) o2 = *o;
    o2.x0_dev = X.p;
    o2.n_x0 = ns;
    rc = davidson_core(c, ns, &o2, omega, Xout ? Xout : X.p, &s2);
    applies += s2.applies;
    applies64 += s2.applies;
    iters += s2.iters;
    if (rc != BSE_OK) return rc;
  }
  BSE_HIP(hipStreamSynchronize(c->st));
  if (stats) {
    stats->iters = iters;
    stats->applies = applies;
    stats->applies_fp64 = applies64;
    stats->learned = s1.learned;
    stats->fallback = (s1.fallback || s2.fallback) ? 1 : 0;
    for (int i = 0; i < 16; ++i) stats->resid[i] = i < ns ? s2.resid[i] : 0.0;
    stats->t_ms = elapsed_ms(t0);
    stats->t_u_ms = 0.0;
  }
  return BSE_OK;
}

// ---------------------------------------------------------------------------
// Self-consistent Kohn-Sham model (Eq. 7, SM Sec. I): H_KS = T + V_ext +
// V_H[rho] + V_xc[rho], rho = 2 sum_v phi_v^2, V_xc Slater exchange with a
// density floor; f_Hxc * g = v_c * g + f_xc g.
// ---------------------------------------------------------------------------
// V_H + V_xc of the occupied orbitals on the grid phir (nvh complex grids)
// into vhxc [nr]; sets c->fxc and c->rho_ks.  One complex grid of scratch.
static int ks_fields(bse_ctx* c, const double2* phir, double* vhxc) {
  const long nr = c->basis.nr;
  DVec rg(c), vx(c);
  BSE_TRY(rg.alloc(2 * (size_t)nr));
  BSE_TRY(vx.alloc((size_t)nr));
  double2* rho = reinterpret_cast<double2*>(rg.p);
  BSE_TRY(occupied_density(phir, c->nv, nr, rho, c->st));  // (sum phi^2, 0)
  BSE_TRY(xc_fields(rho, nr, 2.0, c->rho_floor, vx.p, c->fxc, c->rho_ks, c->st));
  BSE_TRY(fft3d(c->fft, rho, 1, -1, c->st));
  BSE_TRY(mul_real_field(rho, 1, nr, c->vc, 2.0 / (double)nr, c->st));
  BSE_TRY(fft3d(c->fft, rho, 1, +1, c->st));
  BSE_TRY(real_part(rho, nr, vhxc, c->st));
  return axpby(1.0, vx.p, 1.0, vhxc, nr, c->st);
}

// H_KS from orbitals given by the caller: V_eff = V_ext + V_hxc(rho(phi))
int ks_potential_from_orbitals(bse_ctx* c) {
  const long nr = c->basis.nr;
  DVec vh(c);
  BSE_TRY(vh.alloc((size_t)nr));
  BSE_TRY(ks_fields(c, c->phir, vh.p));
  BSE_TRY(copy_dev(c, c->Vext, c->Vr, nr));
  return axpby(1.0, vh.p, 1.0, c->Vr, nr, c->st);
}

// Self-consistent ground state: Chebyshev-filtered eigenpairs of H_KS[V_hxc]
// (warm started from the previous cycle) and Anderson (Pulay) mixing of the
// Hartree-xc potential until the RMS change of V_hxc is <= c->scf_tol.  The
// final orbitals are eigenvectors of the Hamiltonian built from the previous
// cycle's orbitals, as in any SCF.
int ks_ground_state(bse_ctx* c, int n_want) {
  const long nr = c->basis.nr;
  constexpr int kHist = 6;
  constexpr double kBeta = 0.3;
  DVec x(c), xo(c), f(c), hx(c), hf(c), sv(c);
  BSE_TRY(x.alloc((size_t)nr));
  BSE_TRY(xo.alloc((size_t)nr));
  BSE_TRY(f.alloc((size_t)nr));
  BSE_TRY(hx.alloc((size_t)kHist * nr));   // differences of successive inputs
  BSE_TRY(hf.alloc((size_t)kHist * nr));   // and of successive residuals
  BSE_TRY(sv.alloc(4 * (size_t)kHist * kHist + 64));
  if (!c->phir) BSE_TRY(ctx_alloc_t(c, &c->phir, (size_t)c->nvh * nr));
  BSE_TRY(zero_fill(x.p, nr, c->st));
  double res = 1e300;
  int nh = 0, head = 0;
  DVec xprev(c), fprev(c);
  BSE_TRY(xprev.alloc((size_t)nr));
  BSE_TRY(fprev.alloc((size_t)nr));
  for (int it = 0; it < c->scf_max_iter; ++it) {
    BSE_TRY(copy_dev(c, c->Vext, c->Vr, nr));
    BSE_TRY(axpby(1.0, x.p, 1.0, c->Vr, nr, c->st));
    // early cycles need no tighter eigenpairs than the potential they use
    const double gtol = std::max(c->gs_tol, std::min(1e-4, 0.1 * res));
    BSE_TRY(ground_state(c, n_want, gtol, it > 0));
    BSE_TRY(to_grid(c, c->Phi, c->nv, 1, c->phir));
    BSE_TRY(ks_fields(c, c->phir, xo.p));
    BSE_TRY(copy_dev(c, xo.p, f.p, nr));
    BSE_TRY(axpby(-1.0, x.p, 1.0, f.p, nr, c->st));  // f = V_out - V_in
    std::vector<double> r2;
    BSE_TRY(dots_host(c, f.p, f.p, 1, nr, sv.p, r2));
    res = std::sqrt(std::max(0.0, r2[0]) / (double)nr);
    c->scf_iters = it + 1;
    c->scf_resid = res;
    if (res <= c->scf_tol) break;
    if (it > 0) {  // history of differences
      double* dx = hx.p + (size_t)head * nr;
      double* df = hf.p + (size_t)head * nr;
      BSE_TRY(copy_dev(c, x.p, dx, nr));
      BSE_TRY(axpby(-1.0, xprev.p, 1.0, dx, nr, c->st));
      BSE_TRY(copy_dev(c, f.p, df, nr));
      BSE_TRY(axpby(-1.0, fprev.p, 1.0, df, nr, c->st));
      head = (head + 1) % kHist;
      nh = std::min(nh + 1, kHist);
    }
    BSE_TRY(copy_dev(c, x.p, xprev.p, nr));
    BSE_TRY(copy_dev(c, f.p, fprev.p, nr));
    // gamma = argmin |f - dF gamma| (normal equations on the host), then
    // x <- x + beta f - (dX + beta dF) gamma
    std::vector<double> gam(nh, 0.0);
    if (nh > 0) {
      std::vector<double> G((size_t)nh * nh), b(nh);
      BSE_TRY(gram_tall(c, hf.p, nh, hf.p, nh, nr, sv.p));
      BSE_TRY(to_host(c, sv.p, G, G.size()));
      BSE_TRY(gram_tall(c, hf.p, nh, f.p, 1, nr, sv.p));
      BSE_TRY(to_host(c, sv.p, b, b.size()));
      // regularised Cholesky solve of the small system
      double tr = 0.0;
      for (int i = 0; i < nh; ++i) tr += G[(size_t)i * nh + i];
      for (int i = 0; i < nh; ++i) G[(size_t)i * nh + i] += 1e-12 * tr / nh + 1e-300;
      if (host_cholesky(nh, G.data()) == 0) {
        std::vector<double> y(nh);
        for (int i = 0; i < nh; ++i) {
          double t = b[i];
          for (int k = 0; k < i; ++k) t -= G[(size_t)i * nh + k] * y[k];
          y[i] = t / G[(size_t)i * nh + i];
        }
        for (int i = nh - 1; i >= 0; --i) {
          double t = y[i];
          for (int k = i + 1; k < nh; ++k) t -= G[(size_t)k * nh + i] * gam[k];
          gam[i] = t / G[(size_t)i * nh + i];
        }
      }
    }
    BSE_TRY(axpby(kBeta, f.p, 1.0, x.p, nr, c->st));
    for (int i = 0; i < nh; ++i) {
      if (gam[i] == 0.0) continue;
      BSE_TRY(axpby(-gam[i], hx.p + (size_t)i * nr, 1.0, x.p, nr, c->st));
      BSE_TRY(axpby(-gam[i] * kBeta, hf.p + (size_t)i * nr, 1.0, x.p, nr, c->st));
    }
  }
  if (res > c->scf_tol)
    return fail(BSE_ENOCONV, "self-consistent ground state: RMS potential change %.3e above %.3e",
                res, c->scf_tol);
  // the Hamiltonian of the converged orbitals, and its eigenpairs
  BSE_TRY(copy_dev(c, c->Vext, c->Vr, nr));
  BSE_TRY(axpby(1.0, xo.p, 1.0, c->Vr, nr, c->st));
  BSE_TRY(ground_state(c, n_want, c->gs_tol, true));
  BSE_TRY(to_grid(c, c->Phi, c->nv, 1, c->phir));
  // f_xc and rho at the final orbitals (the operator's kernels)
  return ks_fields(c, c->phir, xo.p);
}

// f_Hxc * t for the density on the first (real) component of `w` [one
// complex grid]; `t` receives a copy of the density first.
static int ks_hxc_apply(bse_ctx* c, double2* w, double2* t) {
  const long nr = c->basis.nr;
  BSE_HIP(hipMemcpyAsync(t, w, sizeof(double2) * nr, hipMemcpyDeviceToDevice, c->st));
  BSE_TRY(fft3d(c->fft, w, 1, -1, c->st));
  BSE_TRY(mul_real_field(w, 1, nr, c->vc, 1.0 / (double)nr, c->st));
  BSE_TRY(fft3d(c->fft, w, 1, +1, c->st));
  return hxc_field(w, t, c->fxc, 1, nr, 1.0, c->st);
}

// D part of U for the self-consistent model (SM Sec. I, scissor
// derivation): added to U,
//   u^D_v = P_c { 2 [f_Hxc * Drho_x] phi_v - alpha sum_v' [v_c*(a_v' phi_v)] a_v'
//                 + alpha sum_v' [v_c*(phi_v' phi_v)] sum_v'' <a_v''|a_v'> phi_v'' },
//   Drho_x = sum a_v^2 - sum phi_v phi_v' <a_v'|a_v>
// (the factor 2: V_Hxc depends on <phi_v| through rho = 2 sum phi^2).
// A is the projected exciton; uses agrid sets 0-3 and drho as scratch.
static int ks_u_dpart(bse_ctx* c, const double* A, double* U) {
  const long npw = c->basis.npw, nv = c->nv, L = nv * npw, nr = c->basis.nr;
  const long gs = (long)c->nvh * nr;
  DVec O(c), Pt(c), G(c);
  BSE_TRY(O.alloc((size_t)nv * nv));
  BSE_TRY(Pt.alloc((size_t)L));
  BSE_TRY(G.alloc((size_t)L));
  BSE_TRY(gram_tall(c, A, nv, A, nv, npw, O.p));           // O[v][v'] = <a_v|a_v'>
  BSE_TRY(dgemm(0, 0, nv, npw, nv, 1.0, O.p, nv, c->Phi, npw, 0.0, Pt.p, npw, c->st));
  double2* a = c->agrid;
  double2* pt = c->agrid + gs;
  double2* zz = c->agrid + 2 * gs;
  double2* g = c->agrid + 3 * gs;
  BSE_TRY(to_grid(c, A, c->nv, 1, a));
  BSE_TRY(to_grid(c, Pt.p, c->nv, 1, pt));
  BSE_TRY(zero_fill(reinterpret_cast<double*>(zz), 2 * gs, c->st));
  BSE_TRY(force_density(a, pt, zz, c->phir, c->nv, nr, c->drho, c->st));  // (Drho_x, 0)
  BSE_TRY(ks_hxc_apply(c, c->drho, zz));
  BSE_TRY(combine(a, c->phir, nullptr, c->drho, nullptr, g, c->nv, 1, nr, 2.0, 0, c->st));
  if (c->alpha != 0.0) {
    // - alpha sum_v' [v_c*(a_v' phi_v)] a_v' + alpha sum_v' [v_c*(phi_v' phi_v)] (O phi)_v'
    BSE_TRY(exchange_like(c, a, a, c->phir, c->nv, g, -c->alpha));
    BSE_TRY(exchange_like(c, pt, c->phir, c->phir, c->nv, g, c->alpha));
  }
  BSE_TRY(from_grid(c, g, c->nv, 1, nullptr, nullptr, 0.0, G.p));
  BSE_TRY(proj_c(c, G.p, G.p, 1));
  return axpby(1.0, G.p, 1.0, U, L, c->st);
}

// Z-vector operator of Eq. 7 for the self-consistent model (Zp in the P_c
// space): P_c [ (H_KS - eps_v) Z_v + 4 (f_Hxc * sum_v' phi_v' Z_v') phi_v
//               - alpha sum_v' [v_c*(phi_v' phi_v)] Z_v' - alpha sum_v' [v_c*(Z_v' phi_v)] phi_v' ]
// (2 K^1e,KS + 2 K^2e,KS - K^1d,KS - K^2d,KS for real orbitals; H_KS holds
// -alpha K_x).  agrid sets 0-2 and drho are scratch.
static int ks_zop(bse_ctx* c, const double* Zp, double* out) {
  const long nr = c->basis.nr;
  const long gs = (long)c->nvh * nr;
  double2* z = c->agrid;
  double2* t = c->agrid + gs;
  double2* ex = c->agrid + 2 * gs;
  BSE_TRY(to_grid(c, Zp, c->nv, 1, z));
  if (c->alpha != 0.0) {
    // -alpha K_x Z_v (in H_KS), - K^1d,KS, - K^2d,KS:
    // -alpha sum_w [phi_w v_c*(phi_w Z_v) + Z_w v_c*(phi_w phi_v) + phi_w v_c*(Z_w phi_v)]
    BSE_TRY(zero_fill(reinterpret_cast<double*>(ex), 2 * gs, c->st));
    BSE_TRY(exchange_like(c, c->phir, c->phir, z, c->nv, ex, -c->alpha));
    BSE_TRY(exchange_like(c, z, c->phir, c->phir, c->nv, ex, -c->alpha));
    BSE_TRY(exchange_like(c, c->phir, z, c->phir, c->nv, ex, -c->alpha));
  }
  BSE_TRY(transition_density(c->phir, z, c->nv, 1, nr, c->drho, c->st));
  BSE_TRY(ks_hxc_apply(c, c->drho, t));
  BSE_TRY(combine(z, c->phir, c->Vr, c->drho, nullptr, z, c->nv, 1, nr, 4.0, 1, c->st));
  if (c->alpha != 0.0)
    BSE_TRY(axpby(1.0, reinterpret_cast<const double*>(ex), 1.0, reinterpret_cast<double*>(z),
                  2 * gs, c->st));
  BSE_TRY(from_grid(c, z, c->nv, 1, Zp, c->eps_d, 0.0, out));
  return proj_c(c, out, out, 1);
}

// ---------------------------------------------------------------------------
// U vector:  u_v = P_c[ s (v_c*Drho) a_v - sum_v' W(a_v' a_v) phi_v' ] - sum_v' S_vv' a_v'
// ---------------------------------------------------------------------------
int u_vector(bse_ctx* c, const double* Xs, double* U) {
  const long npw = c->basis.npw, nv = c->nv, L = nv * npw, nr = c->basis.nr;
  BSE_TRY(ensure_apply_work(c, c->ks ? 4 : 2));
  DVec S(c), G(c);
  BSE_TRY(S.alloc((size_t)nv * nv));
  BSE_TRY(G.alloc((size_t)L));
  double* A = c->A_s;
  BSE_TRY(proj_c(c, Xs, A, 1));
  // a localised frame assembles U for A~ = U^T A with the localised
  // orbitals (its pruned W terms) and rotates the result back
  const double* Ak = A;
  const double* Phik = c->Phi;
  if (c->loc) {
    BSE_TRY(rotate_bands(c, 1, A, c->A_rot, false));
    Ak = c->A_rot;
    Phik = c->Phi_loc;
  }
  BSE_TRY(to_grid(c, Ak, c->nv, 1, c->agrid));
  // kernel part before P_c, and S = <phi | K~ A>
  BSE_TRY(kernel_part(c, c->agrid, c->Zs));
  BSE_TRY(dgemm(0, 1, nv, nv, npw, 1.0, Phik, npw, c->Zs, npw, 0.0, S.p, nv, c->st));
  // g(r) = s (v_c*Drho) a - sum_v' sigma_{v'v} phi_v'  (drho holds v_c*Drho from kernel_part)
  double2* g1 = c->agrid + (long)c->nvh * nr;   // set 1: scratch
  const double2* y = nullptr;
  if (c->kmask & (BSE_K_1D_BARE | BSE_K_1D_PDEP)) {
    BSE_TRY(sigma_phi(c, c->agrid, g1));
    y = g1;
  }
  const double2* vd = (c->kmask & BSE_K_1E) ? c->drho : nullptr;
  BSE_TRY(combine(c->phik, c->agrid, c->Vr, vd, y, g1, c->nv, 1, nr, c->spin, 0, c->st));
  BSE_TRY(from_grid(c, g1, c->nv, 1, nullptr, nullptr, 0.0, G.p));
  BSE_TRY(proj_c(c, G.p, U, 1));
  BSE_TRY(dgemm(0, 0, nv, npw, nv, -1.0, S.p, nv, Ak, npw, 1.0, U, npw, c->st));
  if (c->loc) {
    BSE_TRY(rotate_bands(c, 1, U, G.p, true));
    BSE_TRY(copy_dev(c, G.p, U, (size_t)L));
  }
  if (c->ks) BSE_TRY(ks_u_dpart(c, A, U));
  BSE_HIP(hipStreamSynchronize(c->st));
  return BSE_OK;
}

// ---------------------------------------------------------------------------
// Learned preconditioner: per-band features -> (shift sigma_v, gamma_v)
// ---------------------------------------------------------------------------
// Features of every band (layout in the ABI header); U = NULL leaves the
// u-dependent ones at 0 (Davidson).
int learned_features(bse_ctx* c, const double* U, std::vector<float>& F) {
  const int nv = c->nv;
  if (c->norb <= nv || (int)c->eps_h.size() <= nv)
    return fail(BSE_ESTATE, "learned features need eps_{N_v+1} (n_orb > n_val)");
  DVec o(c);
  BSE_TRY(o.alloc(4 * (size_t)nv));
  BSE_TRY(band_features(c->Phi, c->T, c->eps_d, U, c->phir, kPrecondShift, nv, c->basis.npw,
                        c->basis.nr, o.p, c->st));
  std::vector<double> h(4 * (size_t)nv);
  BSE_TRY(to_host(c, o.p, h, h.size()));
  const double eh = c->eps_h[nv - 1], el = c->eps_h[nv], om = c->basis.omega;
  F.assign((size_t)nv * BSE_LEARN_NFEAT, 0.0f);
  for (int v = 0; v < nv; ++v) {
    float* f = F.data() + (size_t)v * BSE_LEARN_NFEAT;
    const double e = c->eps_h[v], t = h[4 * v], u2 = h[4 * v + 1], upu = h[4 * v + 2];
    const double ipr = om * om * h[4 * v + 3] / (double)c->basis.nr;
    f[0] = (float)(e - eh);
    f[1] = (float)(el - e);
    f[2] = (float)t;
    f[3] = (float)(e - t);
    f[4] = (float)std::log(std::max(ipr, 1e-300));
    if (U) {
      f[5] = (float)(0.5 * std::log(std::max(u2, 1e-300)));
      f[6] = (float)(u2 > 0 ? upu / u2 : 0.0);
      f[7] = 1.0f;
    }
  }
  return BSE_OK;
}

// Network outputs -> sigma_v (Ha) and gamma_v; returns false when an output
// is not finite (the caller falls back to the diagonal preconditioner).
int learned_eval(bse_ctx* c, const std::vector<float>& F, std::vector<double>& sigma,
                 std::vector<double>& gamma, bool* ok) {
  const int nv = c->nv;
  float *xd = nullptr, *yd = nullptr;
  BSE_TRY(ctx_alloc_t(c, &xd, F.size()));
  int rc = ctx_alloc_t(c, &yd, (size_t)nv * BSE_LEARN_NOUT);
  std::vector<float> y((size_t)nv * BSE_LEARN_NOUT);
  if (rc == BSE_OK) {
    auto run = [&]() -> int {
      BSE_TRY(stage_h2d(&c->hstage, F.data(), xd, sizeof(float) * F.size(), c->st));
      BSE_TRY(mlp_eval(c->learned, nv, xd, yd, c->st));
      return stage_d2h(&c->hstage, yd, y.data(), sizeof(float) * y.size(), c->st);
    };
    rc = run();
  }
  ctx_release(c, xd);
  ctx_release(c, yd);
  BSE_TRY(rc);
  sigma.assign(nv, kPrecondShift);
  gamma.assign(nv, 0.0);
  *ok = true;
  for (int v = 0; v < nv; ++v) {
    const double o0 = y[(size_t)v * 2], o1 = y[(size_t)v * 2 + 1];
    if (!std::isfinite(o0) || !std::isfinite(o1)) {
      *ok = false;
      return BSE_OK;
    }
    sigma[v] = kPrecondShift * std::exp(std::min(3.0, std::max(-3.0, o0)));
    gamma[v] = std::exp(std::min(8.0, std::max(-6.0, o1)));
  }
  return BSE_OK;
}

// ---------------------------------------------------------------------------
// Z-vector:  P_c (H - eps_v) P_c Z_v = -u_v, block PCG with per-band steps
// ---------------------------------------------------------------------------
struct PcgOut {
  int iters = 0;
  double rel = 0.0;
  bool fallback = false;
};

// Solve P_c (H - eps_v) P_c Z = rhs from the current Z (projected first)
// until ||rhs - D Z||_F <= tol ||rhs||_F (or, with band_iters, until every
// band's own relative residual is <= tol, recording when each got there);
// fp32 selects the FP32-grid H.  vshift: per-band preconditioner shifts
// (NULL: kPrecondShift); dropped for the default if the residual grows in two
// consecutive iterations.
static int pcg(bse_ctx* c, const double* rhs, double* Z, double tol, int maxit, bool fp32,
               const double* vshift, int* band_iters, PcgOut* out, bool two_level) {
  const long npw = c->basis.npw, nv = c->nv, L = nv * npw;
  DVec R(c), P(c), AP(c), Zr(c), sv(c);
  BSE_TRY(R.alloc(L));
  BSE_TRY(P.alloc(L));
  BSE_TRY(AP.alloc(L));
  BSE_TRY(Zr.alloc(L));
  BSE_TRY(sv.alloc(4 * (size_t)nv + 16));
  std::vector<double> d;
  BSE_TRY(dots_host(c, rhs, rhs, nv, npw, sv.p, d));
  const double nb_ = std::sqrt(std::accumulate(d.begin(), d.end(), 0.0));
  // the operator on vectors already in the P_c space (Z after its initial
  // projection, and the search directions, built from projected
  // preconditioned residuals); its output is projected
  auto applyD = [&](const double* in, double* o_) -> int {
    if (c->ks) return ks_zop(c, in, o_);
    if (fp32) return apply_H_f(c, (int)nv, 1, in, o_, 0.0, c->eps_d, 1);
    return apply_H(c, (int)nv, 1, in, o_, c->agrid, 0.0, c->eps_d, 1);
  };
  // with the KS kernels the bands couple: one step length for the block
  const bool block_steps = c->ks != 0;
  auto pool = [&](std::vector<double>& x) {
    if (!block_steps) return;
    const double t = std::accumulate(x.begin(), x.end(), 0.0);
    std::fill(x.begin(), x.end(), t);
  };
  std::vector<double> rz, pap, rzn, rr;
  // P = P_c Prec(R), rz = <R, P> per band
  // Zr = M^-1 R (kinetic diagonal, or two-level on the conduction states held)
  auto prec = [&](const double* r, double* t) -> int {
    auto kin = [&](double* w) {
      return precond_cg(w, w, c->T, c->eps_d, kPrecondShift, (int)nv, (int)npw, c->st, vshift);
    };
    if (t != r) BSE_HIP(hipMemcpyAsync(t, r, sizeof(double) * L, hipMemcpyDeviceToDevice, c->st));
    if (two_level) return precond_two_level(c, t, 1, nullptr, 0.0, 1e-12, kin);
    return kin(t);
  };
  auto restart = [&]() -> int {
    BSE_TRY(prec(R.p, Zr.p));
    BSE_TRY(proj_c(c, Zr.p, P.p, 1));
    BSE_TRY(dots_host(c, R.p, P.p, nv, npw, sv.p, rz));
    pool(rz);
    return BSE_OK;
  };
  BSE_TRY(proj_c(c, Z, Z, 1));
  BSE_TRY(applyD(Z, AP.p));
  BSE_TRY(axpby(1.0, rhs, 0.0, R.p, L, c->st));
  BSE_TRY(axpby(-1.0, AP.p, 1.0, R.p, L, c->st));
  BSE_TRY(restart());
  if (band_iters)
    for (long v = 0; v < nv; ++v) band_iters[v] = -1;
  double rel = 0.0, prev = 1e300;
  int grew = 0;
  int it = 0;
  bool conv = false;
  for (it = 0; it < maxit; ++it) {
    BSE_TRY(dots_host(c, R.p, R.p, nv, npw, sv.p, rr));
    rel = nb_ > 0 ? std::sqrt(std::accumulate(rr.begin(), rr.end(), 0.0)) / nb_ : 0.0;
    if (band_iters) {
      bool all = true;
      for (long v = 0; v < nv; ++v) {
        if (band_iters[v] < 0 && (d[v] <= 0 || std::sqrt(rr[v] / d[v]) <= tol)) band_iters[v] = it;
        all = all && band_iters[v] >= 0;
      }
      if (all) {
        conv = true;
        break;
      }
    } else if (rel <= tol) {
      conv = true;
      break;
    }
    if (vshift) {  // fallback rule of the learned preconditioner
      grew = rel > prev ? grew + 1 : 0;
      if (grew >= 2 || !std::isfinite(rel)) {
        vshift = nullptr;
        out->fallback = true;
        BSE_TRY(restart());
        grew = 0;
      }
    }
    prev = rel;
    BSE_TRY(applyD(P.p, AP.p));
    BSE_TRY(dots_host(c, P.p, AP.p, nv, npw, sv.p, pap));
    pool(pap);
    std::vector<double> al(nv), nal(nv);
    for (long v = 0; v < nv; ++v) {
      al[v] = pap[v] != 0.0 ? rz[v] / pap[v] : 0.0;
      nal[v] = -al[v];
    }
    BSE_TRY(to_dev(c, al, sv.p + nv, nv));
    BSE_TRY(to_dev(c, nal, sv.p + 2 * nv, nv));
    BSE_TRY(row_axpby(sv.p + nv, P.p, nullptr, Z, nv, npw, c->st));
    BSE_TRY(row_axpby(sv.p + 2 * nv, AP.p, nullptr, R.p, nv, npw, c->st));
    BSE_TRY(prec(R.p, AP.p));
    BSE_TRY(proj_c(c, AP.p, Zr.p, 1));
    BSE_TRY(dots_host(c, R.p, Zr.p, nv, npw, sv.p, rzn));
    pool(rzn);
    std::vector<double> be(nv);
    for (long v = 0; v < nv; ++v) be[v] = rz[v] != 0.0 ? rzn[v] / rz[v] : 0.0;
    BSE_TRY(to_dev(c, be, sv.p + 3 * nv, nv));
    BSE_TRY(row_axpby(nullptr, Zr.p, sv.p + 3 * nv, P.p, nv, npw, c->st));
    rz = rzn;
  }
  out->iters = it;
  out->rel = rel;
  return conv ? BSE_OK : BSE_ENOCONV;
}

// p_v = P_c Prec_v(rhs_v) with the default shift (two-level form if asked), into P
static int precond_rhs(bse_ctx* c, const double* rhs, double* P, bool two_level) {
  const long L = (long)c->nv * c->basis.npw;
  BSE_HIP(hipMemcpyAsync(P, rhs, sizeof(double) * L, hipMemcpyDeviceToDevice, c->st));
  auto kin = [&](double* w) {
    return precond_cg(w, w, c->T, c->eps_d, kPrecondShift, c->nv, c->basis.npw, c->st);
  };
  if (two_level && c->norb > c->nv)
    BSE_TRY(precond_two_level(c, P, 1, nullptr, 0.0, 1e-12, kin));
  else
    BSE_TRY(kin(P));
  return proj_c(c, P, P, 1);
}

int zvector(bse_ctx* c, const double* Xs, const bse_solver_opts* o, double* Z,
            bse_solver_stats* stats) {
  const auto t0 = std::chrono::steady_clock::now();
  const double tol = (o && o->tol > 0) ? o->tol : 1e-8;
  const int maxit = (o && o->max_iter > 0) ? o->max_iter : 5000;
  const long npw = c->basis.npw, nv = c->nv, L = nv * npw;
  BSE_TRY(ensure_apply_work(c, c->ks ? 4 : 2));
  DVec U(c), R(c), D(c), sv(c), vs(c);
  BSE_TRY(U.alloc(L));
  BSE_TRY(sv.alloc(16 + 2 * (size_t)nv));
  BSE_TRY(vs.alloc((size_t)nv));
  BSE_TRY(u_vector(c, Xs, U.p));
  BSE_TRY(proj_c(c, U.p, U.p, 1));
  BSE_TRY(axpby(-1.0, U.p, 0.0, U.p, L, c->st));  // U <- -U: the right-hand side
  BSE_HIP(hipStreamSynchronize(c->st));
  const double t_u = elapsed_ms(t0);
  // per-band preconditioner shifts and initial guess
  const double* vshift = nullptr;
  bool learned = false, fallback = false;
  std::vector<double> gam;
  if (o && o->precond_shift_host) {
    BSE_TRY(to_dev(c, o->precond_shift_host, vs.p, nv));
    vshift = vs.p;
  } else if (o && o->use_learned && c->learned) {
    std::vector<float> F;
    std::vector<double> sig;
    BSE_TRY(learned_features(c, U.p, F));  // U holds -u: features use |u| only
    bool ok = false;
    BSE_TRY(learned_eval(c, F, sig, gam, &ok));
    if (ok) {
      BSE_TRY(to_dev(c, sig, vs.p, nv));
      vshift = vs.p;
      learned = true;
    } else {
      fallback = true;
    }
  }
  if (o && o->z0_dev) {
    BSE_TRY(proj_c(c, o->z0_dev, Z, 1));
  } else if (learned) {  // Z0_v = gamma_v P_c Prec_v(-u_v)
    BSE_TRY(precond_rhs(c, U.p, Z, o->two_level && c->norb > c->nv));
    BSE_TRY(to_dev(c, gam, sv.p + 16, nv));
    BSE_TRY(row_scale(sv.p + 16, Z, nv, npw, c->st));
  } else {
    BSE_HIP(hipMemsetAsync(Z, 0, sizeof(double) * L, c->st));
  }
  int* band_iters = o ? o->band_iters_host : nullptr;
  const bool two_level = o && o->two_level && c->norb > c->nv;
  int iters = 0, rc = BSE_OK, applies64 = 0;
  double rel = 0.0;
  PcgOut po;
  if (c->active != BSE_MIXED || band_iters || c->ks) {
    rc = pcg(c, U.p, Z, tol, maxit, false, vshift, band_iters, &po, two_level);
    iters = po.iters;
    rel = po.rel;
    fallback = fallback || po.fallback;
    applies64 = iters + 1;
  } else {
    // iterative refinement: FP64 residual outside, FP32-grid PCG inside
    BSE_TRY(R.alloc(L));
    BSE_TRY(D.alloc(L));
    BSE_TRY(ensure_mixed_work(c, 1));
    std::vector<double> un, rn;
    BSE_TRY(dots_host(c, U.p, U.p, nv, npw, sv.p, un));
    const double nu = std::sqrt(std::accumulate(un.begin(), un.end(), 0.0));
    rc = BSE_ENOCONV;
    for (int outer = 0; outer < 30 && iters < maxit; ++outer) {
      BSE_TRY(proj_c(c, Z, D.p, 1));
      BSE_TRY(apply_H(c, (int)nv, 1, D.p, R.p, c->agrid, 0.0, c->eps_d, 1));
      ++applies64;
      BSE_TRY(axpby(1.0, U.p, -1.0, R.p, L, c->st));  // R = rhs - D Z
      BSE_TRY(dots_host(c, R.p, R.p, nv, npw, sv.p, rn));
      rel = nu > 0 ? std::sqrt(std::accumulate(rn.begin(), rn.end(), 0.0)) / nu : 0.0;
      if (rel <= tol) {
        rc = BSE_OK;
        break;
      }
      // inner target: the FP32 limit, or just past what the outer step needs
      const double itol = std::max(kMixedInnerTol, 0.5 * tol / rel);
      BSE_HIP(hipMemsetAsync(D.p, 0, sizeof(double) * L, c->st));
      const int irc = pcg(c, R.p, D.p, itol, maxit - iters, true, vshift, nullptr, &po, two_level);
      iters += po.iters;
      fallback = fallback || po.fallback;
      if (po.fallback) vshift = nullptr;
      if (irc != BSE_OK && irc != BSE_ENOCONV) return irc;
      BSE_TRY(axpby(1.0, D.p, 1.0, Z, L, c->st));
    }
  }
  BSE_HIP(hipStreamSynchronize(c->st));
  if (stats) {
    stats->iters = iters;
    stats->applies = c->active == BSE_MIXED && !band_iters ? iters + applies64 : iters + 1;
    stats->applies_fp64 = applies64;
    stats->resid[0] = rel;
    stats->t_ms = elapsed_ms(t0);
    stats->t_u_ms = t_u;
    stats->learned = learned ? 1 : 0;
    stats->fallback = fallback ? 1 : 0;
  }
  if (rc == BSE_ENOCONV)
    return fail(BSE_ENOCONV, "Z-vector CG: residual %.3e after %d iterations", rel, iters);
  return rc;
}

// features of the Z-vector solve and, with Zref, the least-squares
// initial-guess coefficients gamma_v* = <p_v, Z_v> / <p_v, p_v>
int learned_targets(bse_ctx* c, const double* Xs, const double* Zref, bool two_level, float* feat,
                    double* gamma) {
  const long npw = c->basis.npw, nv = c->nv, L = nv * npw;
  BSE_TRY(ensure_apply_work(c, 2));
  DVec U(c), P(c), sv(c);
  BSE_TRY(U.alloc(L));
  BSE_TRY(sv.alloc(2 * (size_t)nv + 16));
  BSE_TRY(u_vector(c, Xs, U.p));
  BSE_TRY(proj_c(c, U.p, U.p, 1));
  BSE_TRY(axpby(-1.0, U.p, 0.0, U.p, L, c->st));
  std::vector<float> F;
  BSE_TRY(learned_features(c, U.p, F));
  if (feat) std::copy(F.begin(), F.end(), feat);
  if (Zref && gamma) {
    BSE_TRY(P.alloc(L));
    BSE_TRY(precond_rhs(c, U.p, P.p, two_level));
    std::vector<double> pz, pp;
    BSE_TRY(dots_host(c, P.p, Zref, nv, npw, sv.p, pz));
    BSE_TRY(dots_host(c, P.p, P.p, nv, npw, sv.p, pp));
    for (long v = 0; v < nv; ++v) gamma[v] = pp[v] > 0 ? pz[v] / pp[v] : 0.0;
  }
  return BSE_OK;
}

// ---------------------------------------------------------------------------
// d omega / d R (Eqs. 4-6)
// ---------------------------------------------------------------------------
int forces(bse_ctx* c, const double* Xs, const double* Zin, double* dwdR_host) {
  const long npw = c->basis.npw, nv = c->nv, L = nv * npw, nr = c->basis.nr;
  BSE_TRY(ensure_apply_work(c, 3));
  DVec O(c), Pt(c), Zp(c), part(c), outd(c);
  BSE_TRY(O.alloc((size_t)nv * nv));
  BSE_TRY(Pt.alloc(L));
  BSE_TRY(Zp.alloc(L));
  const long pl = force_reduce_work(c->nsites, nr);
  BSE_TRY(part.alloc((size_t)std::max(pl, 1L)));
  BSE_TRY(outd.alloc((size_t)3 * std::max(c->nsites, 1)));
  BSE_TRY(proj_c(c, Xs, c->A_s, 1));
  BSE_TRY(proj_c(c, Zin, Zp.p, 1));
  BSE_TRY(gram_tall(c, c->A_s, nv, c->A_s, nv, npw, O.p));  // O[v][v'] = <a_v|a_v'>
  BSE_TRY(dgemm(0, 0, nv, npw, nv, 1.0, O.p, nv, c->Phi, npw, 0.0, Pt.p, npw, c->st));
  const long gs = (long)c->nvh * nr;
  BSE_TRY(to_grid(c, c->A_s, c->nv, 1, c->agrid));
  BSE_TRY(to_grid(c, Pt.p, c->nv, 1, c->agrid + gs));
  BSE_TRY(to_grid(c, Zp.p, c->nv, 1, c->agrid + 2 * gs));
  BSE_TRY(force_density(c->agrid, c->agrid + gs, c->agrid + 2 * gs, c->phir, c->nv, nr, c->drho,
                        c->st));
  BSE_TRY(fft3d(c->fft, c->drho, 1, -1, c->st));
  if (c->nsites > 0) {
    BSE_TRY(force_reduce(c->drho, c->sites, c->sites + 3 * c->nsites, c->sites + 4 * c->nsites,
                         c->nsites, c->basis.grid, c->basis.cell, part.p, pl, outd.p, c->st));
    BSE_TRY(to_host(c, outd.p, dwdR_host, (size_t)3 * c->nsites));
  }
  BSE_HIP(hipStreamSynchronize(c->st));
  return BSE_OK;
}

// d(sum_v eps_v)/dR = sum_v <phi_v| dV/dR |phi_v> (Hellmann-Feynman): the
// occupied density contracted with each site's potential derivative, the
// same reduction as d omega/d R with rho_t replaced by sum_v phi_v^2.
int ground_state_forces(bse_ctx* c, double* dEdR_host) {
  const long nr = c->basis.nr;
  if (c->nsites <= 0) return BSE_OK;
  DVec rho(c), part(c), outd(c);
  const long pl = force_reduce_work(c->nsites, nr);
  BSE_TRY(rho.alloc((size_t)2 * nr));  // one complex grid
  BSE_TRY(part.alloc((size_t)std::max(pl, 1L)));
  BSE_TRY(outd.alloc((size_t)3 * c->nsites));
  double2* rg = reinterpret_cast<double2*>(rho.p);
  BSE_TRY(occupied_density(c->phir, c->nv, nr, rg, c->st));
  BSE_TRY(fft3d(c->fft, rg, 1, -1, c->st));
  BSE_TRY(force_reduce(rg, c->sites, c->sites + 3 * c->nsites, c->sites + 4 * c->nsites,
                       c->nsites, c->basis.grid, c->basis.cell, part.p, pl, outd.p, c->st));
  BSE_TRY(to_host(c, outd.p, dEdR_host, (size_t)3 * c->nsites));
  BSE_HIP(hipStreamSynchronize(c->st));
  return BSE_OK;
}

// ---------------------------------------------------------------------------
// Ground state: lowest n_want eigenpairs of H = T + V by Chebyshev-filtered
// subspace iteration (the scaled three-term filter of Zhou, Saad, Tiago and
// Chelikowsky, J. Comput. Phys. 219, 172 (2006)) with Rayleigh-Ritz.
// ---------------------------------------------------------------------------
int ground_state(bse_ctx* c, int n_want, double tol, bool warm) {
  PhaseScope ps(c, PH_GS);
  const long npw = c->basis.npw;
  int ns = n_want + std::max(8, n_want / 10);
  if (ns > npw) ns = (int)npw;
  if (n_want > ns) return fail(BSE_EINVAL, "ground state: %d states exceed the basis", n_want);
  const long nsl = ns;
  DVec X(c), Y(c), Z(c), HX(c), sm(c);
  BSE_TRY(X.alloc(nsl * npw));
  BSE_TRY(Y.alloc(nsl * npw));
  BSE_TRY(Z.alloc(nsl * npw));
  BSE_TRY(HX.alloc(nsl * npw));
  BSE_TRY(sm.alloc(nsl * nsl + 4 * nsl + 16));
  double2* grids = nullptr;
  BSE_TRY(ctx_alloc_t(c, &grids, (size_t)((ns + 1) / 2) * c->basis.nr));
  struct Rel {
    bse_ctx* c;
    void* p;
    ~Rel() { ctx_release(c, p); }
  } rel_g{c, grids};
  double* Cd = sm.p;
  double* vec = sm.p + nsl * nsl;
  // random start (fixed seed, drawn on the device), smooth: divided by
  // (1 + |G|^2/2)
  BSE_TRY(random_smooth(X.p, nsl, npw, c->T, 12345ULL, c->st));
  // a warm start keeps the previous solution's states (self-consistent
  // cycles), the rest of the block stays random
  if (warm && c->Phi && c->norb > 0)
    BSE_TRY(copy_dev(c, c->Phi, X.p, (size_t)std::min(c->norb, ns) * npw));
  auto Happly = [&](const double* in, double* out, double shift) -> int {
    return apply_H(c, ns, 1, in, out, grids, shift, nullptr, 0);
  };
  std::vector<double> theta(ns);
  auto rayleigh_ritz = [&]() -> int {
    // Cholesky QR once the filtered basis is well conditioned; the Gram
    // eigen-decomposition (which can drop directions) otherwise
    int k = chol_orth(c, X.p, nsl, npw, Z.p);
    if (k == 0) k = orth_block(c, nullptr, 0, X.p, nsl, npw, Z.p, 2, 1e-12);
    if (k < 0) return -k;
    if (k < ns) return fail(BSE_EINVAL, "ground state: subspace collapsed (%d of %d)", k, ns);
    BSE_TRY(Happly(X.p, HX.p, 0.0));
    BSE_TRY(gram_tall(c, X.p, nsl, HX.p, nsl, npw, Cd));
    std::vector<double> Hs(nsl * nsl);
    BSE_TRY(to_host(c, Cd, Hs, Hs.size()));
    if (host_syev(ns, Hs.data(), theta.data())) return fail(BSE_EINVAL, "ground state: RR failed");
    BSE_TRY(to_dev(c, Hs, Cd, Hs.size()));
    BSE_TRY(dgemm(1, 0, nsl, npw, nsl, 1.0, Cd, nsl, X.p, npw, 0.0, Z.p, npw, c->st));
    BSE_TRY(copy_dev(c, Z.p, X.p, nsl * npw));
    BSE_TRY(dgemm(1, 0, nsl, npw, nsl, 1.0, Cd, nsl, HX.p, npw, 0.0, Z.p, npw, c->st));
    BSE_TRY(copy_dev(c, Z.p, HX.p, nsl * npw));
    return BSE_OK;
  };
  // upper bound of the spectrum: |G|^2/2 <= ecut and <x|V|x> <= max V(r)
  std::vector<double> vr(c->basis.nr);
  BSE_TRY(to_host(c, c->Vr, vr, vr.size()));
  const double vmax = *std::max_element(vr.begin(), vr.end());
  const double bup = c->basis.ecut + std::max(0.0, vmax) + 0.5;
  BSE_TRY(rayleigh_ritz());
  const int degree = 16;
  double resid = 1e300;
  for (int it = 0; it < 200; ++it) {
    // residuals of the wanted states
    std::vector<double> nt(n_want);
    for (int i = 0; i < n_want; ++i) nt[i] = -theta[i];
    BSE_TRY(to_dev(c, nt, vec, n_want));
    BSE_TRY(copy_dev(c, HX.p, Z.p, (size_t)n_want * npw));
    BSE_TRY(row_axpby(vec, X.p, nullptr, Z.p, n_want, npw, c->st));
    std::vector<double> r2;
    BSE_TRY(dots_host(c, Z.p, Z.p, n_want, npw, vec, r2));
    resid = 0;
    double resid_x = 0;  // the states above the occupied ones
    for (int i = 0; i < n_want; ++i) {
      const double r = std::sqrt(std::max(0.0, r2[i]));
      if (i < c->nv)
        resid = std::max(resid, r);
      else
        resid_x = std::max(resid_x, r);
    }
    if (resid <= tol && resid_x <= std::max(tol, kExtraStateTol)) break;
    // filter [a, bup] out, amplify below a
    const double a = theta[ns - 1], a0 = theta[0];
    const double e = 0.5 * (bup - a), cc = 0.5 * (bup + a);
    double sigma = e / (a0 - cc);
    const double tau = 2.0 / sigma;
    // Y = (H - cc) X * sigma / e
    BSE_TRY(Happly(X.p, Y.p, -cc));
    BSE_TRY(axpby(0.0, X.p, sigma / e, Y.p, nsl * npw, c->st));
    for (int d = 2; d <= degree; ++d) {
      const double sn = 1.0 / (tau - sigma);
      BSE_TRY(Happly(Y.p, Z.p, -cc));
      // Z = 2 sn/e (H - cc) Y - sigma sn X
      BSE_TRY(axpby(-sigma * sn, X.p, 2.0 * sn / e, Z.p, nsl * npw, c->st));
      std::swap(X.p, Y.p);  // X <- Y
      std::swap(Y.p, Z.p);  // Y <- Z, Z free
      sigma = sn;
    }
    std::swap(X.p, Y.p);
    BSE_TRY(rayleigh_ritz());
    ++c->gs_sweeps;
  }
  c->gs_resid = resid;
  if (resid > tol) return fail(BSE_ENOCONV, "ground state: residual %.3e above %.3e", resid, tol);
  if (c->Phi && c->norb != n_want) {
    ctx_release(c, c->Phi);
    ctx_release(c, c->eps_d);
    c->Phi = nullptr;
    c->eps_d = nullptr;
  }
  c->norb = n_want;
  if (!c->Phi) {
    BSE_TRY(ctx_alloc_t(c, &c->Phi, (size_t)n_want * npw));
    BSE_TRY(ctx_alloc_t(c, &c->eps_d, (size_t)n_want));
  }
  BSE_TRY(copy_dev(c, X.p, c->Phi, (size_t)n_want * npw));
  c->eps_h.assign(theta.begin(), theta.begin() + n_want);
  BSE_TRY(to_dev(c, c->eps_h.data(), c->eps_d, n_want));
  return BSE_OK;
}

}  // namespace bsex
