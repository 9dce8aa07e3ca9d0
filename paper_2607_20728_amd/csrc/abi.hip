// C ABI entry points: validation, context set-up, dispatch to the solvers.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>

#include "context.h"

namespace bsex {
const char* last_error();
int davidson(bse_ctx* c, int ns, const bse_solver_opts* o, double* omega, double* Xout,
             bse_solver_stats* stats);
int u_vector(bse_ctx* c, const double* Xs, double* U);
int zvector(bse_ctx* c, const double* Xs, const bse_solver_opts* o, double* Z,
            bse_solver_stats* stats);
int forces(bse_ctx* c, const double* Xs, const double* Zin, double* dwdR_host);
int ground_state_forces(bse_ctx* c, double* dEdR_host);
}  // namespace bsex

using namespace bsex;

namespace {

bool finite_all(const double* p, long n) {
  for (long i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

void ctx_destroy(bse_ctx* c) {
  if (!c) return;
  if (c->st) (void)hipStreamSynchronize(c->st);
  graphs_destroy(c);
  if (c->cap_st) (void)hipStreamDestroy(c->cap_st);
  if (cache_keeps()) {  // once the stream (the null stream too) has drained
    (void)hipStreamSynchronize(c->st);
    for (auto& b : c->allocs) cache_put(b);
    for (auto& b : c->pool) cache_put(b);
  } else {
    for (auto& b : c->allocs) (void)hipFree(b.p);
    for (auto& b : c->pool) (void)hipFree(b.p);
  }
  c->allocs.clear();
  c->pool.clear();
  fft_plan_free(&c->fft);
  sphere_plan_free(&c->sp);
  for (auto e : c->ev_pool) (void)hipEventDestroy(e);
  stage_free(&c->hstage);
  delete c;
}

int upload(bse_ctx* c, void* dst, const void* src, size_t bytes) {
  return stage_h2d(&c->hstage, src, dst, bytes, c->st);
}

int validate(const bse_system_desc* d) {
  if (!d) return fail(BSE_EINVAL, "desc is NULL");
  if (d->abi_version != BSEX_ABI_VERSION)
    return fail(BSE_EABI, "desc.abi_version %d, library %d", d->abi_version, BSEX_ABI_VERSION);
  if (d->n_sites < 0) return fail(BSE_EINVAL, "n_sites < 0");
  if (d->n_sites > 0) {
    if (!d->site_xyz || !d->site_depth || !d->site_width)
      return fail(BSE_EINVAL, "site arrays must be given when n_sites > 0");
    if (!finite_all(d->site_xyz, 3L * d->n_sites) || !finite_all(d->site_depth, d->n_sites) ||
        !finite_all(d->site_width, d->n_sites))
      return fail(BSE_EINVAL, "non-finite site data");
    for (int i = 0; i < d->n_sites; ++i)
      if (!(d->site_width[i] > 0)) return fail(BSE_EINVAL, "site_width[%d] must be positive", i);
  }
  if (d->n_val < 1) return fail(BSE_EINVAL, "n_val must be >= 1");
  if (d->n_pdep < 0) return fail(BSE_EINVAL, "n_pdep < 0");
  if (d->n_pdep > 0 && (!d->pdep || !d->lambda))
    return fail(BSE_EINVAL, "pdep and lambda must be given when n_pdep > 0");
  if (!std::isfinite(d->scissor) || !std::isfinite(d->spin_factor))
    return fail(BSE_EINVAL, "scissor and spin_factor must be finite");
  if (d->precision != BSE_FP64 && d->precision != BSE_MIXED)
    return fail(BSE_EINVAL, "precision %d unsupported", d->precision);
  if (d->precision == BSE_MIXED && d->tau_policy == BSE_TAU_REBUILD)
    return fail(BSE_EINVAL, "BSE_MIXED keeps the FP32 tau cache; tau_policy REBUILD conflicts");
  if (d->tau_policy < BSE_TAU_AUTO || d->tau_policy > BSE_TAU_REBUILD)
    return fail(BSE_EINVAL, "tau_policy %d unknown", d->tau_policy);
  if (d->tau_budget_bytes < 0) return fail(BSE_EINVAL, "tau_budget_bytes < 0");
  if (d->kernel_mask < 0 || d->kernel_mask > BSE_K_ALL)
    return fail(BSE_EINVAL, "kernel_mask %d out of range", d->kernel_mask);
  if (d->n_orb < 0 || (d->n_orb > 0 && d->n_orb < d->n_val))
    return fail(BSE_EINVAL, "n_orb must be 0 or >= n_val");
  if (d->n_orb > 0 && (!d->orbitals || !d->eps))
    return fail(BSE_EINVAL, "orbitals and eps must be given when n_orb > 0");
  if (d->n_extra < 0) return fail(BSE_EINVAL, "n_extra < 0");
  if (!std::isfinite(d->gap_min) || !std::isfinite(d->gs_tol) || d->gs_tol < 0)
    return fail(BSE_EINVAL, "gap_min / gs_tol invalid");
  if (d->ks_model != 0 && d->ks_model != 1) return fail(BSE_EINVAL, "ks_model %d unknown", d->ks_model);
  if (!std::isfinite(d->rho_floor) || d->rho_floor < 0 || !std::isfinite(d->scf_tol) ||
      d->scf_tol < 0)
    return fail(BSE_EINVAL, "rho_floor / scf_tol invalid");
  if (!std::isfinite(d->alpha_exx) || d->alpha_exx < 0 || d->alpha_exx > 1)
    return fail(BSE_EINVAL, "alpha_exx must be in [0, 1]");
  if (d->alpha_exx != 0 && (d->ks_model != 1 || d->n_orb <= 0 || d->precision != BSE_FP64))
    return fail(BSE_EINVAL, "alpha_exx needs ks_model 1, orbitals supplied and BSE_FP64");
  if (d->localize != 0 && d->localize != 1) return fail(BSE_EINVAL, "localize %d unknown", d->localize);
  if (d->localize) {
    if (d->ks_model != 0) return fail(BSE_EINVAL, "localize needs ks_model 0");
    if (!std::isfinite(d->prune_threshold) || d->prune_threshold < 0 || d->prune_threshold > 1)
      return fail(BSE_EINVAL, "prune_threshold must be in [0, 1]");
    if (d->loc_max_sweeps < 0 || !std::isfinite(d->loc_tol) || d->loc_tol < 0)
      return fail(BSE_EINVAL, "loc_max_sweeps / loc_tol invalid");
    if (d->loc_rotation) {
      const long n = d->n_val;
      if (!finite_all(d->loc_rotation, n * n)) return fail(BSE_EINVAL, "non-finite loc_rotation");
      double worst = 0.0;  // U^T U = 1
      for (long i = 0; i < n; ++i)
        for (long j = i; j < n; ++j) {
          double s = 0.0;
          for (long v = 0; v < n; ++v) s += d->loc_rotation[v * n + i] * d->loc_rotation[v * n + j];
          worst = std::max(worst, std::fabs(s - (i == j ? 1.0 : 0.0)));
        }
      if (worst > 1e-8) return fail(BSE_EINVAL, "loc_rotation is not orthogonal (%.1e)", worst);
    }
  }
  return BSE_OK;
}

double ms_since(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

int plan_tau(bse_ctx* c, const bse_system_desc* d) {
  const long nr = c->basis.nr, npw = c->basis.npw;
  const long nB = (c->nv + 7) / 8;
  c->nblk_all = nB * (nB + 1) / 2;
  // the upper block triangle in row order, or the blocks a localised frame keeps
  std::vector<int2> ij;
  if (c->loc) {
    ij = c->blkIJ_h;
  } else {
    for (long I = 0; I < nB; ++I)
      for (long J = I; J < nB; ++J) ij.push_back(make_int2((int)I, (int)J));
  }
  c->nblk = (long)ij.size();
  BSE_TRY(ctx_alloc_t(c, &c->blkIJ, ij.size()));
  BSE_TRY(upload(c, c->blkIJ, ij.data(), sizeof(int2) * ij.size()));
  c->blkIJ_h = ij;
  // stream kernel geometry from the device LDS size
  int dev = 0;
  BSE_HIP(hipGetDevice(&dev));
  hipDeviceProp_t prop;
  BSE_HIP(hipGetDeviceProperties(&prop, dev));
  c->max_lds = prop.sharedMemPerBlock;
  // tuning knob of the stream kernel: 1 = quad-shared loads (default), 4 or
  // 2 = lanes sharing one grid point's vectors, each reading whole blocks
  if (const char* e = getenv("BSEX_TAU_BL")) {
    const int v = atoi(e);
    c->tau_bl = (v == 2 || v == 4) ? v : 1;
  }
  // grid points per stream workgroup: 2 when the kernel's LDS allows
  c->R = (tau_stream_lds(c->nv, 2, sizeof(double), c->tau_bl) <= c->max_lds) ? 2 : 1;
  if (const char* e = getenv("BSEX_TAU_R")) c->R = (atoi(e) == 1) ? 1 : c->R;
  if (tau_stream_lds(c->nv, c->R, sizeof(double), c->tau_bl) > c->max_lds)
    return fail(BSE_EINVAL, "n_val %d too large for the device LDS (%zu bytes)", c->nv, c->max_lds);
  const bool mixed = c->precision == BSE_MIXED;
  c->Rf = (tau_stream_lds(c->nv, 2, sizeof(float), c->tau_bl) <= c->max_lds) ? 2 : 1;
  if (const char* e = getenv("BSEX_TAU_R")) c->Rf = (atoi(e) == 1) ? 1 : c->Rf;
  if (mixed && tau_stream_lds(c->nv, c->Rf, sizeof(float), c->tau_bl) > c->max_lds)
    return fail(BSE_EINVAL, "n_val %d too large for the device LDS (%zu bytes)", c->nv, c->max_lds);
  BSE_TRY(tau_stream_set_lds_limit(c->max_lds));
  const bool need_k1d = (c->kmask & (BSE_K_1D_BARE | BSE_K_1D_PDEP)) != 0;
  // work for one apply chunk of 8 vectors (a(r) buffer; z is written in place)
  BSE_TRY(ensure_apply_work(c, 8));
  if (mixed) BSE_TRY(ensure_mixed_work(c, c->nbc));
  c->tau_policy = d->tau_policy;
  if (!need_k1d) return BSE_OK;
  // per 8x8 block: tau (64 N_r doubles) and, for a build tile, the complex
  // grids, rho_S, the PDEP coefficients and the result
  const double blk_bytes = 8.0 * 64 * nr;
  const double blk_tile_bytes = 8.0 * 64 * (2.0 * nr + 2.0 * npw + std::max(c->npdep, 1));
  size_t freeb = 0, totalb = 0;
  ctx_pool_flush(c);  // scratch of the ground-state solve goes back first
  BSE_TRY(mem_info(&freeb, &totalb));
  const bool has_budget = d->tau_budget_bytes > 0;
  // without an explicit budget, keep room for the solvers: a 128-vector
  // Davidson subspace and its products, the blocks beside them, graph
  // staging and the caller's own vectors, about 330 trial vectors in all,
  // but at most 12% of the device (the subspace shrinks to what is left)
  const double reserve =
      has_budget ? 1.0e9
                 : 4.0e9 + std::min(330 * 8.0 * c->nv * npw, 0.12 * (double)totalb);
  const long small_tile = std::min(c->nblk, 4L);
  double budget_left = has_budget ? (double)d->tau_budget_bytes : 0.0;
  // rebuild tiles: ~6% of the device, or, for a budgeted context (batches),
  // at most a quarter of its budget
  double tile_target = std::max(1.0e9, 0.06 * (double)totalb);
  if (has_budget)
    tile_target = std::min(tile_target, std::max(blk_tile_bytes, 0.25 * (double)d->tau_budget_bytes));
  if (mixed) {
    // the whole FP32 cache first; the FP64 cache gets what is left
    const double fbytes = 4.0 * 64 * nr * c->nblk;
    double cap = (double)freeb - reserve - tile_target;
    if (has_budget) cap = std::min(cap, budget_left);
    if (fbytes > cap)
      return fail(BSE_ENOMEM, "FP32 tau cache needs %.1f GB, %.1f GB free", fbytes / 1e9,
                  (double)freeb / 1e9);
    const auto ta = std::chrono::steady_clock::now();
    BSE_TRY(ctx_alloc_t(c, &c->tau_f, (size_t)c->nblk * 64 * nr));
    c->t_tau_alloc_ms += ms_since(ta);
    budget_left -= fbytes;
    BSE_TRY(mem_info(&freeb, &totalb));
  }
  bool full = false;
  if (d->tau_policy != BSE_TAU_REBUILD) {
    double cap = (double)freeb - reserve - small_tile * blk_tile_bytes;
    if (has_budget) cap = std::min(cap, budget_left);
    full = c->nblk * blk_bytes <= cap;
  }
  if (d->tau_policy == BSE_TAU_CACHE && !full)
    return fail(BSE_ENOMEM, "tau cache needs %.1f GB, %.1f GB free", c->nblk * blk_bytes / 1e9,
                (double)freeb / 1e9);
  if (full && has_budget) {
    c->tile_blk = small_tile;  // a budgeted context stays within its share
  } else if (full) {
    // device memory beyond the cache and the reserve goes to larger rebuild
    // tiles: the U vector rebuilds every block from the exciton
    const double spare = (double)freeb - reserve - c->nblk * blk_bytes;
    const double tb = std::min(tile_target, std::max(small_tile * blk_tile_bytes, spare));
    c->tile_blk = std::max(small_tile, std::min(c->nblk, (long)(tb / blk_tile_bytes)));
  } else {
    BSE_TRY(ensure_ygrid(c));  // accumulation across launches
    c->tile_blk = std::max(1L, std::min(c->nblk, (long)(tile_target / blk_tile_bytes)));
  }
  const long te = c->tile_blk * 64;
  BSE_TRY(ctx_alloc_t(c, &c->tile_grids, (size_t)c->tile_blk * 32 * nr));
  BSE_TRY(ctx_alloc_t(c, &c->rebuild_buf, (size_t)c->tile_blk * 64 * nr));
  if (c->npdep > 0) {
    BSE_TRY(ctx_alloc_t(c, &c->tile_RS, (size_t)te * npw));
    BSE_TRY(ctx_alloc_t(c, &c->tile_cmp, (size_t)c->tile_blk * 32 * npw));
    BSE_TRY(ctx_alloc_t(c, &c->tile_F, (size_t)te * npw));
    BSE_TRY(ctx_alloc_t(c, &c->tile_T, (size_t)te * c->npdep));
  }
  long ncache = 0;
  if (full) {
    ncache = c->nblk;
  } else if (d->tau_policy != BSE_TAU_REBUILD) {
    BSE_TRY(mem_info(&freeb, &totalb));
    double budget = (double)freeb - reserve;
    if (has_budget) budget = std::min(budget, budget_left);
    const long fit = budget > 0 ? (long)(budget / blk_bytes) : 0;
    ncache = std::min(fit, c->nblk);
  }
  c->nblk_cached = ncache;
  if (ncache > 0) {
    const auto ta = std::chrono::steady_clock::now();
    BSE_TRY(ctx_alloc_t(c, &c->tau_cache, (size_t)ncache * 64 * nr));
    c->t_tau_alloc_ms += ms_since(ta);
  }
  // one build feeds both caches: blocks below ncache go to the FP64 cache,
  // every block to the FP32 cache of a mixed context
  const long nbuild = mixed ? c->nblk : ncache;
  if (nbuild > 0) {
    PhaseScope ps(c, PH_INIT_TAU);
    for (long gb0 = 0; gb0 < nbuild;) {
      long nt = std::min(c->tile_blk, nbuild - gb0);
      if (gb0 < ncache) nt = std::min(nt, ncache - gb0);
      if (gb0 < ncache)
        BSE_TRY(tau_build_range(c, c->phik, gb0, nt, c->tau_cache, ncache, gb0, c->kmask,
                                c->tau_f));
      else
        BSE_TRY(tau_build_range_f(c, c->phik_f, gb0, nt, c->tau_f, c->nblk, gb0, c->kmask));
      gb0 += nt;
    }
  }
  if (c->nblk_cached == c->nblk && c->nblk > 0)
    c->tau_policy = BSE_TAU_CACHE;
  else if (need_k1d)
    c->tau_policy = (c->nblk_cached == 0) ? BSE_TAU_REBUILD : BSE_TAU_AUTO;
  return BSE_OK;
}


int init_impl(const bse_system_desc* d, bse_ctx* c) {
  BSE_TRY(validate(d));
  BSE_TRY(basis_build(d->cell, d->grid, d->ecut, &c->basis));
  const long npw = c->basis.npw, nr = c->basis.nr;
  if (d->n_val >= npw) return fail(BSE_EINVAL, "n_val %d must be below n_pw %ld", d->n_val, npw);
  if (d->n_pdep >= npw) return fail(BSE_EINVAL, "n_pdep %d must be below n_pw %ld", d->n_pdep, npw);
  if (d->n_orb > npw) return fail(BSE_EINVAL, "n_orb above n_pw");
  if (d->n_pdep > 0) {
    if (!finite_all(d->pdep, npw * d->n_pdep) || !finite_all(d->lambda, d->n_pdep))
      return fail(BSE_EINVAL, "non-finite PDEP data");
    for (int a = 0; a < d->n_pdep; ++a)
      if (!(d->lambda[a] < 1.0)) return fail(BSE_EINVAL, "lambda[%d] must be below 1", a);
  }
  if (d->n_orb > 0 && (!finite_all(d->orbitals, (long)d->n_orb * npw) || !finite_all(d->eps, d->n_orb)))
    return fail(BSE_EINVAL, "non-finite orbitals");
  c->st = (hipStream_t)d->stream;
  c->nv = d->n_val;
  c->nvh = (c->nv + 1) / 2;
  c->npdep = d->n_pdep;
  c->nsites = d->n_sites;
  c->kmask = d->kernel_mask ? d->kernel_mask : BSE_K_ALL;
  c->scissor = d->scissor;
  c->spin = d->spin_factor;
  c->gap_min = d->gap_min;
  c->gs_tol = d->gs_tol > 0 ? d->gs_tol : 1e-10;
  c->n_extra = d->n_extra;
  c->ks = d->ks_model;
  c->alpha = d->alpha_exx;
  if (d->rho_floor > 0) c->rho_floor = d->rho_floor;
  if (d->scf_tol > 0) c->scf_tol = d->scf_tol;
  // the device work starts here: record the device and its allocation-free
  // scratch address
  BSE_HIP(hipGetDevice(&c->dev));
  BSE_TRY(noalloc_setup(c->dev));
  BSE_TRY(fft_plan_init(&c->fft, d->grid));
  // basis maps and kinetic energy
  BSE_TRY(ctx_alloc_t(c, &c->idx_p, c->basis.nhalf + 1));
  BSE_TRY(ctx_alloc_t(c, &c->idx_m, c->basis.nhalf + 1));
  BSE_TRY(upload(c, c->idx_p, c->basis.idx_p.data(), sizeof(int) * c->basis.nhalf));
  BSE_TRY(upload(c, c->idx_m, c->basis.idx_m.data(), sizeof(int) * c->basis.nhalf));
  std::vector<double> T(npw);
  for (long j = 0; j < npw; ++j) T[j] = 0.5 * c->basis.g2[j];
  BSE_TRY(ctx_alloc_t(c, &c->T, npw));
  BSE_TRY(upload(c, c->T, T.data(), sizeof(double) * npw));
  c->map = SphereMap{c->idx_p, c->idx_m, c->basis.nhalf, (int)npw, nr, c->basis.omega, 0};
  BSE_TRY(sphere_plan_build(c->fft, c->basis, &c->sp));
  c->cmap = SphereMap{c->sp.e_plus, c->sp.e_minus, c->basis.nhalf, (int)npw, npw, c->basis.omega,
                      c->sp.e_zero};
  // sites, potential, Coulomb kernel
  const int ns = std::max(1, c->nsites);
  c->site_h.assign(5 * (size_t)ns, 0.0);
  for (int i = 0; i < c->nsites; ++i) {
    for (int a = 0; a < 3; ++a) c->site_h[3 * i + a] = d->site_xyz[3 * i + a];
    c->site_h[3 * c->nsites + i] = d->site_depth[i];
    c->site_h[4 * c->nsites + i] = d->site_width[i];
  }
  BSE_TRY(ctx_alloc_t(c, &c->sites, c->site_h.size()));
  BSE_TRY(upload(c, c->sites, c->site_h.data(), sizeof(double) * c->site_h.size()));
  {
    double2* vg = nullptr;
    BSE_TRY(ctx_alloc_t(c, &vg, nr));
    BSE_TRY(site_potential(c->sites, c->sites + 3 * c->nsites, c->sites + 4 * c->nsites,
                           c->nsites, c->basis.grid, c->basis.cell, vg, c->st));
    BSE_TRY(fft3d(c->fft, vg, 1, +1, c->st));
    BSE_TRY(ctx_alloc_t(c, &c->Vr, nr));
    BSE_TRY(real_part(vg, nr, c->Vr, c->st));
    BSE_HIP(hipStreamSynchronize(c->st));
    ctx_release(c, vg);
  }
  BSE_TRY(ctx_alloc_t(c, &c->vc, nr));
  BSE_TRY(coulomb_kernel(c->basis.grid, c->basis.cell, c->vc, c->st));
  if (c->ks) {  // V_ext kept apart: Vr becomes V_ext + V_H + V_xc
    BSE_TRY(ctx_alloc_t(c, &c->Vext, nr));
    BSE_TRY(ctx_alloc_t(c, &c->fxc, nr));
    BSE_TRY(ctx_alloc_t(c, &c->rho_ks, nr));
    BSE_HIP(hipMemcpyAsync(c->Vext, c->Vr, sizeof(double) * nr, hipMemcpyDeviceToDevice, c->st));
  }
  // PDEP: Pt = v_c^1/2 P, Ptc = v_c^1/2 P c
  if (c->npdep > 0) {
    std::vector<double> pt((size_t)npw * c->npdep), ptc((size_t)npw * c->npdep);
    for (long j = 0; j < npw; ++j) {
      const double vs = j == 0 ? 0.0 : std::sqrt(4.0 * M_PI / c->basis.g2[j]);
      for (int a = 0; a < c->npdep; ++a) {
        const double ca = d->lambda[a] / (1.0 - d->lambda[a]);
        const double x = vs * d->pdep[j * c->npdep + a];
        pt[(size_t)j * c->npdep + a] = x;
        ptc[(size_t)j * c->npdep + a] = x * ca;
      }
    }
    BSE_TRY(ctx_alloc_t(c, &c->Pt, pt.size()));
    BSE_TRY(ctx_alloc_t(c, &c->Ptc, ptc.size()));
    BSE_TRY(upload(c, c->Pt, pt.data(), sizeof(double) * pt.size()));
    BSE_TRY(upload(c, c->Ptc, ptc.data(), sizeof(double) * ptc.size()));
  }
  // occupied orbitals
  if (d->n_orb > 0) {
    c->norb = d->n_orb;
    BSE_TRY(ctx_alloc_t(c, &c->Phi, (size_t)c->norb * npw));
    BSE_TRY(ctx_alloc_t(c, &c->eps_d, (size_t)c->norb));
    BSE_TRY(upload(c, c->Phi, d->orbitals, sizeof(double) * c->norb * npw));
    BSE_TRY(upload(c, c->eps_d, d->eps, sizeof(double) * c->norb));
    c->eps_h.assign(d->eps, d->eps + c->norb);
  } else {
    const int extra = d->n_extra > 0 ? d->n_extra : 8;
    const int want = (int)std::min<long>(npw, (long)c->nv + extra);
    const auto t0 = std::chrono::steady_clock::now();
    if (c->ks)
      BSE_TRY(ks_ground_state(c, want));
    else
      BSE_TRY(ground_state(c, want, c->gs_tol));
    BSE_HIP(hipStreamSynchronize(c->st));
    c->t_gs_ms = ms_since(t0);
  }
  if (c->norb > c->nv) {
    c->ks_gap = c->eps_h[c->nv] - c->eps_h[c->nv - 1];
    if (c->gap_min > 0 && c->ks_gap < c->gap_min)
      return fail(BSE_EGAP, "Kohn-Sham gap %.3e Ha below gap_min %.3e", c->ks_gap, c->gap_min);
  }
  // phi(r)
  if (!c->phir) BSE_TRY(ctx_alloc_t(c, &c->phir, (size_t)c->nvh * nr));
  BSE_TRY(to_grid(c, c->Phi, c->nv, 1, c->phir));
  // orbitals supplied for the KS model: H_KS from their density
  if (c->ks && d->n_orb > 0) BSE_TRY(ks_potential_from_orbitals(c));
  // localised frame of the occupied-pair W integrals
  c->phik = c->phir;
  if (d->localize) {
    c->loc = 1;
    c->prune_thr = d->prune_threshold;
    BSE_TRY(localize(c, d));
    c->phik = c->phir_loc;
  }
  c->precision = d->precision;
  if (c->precision == BSE_MIXED) {  // FP32 copies of the real-space fields
    BSE_TRY(ctx_alloc_t(c, &c->phir_f, (size_t)c->nvh * nr));
    BSE_TRY(ctx_alloc_t(c, &c->Vr_f, (size_t)nr));
    BSE_TRY(ctx_alloc_t(c, &c->vc_f, (size_t)nr));
    BSE_TRY(to_f32((const double*)c->phir, (float*)c->phir_f, 2L * c->nvh * nr, c->st));
    BSE_TRY(to_f32(c->Vr, c->Vr_f, nr, c->st));
    BSE_TRY(to_f32(c->vc, c->vc_f, nr, c->st));
    // the FP32 tiles' PDEP projections as FP32 GEMMs (BSEX_PDEP_FP32=0: FP64)
    const char* e = getenv("BSEX_PDEP_FP32");
    if (c->npdep > 0 && !(e && atoi(e) == 0)) {
      const size_t n = (size_t)npw * c->npdep;
      BSE_TRY(ctx_alloc_t(c, &c->Pt_f, n));
      BSE_TRY(ctx_alloc_t(c, &c->Ptc_f, n));
      BSE_TRY(to_f32(c->Pt, c->Pt_f, (long)n, c->st));
      BSE_TRY(to_f32(c->Ptc, c->Ptc_f, (long)n, c->st));
    }
    if (c->loc) {
      BSE_TRY(ctx_alloc_t(c, &c->phir_loc_f, (size_t)c->nvh * nr));
      BSE_TRY(to_f32((const double*)c->phir_loc, (float*)c->phir_loc_f, 2L * c->nvh * nr, c->st));
    }
  }
  c->phik_f = c->loc ? c->phir_loc_f : c->phir_f;
  BSE_HIP(hipStreamSynchronize(c->st));
  const auto t1 = std::chrono::steady_clock::now();
  BSE_TRY(plan_tau(c, d));
  c->active = c->precision;
  BSE_HIP(hipStreamSynchronize(c->st));
  c->t_tau_ms = ms_since(t1);
  return BSE_OK;
}

template <typename F>
int guarded(bse_ctx* c, F f) {
  try {
    int rc = f();
    if (c) {
      int rc2 = prof_collect(c);
      if (rc == BSE_OK) rc = rc2;
    }
    return rc;
  } catch (const std::bad_alloc&) {
    return fail(BSE_ENOMEM, "host allocation failed");
  } catch (...) {
    return fail(BSE_EINVAL, "unexpected exception");
  }
}

}  // namespace

extern "C" {

int32_t bse_abi_version(void) { return BSEX_ABI_VERSION; }

const char* bse_last_error(void) { return last_error(); }

int bse_warm_up(void) {
  double* p = nullptr;
  BSE_HIP(hipMalloc(&p, 256));
  int rc = zero_fill(p, 32, nullptr);
  if (rc == BSE_OK && hipStreamSynchronize(nullptr) != hipSuccess)
    rc = fail(BSE_EHIP, "warm-up launch failed");
  (void)hipFree(p);
  return rc;
}

int bse_basis_size(const double cell[3], const int32_t grid[3], double ecut, int32_t* n_pw) {
  if (!cell || !grid || !n_pw) return fail(BSE_EINVAL, "NULL argument");
  Basis b;
  const int g[3] = {grid[0], grid[1], grid[2]};
  BSE_TRY(basis_build(cell, g, ecut, &b));
  *n_pw = b.npw;
  return BSE_OK;
}

int bse_basis_gvectors(const double cell[3], const int32_t grid[3], double ecut,
                       int32_t* miller_host, int8_t* kind_host) {
  if (!cell || !grid) return fail(BSE_EINVAL, "NULL argument");
  Basis b;
  const int g[3] = {grid[0], grid[1], grid[2]};
  BSE_TRY(basis_build(cell, g, ecut, &b));
  if (miller_host) {
    for (int a = 0; a < 3; ++a) miller_host[a] = 0;
    for (int s = 0; s < b.nhalf; ++s)
      for (int q = 0; q < 2; ++q)
        for (int a = 0; a < 3; ++a) miller_host[3 * (1 + 2 * s + q) + a] = b.mill_half[3 * s + a];
  }
  if (kind_host) {
    kind_host[0] = 0;
    for (int s = 0; s < b.nhalf; ++s) {
      kind_host[1 + 2 * s] = 1;
      kind_host[2 + 2 * s] = 2;
    }
  }
  return BSE_OK;
}

int bse_init_system(const bse_system_desc* desc, bse_ctx** out) {
  if (!out) return fail(BSE_EINVAL, "out is NULL");
  *out = nullptr;
  bse_ctx* c = nullptr;
  try {
    c = new bse_ctx();
  } catch (...) {
    return fail(BSE_ENOMEM, "host allocation failed");
  }
  const auto t0 = std::chrono::steady_clock::now();
  int rc = guarded(nullptr, [&] { return init_impl(desc, c); });
  c->t_init_ms = ms_since(t0);
  if (rc != BSE_OK) {
    std::string keep = last_error();
    ctx_destroy(c);
    set_error("%s", keep.c_str());
    return rc;
  }
  *out = c;
  return BSE_OK;
}

int bse_get_info(bse_ctx* c, bse_info* info) {
  if (!c || !info) return fail(BSE_EINVAL, "NULL argument");
  info->n_pw = c->basis.npw;
  info->n_val = c->nv;
  info->n_pdep = c->npdep;
  info->n_orb = c->norb;
  for (int a = 0; a < 3; ++a) info->grid[a] = c->basis.grid[a];
  info->tau_policy = c->tau_policy;
  info->tau_blocks = c->nblk;
  info->tau_blocks_cached = c->nblk_cached;
  info->tau_bytes = (int64_t)c->nblk_cached * 64 * c->basis.nr * 8;
  info->precision = c->precision;
  info->active_precision = c->active;
  info->tau_bytes_f32 = c->tau_f ? (int64_t)c->nblk * 64 * c->basis.nr * 4 : 0;
  info->gs_resid = c->gs_resid;
  info->ks_gap = c->ks_gap;
  info->gs_sweeps = c->gs_sweeps;
  info->t_ground_state_ms = c->t_gs_ms;
  info->t_tau_ms = c->t_tau_ms;
  info->t_tau_alloc_ms = c->t_tau_alloc_ms;
  info->t_init_ms = c->t_init_ms;
  info->scf_iters = c->scf_iters;
  info->scf_resid = c->ks ? c->scf_resid : -1.0;
  info->tau_blocks_all = c->nblk_all;
  info->loc_spread = c->loc ? c->loc_spread : -1.0;
  info->loc_sweeps = c->loc_sweeps;
  return BSE_OK;
}

int bse_get_frame(bse_ctx* c, double* U_host, double* centres_host) {
  if (!c) return fail(BSE_EINVAL, "ctx is NULL");
  if (!c->loc) return fail(BSE_ESTATE, "the context has no localised frame");
  if (U_host) std::copy(c->loc_U_h.begin(), c->loc_U_h.end(), U_host);
  if (centres_host) std::copy(c->loc_cen_h.begin(), c->loc_cen_h.end(), centres_host);
  return BSE_OK;
}

int bse_get_orbitals(bse_ctx* c, int32_t n, double* orbitals_dev, double* eps_host) {
  if (!c) return fail(BSE_EINVAL, "ctx is NULL");
  if (n < 1 || n > c->norb) return fail(BSE_EINVAL, "n must be in 1..%d", c->norb);
  return guarded(c, [&]() -> int {
    if (orbitals_dev) {
      BSE_HIP(hipMemcpyAsync(orbitals_dev, c->Phi, sizeof(double) * n * c->basis.npw,
                             hipMemcpyDeviceToDevice, c->st));
      BSE_HIP(hipStreamSynchronize(c->st));
    }
    if (eps_host) std::copy(c->eps_h.begin(), c->eps_h.begin() + n, eps_host);
    return BSE_OK;
  });
}

int bse_apply(bse_ctx* c, int32_t n_b, const double* X, double* Y) {
  if (!c) return fail(BSE_EINVAL, "ctx is NULL");
  if (n_b < 0) return fail(BSE_EINVAL, "n_b < 0");
  if (n_b == 0) return BSE_OK;
  if (!X || !Y) return fail(BSE_EINVAL, "NULL vector");
  const size_t bytes = sizeof(double) * (size_t)n_b * c->nv * c->basis.npw;
  const char* xa = (const char*)X;
  const char* ya = (const char*)Y;
  if (xa < ya + bytes && ya < xa + bytes) return fail(BSE_EINVAL, "X and Y overlap");
  return guarded(c, [&]() -> int {
    const long L = (long)c->nv * c->basis.npw;
    for (long i = 0; i < n_b; i += c->nbc) {
      const int k = (int)std::min<long>(c->nbc, n_b - i);
      if (c->use_graph && !c->prof)
        BSE_TRY(graph_apply(c, k, X + i * L, Y + i * L));
      else
        BSE_TRY(apply_any(c, k, X + i * L, Y + i * L));
    }
    BSE_HIP(hipStreamSynchronize(c->st));
    return BSE_OK;
  });
}

int bse_set_precision(bse_ctx* c, int32_t precision) {
  if (!c) return fail(BSE_EINVAL, "ctx is NULL");
  if (precision != BSE_FP64 && precision != BSE_MIXED)
    return fail(BSE_EINVAL, "precision %d unknown", precision);
  if (precision == BSE_MIXED && c->precision != BSE_MIXED)
    return fail(BSE_ESTATE, "context was built without BSE_MIXED");
  c->active = precision;
  return BSE_OK;
}

int bse_set_graphs(bse_ctx* c, int32_t on) {
  if (!c) return fail(BSE_EINVAL, "ctx is NULL");
  if (!on) graphs_destroy(c);
  c->use_graph = on != 0;
  return BSE_OK;
}

int bse_set_learned(bse_ctx* c, bse_mlp* mlp) {
  if (!c) return fail(BSE_EINVAL, "ctx is NULL");
  if (mlp && (mlp_n_in(mlp) != BSE_LEARN_NFEAT || mlp_n_out(mlp) != BSE_LEARN_NOUT))
    return fail(BSE_EINVAL, "network must map %d features to %d outputs", BSE_LEARN_NFEAT,
                BSE_LEARN_NOUT);
  c->learned = mlp;
  return BSE_OK;
}

int bse_learned_features(bse_ctx* c, const double* Xs, const double* Zref, int32_t two_level,
                         float* feat, double* gamma) {
  if (!c || !Xs || !feat) return fail(BSE_EINVAL, "NULL argument");
  if (Zref && !gamma) return fail(BSE_EINVAL, "gamma_host needed with Zref_dev");
  return guarded(c, [&] { return learned_targets(c, Xs, Zref, two_level != 0, feat, gamma); });
}

int bse_davidson(bse_ctx* c, int32_t n_states, const bse_solver_opts* opts, double* omega_host,
                 double* X_dev, bse_solver_stats* stats) {
  if (!c || !omega_host) return fail(BSE_EINVAL, "NULL argument");
  if (n_states < 1 || n_states > 16) return fail(BSE_EINVAL, "n_states must be 1..16");
  if (opts && opts->block > 0 && opts->block < n_states)
    return fail(BSE_EINVAL, "block below n_states");
  return guarded(c, [&] { return davidson(c, n_states, opts, omega_host, X_dev, stats); });
}

int bse_apply_coupling(bse_ctx* c, int32_t n_b, const double* X_dev, double* Y_dev) {
  if (!c) return fail(BSE_EINVAL, "ctx is NULL");
  if (n_b < 0) return fail(BSE_EINVAL, "n_b < 0");
  if (n_b == 0) return BSE_OK;
  if (!X_dev || !Y_dev) return fail(BSE_EINVAL, "NULL argument");
  if (c->ks) return fail(BSE_EINVAL, "the coupling beyond the TDA needs ks_model 0");
  return guarded(c, [&]() -> int {
    BSE_TRY(ensure_apply_work(c, std::min(n_b, 8)));
    BSE_TRY(apply_coupling(c, n_b, X_dev, Y_dev));
    BSE_HIP(hipStreamSynchronize(c->st));
    return BSE_OK;
  });
}

int bse_full_bse(bse_ctx* c, int32_t n_states, const bse_solver_opts* opts, double* omega_host,
                 double* X_dev, double* Y_dev, bse_solver_stats* stats) {
  if (!c || !omega_host) return fail(BSE_EINVAL, "NULL argument");
  if (n_states < 1 || n_states > 16) return fail(BSE_EINVAL, "n_states must be 1..16");
  if (opts && opts->block > 0 && opts->block < n_states)
    return fail(BSE_EINVAL, "block below n_states");
  if (c->ks) return fail(BSE_EINVAL, "the coupling beyond the TDA needs ks_model 0");
  return guarded(c, [&] { return full_bse(c, n_states, opts, omega_host, X_dev, Y_dev, stats); });
}

int bse_u_vector(bse_ctx* c, const double* Xs, double* U) {
  if (!c || !Xs || !U) return fail(BSE_EINVAL, "NULL argument");
  return guarded(c, [&] { return u_vector(c, Xs, U); });
}

int bse_zvector_solve(bse_ctx* c, const double* Xs, const bse_solver_opts* opts, double* Z,
                      bse_solver_stats* stats) {
  if (!c || !Xs || !Z) return fail(BSE_EINVAL, "NULL argument");
  return guarded(c, [&] { return zvector(c, Xs, opts, Z, stats); });
}

int bse_forces(bse_ctx* c, const double* Xs, const double* Z, double* dwdR_host) {
  if (!c || !Xs || !Z || (!dwdR_host && c->nsites > 0)) return fail(BSE_EINVAL, "NULL argument");
  return guarded(c, [&] { return forces(c, Xs, Z, dwdR_host); });
}

int bse_ground_state_forces(bse_ctx* c, double* dEdR_host) {
  if (!c || (!dEdR_host && c->nsites > 0)) return fail(BSE_EINVAL, "NULL argument");
  return guarded(c, [&] { return ground_state_forces(c, dEdR_host); });
}

int bse_set_profiling(bse_ctx* c, int32_t on) {
  if (!c) return fail(BSE_EINVAL, "ctx is NULL");
  c->prof = on != 0;
  return BSE_OK;
}

int bse_get_phase_times(bse_ctx* c, bse_phase_times* out, int32_t reset) {
  if (!c || !out) return fail(BSE_EINVAL, "NULL argument");
  static const char* names[PH_COUNT] = {"proj",      "fft_inv", "k1e",    "tau_stream",
                                        "tau_tile",  "tau_build", "combine", "fft_fwd",
                                        "solver",    "init_tau",  "ground_state"};
  out->n_phase = PH_COUNT;
  for (int i = 0; i < PH_COUNT; ++i) {
    out->name[i] = names[i];
    out->ms[i] = c->ph_ms[i];
    out->count[i] = c->ph_n[i];
    if (reset) {
      c->ph_ms[i] = 0;
      c->ph_n[i] = 0;
    }
  }
  return BSE_OK;
}

int bse_free(bse_ctx* c) {
  if (!c) return BSE_OK;
  ctx_destroy(c);
  return BSE_OK;
}

int bse_memory_cache(int32_t on) { return memory_cache(on); }

}  // extern "C"
