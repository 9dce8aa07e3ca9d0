// The DMPT BSE operator on the device: projector, transforms, K1e, tau
// build and stream, combine, diagonal term (Eqs. 1-3).
#include <algorithm>
#include <mutex>
#include <cmath>

#include "context.h"

namespace bsex {

// ---------------------------------------------------------------------------
// allocation and profiling helpers
// ---------------------------------------------------------------------------
// Device memory of a context.  Released blocks go to a per-context cache and
// are handed out again (smallest block that fits, at most twice the request),
// so the solvers' scratch does not call hipMalloc/hipFree in steady state:
// hipFree waits for the whole device, which would serialise the streams of a
// batch.  Blocks are reused on the context's own stream only, so stream order
// keeps every earlier use of a block ahead of its next one.  The cache is
// returned to the device when an allocation fails, and at bse_free.
//
// Across contexts (bse_memory_cache): with the cache on, a context's blocks
// go at bse_free to a process-wide cache (after its stream has drained),
// and later contexts on the same device take their blocks from it before
// calling hipMalloc.  A run that builds one context per geometry then
// reuses the same memory instead of freeing and allocating ~10^11 bytes
// per geometry (a fresh allocation of memory the device has just freed
// can wait seconds while the driver clears it).
namespace {
std::mutex g_cache_mu;
struct CachedBuf {
  DevBuf b;
  int dev;
};
std::vector<CachedBuf> g_cache;
bool g_keep = false;

int cur_dev() {
  int d = 0;
  (void)hipGetDevice(&d);
  return d;
}

// best fit (at most twice the request) among blocks of `v`
template <class V, class Get>
long best_fit(const V& v, size_t bytes, Get get) {
  long best = -1;
  for (size_t i = 0; i < v.size(); ++i) {
    const size_t b = get(v[i]).bytes;
    if (b >= bytes && b <= 2 * bytes + (1u << 20) &&
        (best < 0 || b < get(v[(size_t)best]).bytes))
      best = (long)i;
  }
  return best;
}

bool cache_take(size_t bytes, DevBuf* out) {
  std::lock_guard<std::mutex> lk(g_cache_mu);
  if (g_cache.empty()) return false;
  const int dev = cur_dev();
  long best = -1;
  for (size_t i = 0; i < g_cache.size(); ++i) {
    const size_t b = g_cache[i].b.bytes;
    if (g_cache[i].dev == dev && b >= bytes && b <= 2 * bytes + (1u << 20) &&
        (best < 0 || b < g_cache[(size_t)best].b.bytes))
      best = (long)i;
  }
  if (best < 0) return false;
  *out = g_cache[(size_t)best].b;
  g_cache.erase(g_cache.begin() + best);
  return true;
}

// return this device's cached blocks to the device
void cache_flush_dev() {
  std::lock_guard<std::mutex> lk(g_cache_mu);
  const int dev = cur_dev();
  std::vector<CachedBuf> keep;
  for (auto& cb : g_cache) {
    if (cb.dev == dev)
      (void)hipFree(cb.b.p);
    else
      keep.push_back(cb);
  }
  g_cache.swap(keep);
}
}  // namespace

int mem_info(size_t* freeb, size_t* totalb) {
  BSE_HIP(hipMemGetInfo(freeb, totalb));
  std::lock_guard<std::mutex> lk(g_cache_mu);
  const int dev = cur_dev();
  for (auto& cb : g_cache)
    if (cb.dev == dev) *freeb += cb.b.bytes;
  return BSE_OK;
}

bool cache_keeps() {
  std::lock_guard<std::mutex> lk(g_cache_mu);
  return g_keep;
}

void cache_put(const DevBuf& b) {
  std::lock_guard<std::mutex> lk(g_cache_mu);
  g_cache.push_back(CachedBuf{b, cur_dev()});
}

int memory_cache(int on) {
  {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    g_keep = on != 0;
  }
  if (!on) {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    for (auto& cb : g_cache) (void)hipFree(cb.b.p);
    g_cache.clear();
  }
  return BSE_OK;
}

int ctx_alloc(bse_ctx* c, void** p, size_t bytes) {
  *p = nullptr;
  if (bytes == 0) bytes = 16;
  const long best = best_fit(c->pool, bytes, [](const DevBuf& d) -> const DevBuf& { return d; });
  if (best >= 0) {
    const DevBuf d = c->pool[(size_t)best];
    c->pool.erase(c->pool.begin() + best);
    c->allocs.push_back(d);
    *p = d.p;
    return BSE_OK;
  }
  DevBuf cd;
  if (cache_take(bytes, &cd)) {
    c->allocs.push_back(cd);
    *p = cd.p;
    return BSE_OK;
  }
  void* q = nullptr;
  hipError_t e = hipMalloc(&q, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    if (c->st) (void)hipStreamSynchronize(c->st);
    for (auto& b : c->pool) (void)hipFree(b.p);
    c->pool.clear();
    cache_flush_dev();
    e = hipMalloc(&q, bytes);
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(BSE_ENOMEM, "device allocation of %zu bytes failed (%s)", bytes,
                hipGetErrorString(e));
  }
  c->allocs.push_back(DevBuf{q, bytes});
  *p = q;
  return BSE_OK;
}

void ctx_pool_flush(bse_ctx* c) {
  if (c->pool.empty()) return;
  if (c->st) (void)hipStreamSynchronize(c->st);
  for (auto& b : c->pool) (void)hipFree(b.p);
  c->pool.clear();
}

void ctx_release(bse_ctx* c, void* p) {
  if (!p) return;
  if (!c->graphs.empty() &&
      std::find(c->graph_bufs.begin(), c->graph_bufs.end(), p) != c->graph_bufs.end())
    graphs_destroy(c);
  for (size_t i = 0; i < c->allocs.size(); ++i)
    if (c->allocs[i].p == p) {
      c->pool.push_back(c->allocs[i]);
      c->allocs.erase(c->allocs.begin() + i);
      return;
    }
}

static hipEvent_t ev_get(bse_ctx* c) {
  if (c->ev_used < c->ev_pool.size()) return c->ev_pool[c->ev_used++];
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  c->ev_pool.push_back(e);
  ++c->ev_used;
  return e;
}

PhaseScope::PhaseScope(bse_ctx* c_, int ph_) : c(c_), ph(ph_) {
  if (!c->prof) return;
  e1 = ev_get(c);
  if (e1) (void)hipEventRecord(e1, c->st);
}

PhaseScope::~PhaseScope() {
  if (!c->prof || !e1) return;
  hipEvent_t e2 = ev_get(c);
  if (!e2) return;
  (void)hipEventRecord(e2, c->st);
  c->ev_open.push_back({ph, {e1, e2}});
}

int prof_collect(bse_ctx* c) {
  if (c->ev_open.empty()) {
    c->ev_used = 0;
    return BSE_OK;
  }
  BSE_HIP(hipStreamSynchronize(c->st));
  for (auto& o : c->ev_open) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, o.second.first, o.second.second) == hipSuccess) {
      c->ph_ms[o.first] += ms;
      c->ph_n[o.first] += 1;
    }
  }
  c->ev_open.clear();
  c->ev_used = 0;
  return BSE_OK;
}

// ---------------------------------------------------------------------------
// projector P_c = 1 - sum_v |phi_v><phi_v| on nset sets of nv orbitals
// ---------------------------------------------------------------------------
static int ensure_ov(bse_ctx* c, int nset) {
  const size_t need = (size_t)c->nv * c->nv * nset;
  static_assert(sizeof(double) == 8, "");
  for (auto& b : c->allocs)
    if (b.p == c->Ov && b.bytes >= need * sizeof(double)) return BSE_OK;
  ctx_release(c, c->Ov);
  c->Ov = nullptr;
  return ctx_alloc_t(c, &c->Ov, need);
}

// GEMM with a context-owned split-K workspace
int gemm(bse_ctx* c, int ta, int tb, long M, long N, long K, double alpha, const double* A,
         long lda, const double* B, long ldb, double beta, double* C, long ldc) {
  const long need = dgemm_work(M, N, K);
  if (need > c->gw_len) {
    ctx_release(c, c->gw);
    c->gw = nullptr;
    c->gw_len = 0;
    BSE_TRY(ctx_alloc_t(c, &c->gw, (size_t)need));
    c->gw_len = need;
  }
  return dgemm_ws(ta, tb, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, c->gw, c->gw_len, c->st);
}

int proj_c(bse_ctx* c, const double* X, double* Y, int nset) {
  if (nset <= 0) return BSE_OK;
  PhaseScope ps(c, PH_PROJ);
  BSE_TRY(ensure_ov(c, nset));
  const long npw = c->basis.npw, nv = c->nv, n = (long)nset * nv;
  // Ov[w][(s,v)] = <phi_w | x_{s,v}>
  BSE_TRY(gemm(c, 0, 1, nv, n, npw, 1.0, c->Phi, npw, X, npw, 0.0, c->Ov, n));
  // Y = X - Ov^T Phi (the GEMM reads X as its C input: no copy when Y != X)
  BSE_TRY(dgemm_from(1, 0, n, npw, nv, -1.0, c->Ov, n, c->Phi, npw, 1.0, Y != X ? X : nullptr, Y,
                     npw, c->st));
  return BSE_OK;
}

// grid values of nset sets of nvs orbitals (two orbitals per complex grid)
int to_grid(bse_ctx* c, const double* X, int nvs, int nset, double2* grids) {
  PhaseScope ps(c, PH_FFT_INV);
  return sphere_to_grid(c->fft, c->sp, c->basis.omega, X, nvs, nset, grids, c->st);
}

static int ensure_compact(bse_ctx* c, long ngrids) {
  if (c->compact_grids >= ngrids) return BSE_OK;
  ctx_release(c, c->compact);
  c->compact = nullptr;
  c->compact_grids = 0;
  BSE_TRY(ctx_alloc_t(c, &c->compact, (size_t)ngrids * c->basis.npw));
  c->compact_grids = ngrids;
  return BSE_OK;
}

int from_grid(bse_ctx* c, double2* grids, int nvs, int nset, const double* A, const double* eps,
              double shift, double* Y) {
  PhaseScope ps(c, PH_FFT_FWD);
  const long ng = (long)nset * ((nvs + 1) / 2);
  BSE_TRY(ensure_compact(c, ng));
  BSE_TRY(grid_to_compact(c->fft, c->sp, grids, ng, c->compact, c->st));
  return gather_sets(c->cmap, c->compact, nvs, nset, 1.0 / (double)c->basis.nr, A, c->T, eps,
                     shift, 0.0, Y, c->st);
}

// Y = (T + shift - eps_v) X + <e| V(r) x(r)> on nset sets of nvs orbitals
// (eps indexed by position in the set, NULL for none), optionally projected
// by P_c (then nvs must be c->nv).
int apply_H(bse_ctx* c, int nvs, int nset, const double* X, double* Y, double2* grids,
            double shift, const double* eps, int project) {
  BSE_TRY(to_grid(c, X, nvs, nset, grids));
  const long ng = (long)nset * ((nvs + 1) / 2);
  {
    PhaseScope ps(c, PH_COMBINE);
    BSE_TRY(mul_real_field(grids, ng, c->basis.nr, c->Vr, 1.0, c->st));
  }
  BSE_TRY(from_grid(c, grids, nvs, nset, X, eps, shift, Y));
  if (project) BSE_TRY(proj_c(c, Y, Y, nset));
  return BSE_OK;
}

// ---------------------------------------------------------------------------
// tau_{vv'} = W(orb_v orb_v') for the 8x8 blocks [gb0, gb0 + nblk)
//   bare part: v_c(G) on every grid frequency; PDEP part (Eq. 3):
//   sum_j e_j [V^1/2 P C P^T V^1/2 rho_S]_j  via two GEMMs per tile.
// ---------------------------------------------------------------------------
// the forward transform of a W build with the bare Coulomb multiply (or the
// zero fill) fused into its last pass and the PDEP projection's sphere
// entries taken there (fft3d_fwd_w); BSEX_W_FUSED=0 selects the separate
// transform, gather and multiply kernels
static bool w_fused_on() {
  static const bool on = [] {
    const char* e = getenv("BSEX_W_FUSED");
    return !e || atoi(e) != 0;
  }();
  return on;
}
// ... and with the pair products formed in its first pass (fft3d_fwd_pairs)
// where the axis-1 length allows; BSEX_W_PAIRS=0 keeps the pair-density kernel
static bool w_pairs_on(const bse_ctx* c, bool f32) {
  static const bool on = [] {
    const char* e = getenv("BSEX_W_PAIRS");
    return !e || atoi(e) != 0;
  }();
  return on && w_fused_on() && fwd_pairs_supported(c->fft, f32);
}

int tau_build_range(bse_ctx* c, const double2* orbr, long gb0, long nblk, double* dst,
                    long dst_nblk, long dst_blk0, int mask, float* dstf) {
  if (nblk <= 0) return BSE_OK;
  if (nblk > c->tile_blk) return fail(BSE_EINVAL, "tau build: tile of %ld blocks too large", nblk);
  const long nr = c->basis.nr, npw = c->basis.npw;
  const long ng = nblk * 32, ne = nblk * 64;
  SphereMap m64 = c->map;
  const bool pdep = (mask & BSE_K_1D_PDEP) && c->npdep > 0;
  const bool bare = (mask & BSE_K_1D_BARE) != 0;
  const bool fused = w_fused_on();
  // the grids leave the forward transform times v_c / N_r, their sphere
  // entries in tile_cmp
  if (w_pairs_on(c, false)) {
    BSE_TRY(fft3d_fwd_pairs(c->fft, c->sp, orbr, c->nv, c->blkIJ + gb0, nblk, c->tile_grids,
                            bare ? c->vc : nullptr, 1.0 / (double)nr,
                            pdep ? c->tile_cmp : nullptr, c->st));
  } else {
    BSE_TRY(pair_density(orbr, c->nv, c->blkIJ + gb0, nblk, nr, c->tile_grids, c->st));
    if (fused)
      BSE_TRY(fft3d_fwd_w(c->fft, c->sp, c->tile_grids, ng, bare ? c->vc : nullptr,
                          1.0 / (double)nr, pdep ? c->tile_cmp : nullptr, c->st));
    else
      BSE_TRY(fft3d(c->fft, c->tile_grids, ng, -1, c->st));
  }
  if (pdep) {
    // rho_S[e][j] = <e_j | rho_e>
    BSE_TRY(gather_sets(fused ? c->cmap : m64, fused ? c->tile_cmp : c->tile_grids, 64,
                        (int)nblk, 1.0 / (double)nr, nullptr, nullptr, nullptr, 0.0, 0.0,
                        c->tile_RS, c->st));
    BSE_TRY(gemm(c, 0, 0, ne, c->npdep, npw, 1.0, c->tile_RS, npw, c->Pt, c->npdep, 0.0,
                 c->tile_T, c->npdep));
    BSE_TRY(dgemm(0, 1, ne, npw, c->npdep, 1.0, c->tile_T, c->npdep, c->Ptc, c->npdep, 0.0,
                  c->tile_F, npw, c->st));
  }
  if (!fused && bare)
    BSE_TRY(mul_real_field(c->tile_grids, ng, nr, c->vc, 1.0 / (double)nr, c->st));
  else if (!fused)  // a fill kernel, not a memset: this may run inside a captured graph
    BSE_TRY(zero_fill(reinterpret_cast<double*>(c->tile_grids), 2 * ng * nr, c->st));
  if (pdep) BSE_TRY(scatter_sets(m64, c->tile_F, 64, (int)nblk, c->tile_grids, 1, c->st));
  BSE_TRY(fft3d(c->fft, c->tile_grids, ng, +1, c->st));
  if (dstf)
    BSE_TRY(tau_store(c->tile_grids, c->blkIJ + gb0, nblk, nr, c->Rf, dstf, c->nblk, gb0, c->st));
  if (dst)
    BSE_TRY(tau_store(c->tile_grids, c->blkIJ + gb0, nblk, nr, c->R, dst, dst_nblk, dst_blk0,
                      c->st));
  return BSE_OK;
}

// The same tile in FP32 (mixed contexts): pair densities, transforms, the
// bare Coulomb kernel and the stored tile in FP32; the PDEP projections and
// their GEMMs in FP64.  The tile grids and dst are the FP64 buffers'
// storage reused at half the size.
int tau_build_range_f(bse_ctx* c, const float2* orbr, long gb0, long nblk, float* dst,
                      long dst_nblk, long dst_blk0, int mask) {
  if (nblk <= 0) return BSE_OK;
  if (nblk > c->tile_blk) return fail(BSE_EINVAL, "tau build: tile of %ld blocks too large", nblk);
  const long nr = c->basis.nr, npw = c->basis.npw;
  const long ng = nblk * 32, ne = nblk * 64;
  float2* tg = reinterpret_cast<float2*>(c->tile_grids);
  SphereMap m64 = c->map;
  const bool pdep = (mask & BSE_K_1D_PDEP) && c->npdep > 0;
  const bool bare = (mask & BSE_K_1D_BARE) != 0;
  const bool fused = w_fused_on();
  float2* cmp = reinterpret_cast<float2*>(c->tile_cmp);
  if (w_pairs_on(c, true)) {
    BSE_TRY(fft3d_fwd_pairs(c->fft, c->sp, orbr, c->nv, c->blkIJ + gb0, nblk, tg,
                            bare ? c->vc_f : nullptr, 1.0f / (float)nr, pdep ? cmp : nullptr,
                            c->st));
  } else {
    BSE_TRY(pair_density(orbr, c->nv, c->blkIJ + gb0, nblk, nr, tg, c->st));
    if (fused)
      BSE_TRY(fft3d_fwd_w(c->fft, c->sp, tg, ng, bare ? c->vc_f : nullptr, 1.0f / (float)nr,
                          pdep ? cmp : nullptr, c->st));
    else
      BSE_TRY(fft3d(c->fft, tg, ng, -1, c->st));
  }
  const SphereMap& mg = fused ? c->cmap : m64;
  const float2* src = fused ? cmp : tg;
  // PDEP part (Eq. 3) in FP32 when the context holds FP32 copies of the
  // basis (the tile buffers hold twice the floats needed), else FP64
  const bool f32 = pdep && c->Pt_f;
  float* rs = reinterpret_cast<float*>(c->tile_RS);
  float* tt = reinterpret_cast<float*>(c->tile_T);
  float* tf = reinterpret_cast<float*>(c->tile_F);
  if (f32) {
    BSE_TRY(gather_sets(mg, src, 64, (int)nblk, 1.0 / (double)nr, rs, c->st));
    BSE_TRY(sgemm(0, 0, ne, c->npdep, npw, 1.0f, rs, npw, c->Pt_f, c->npdep, 0.0f, tt,
                  c->npdep, c->st));
    BSE_TRY(sgemm(0, 1, ne, npw, c->npdep, 1.0f, tt, c->npdep, c->Ptc_f, c->npdep, 0.0f, tf,
                  npw, c->st));
  } else if (pdep) {
    BSE_TRY(gather_sets(mg, src, 64, (int)nblk, 1.0 / (double)nr, nullptr, nullptr, nullptr, 0.0,
                        0.0, c->tile_RS, c->st));
    BSE_TRY(gemm(c, 0, 0, ne, c->npdep, npw, 1.0, c->tile_RS, npw, c->Pt, c->npdep, 0.0,
                 c->tile_T, c->npdep));
    BSE_TRY(dgemm(0, 1, ne, npw, c->npdep, 1.0, c->tile_T, c->npdep, c->Ptc, c->npdep, 0.0,
                  c->tile_F, npw, c->st));
  }
  if (!fused && bare)
    BSE_TRY(mul_real_field(tg, ng, nr, c->vc_f, 1.0f / (float)nr, c->st));
  else if (!fused)  // one float2 per double
    BSE_TRY(zero_fill(reinterpret_cast<double*>(tg), ng * nr, c->st));
  if (f32)
    BSE_TRY(scatter_sets(m64, tf, 64, (int)nblk, tg, 1, c->st));
  else if (pdep)
    BSE_TRY(scatter_sets(m64, c->tile_F, 64, (int)nblk, tg, 1, c->st));
  BSE_TRY(fft3d(c->fft, tg, ng, +1, c->st));
  return tau_store(tg, c->blkIJ + gb0, nblk, nr, c->Rf, dst, dst_nblk, dst_blk0, c->st);
}

// band rows [row0, row0 + rows) that blocks [gb0, gb0 + nt) of the block list
// touch: a launch that accumulates into y stages only those
static void tile_rows(const bse_ctx* c, long gb0, long nt, int* row0, int* rows) {
  int imin = c->blkIJ_h[gb0].x, jmax = 0;
  for (long k = gb0; k < gb0 + nt; ++k) {
    imin = std::min(imin, c->blkIJ_h[k].x);
    jmax = std::max(jmax, c->blkIJ_h[k].y);
  }
  *row0 = 8 * imin;
  *rows = 8 * (jmax + 1) - *row0;
}

// y[b][v] = sum_v' tau_{vv'} a[b][v'] over all pairs: cached blocks, then
// tiles rebuilt on the fly.  orbr are the orbitals tau is built from.
static int tau_contract(bse_ctx* c, const double2* orbr, const double2* a, double2* y, int nb,
                        int mask, bool use_cache, const FuseArgs* fuse = nullptr) {
  int first = 1;
  const long nr = c->basis.nr;
  long start = 0;
  if (fuse && !(use_cache && c->nblk_cached == c->nblk))
    return fail(BSE_EINVAL, "fused tau stream needs the whole cache");
  if (use_cache && c->nblk_cached > 0) {
    PhaseScope ps(c, PH_TAU_STREAM);
    BSE_TRY(tau_stream(c->tau_cache, c->nblk_cached, c->nblk_cached, c->blkIJ, c->R, a, y, nb,
                       c->nv, nr, 0, c->max_lds, c->st, fuse, c->tau_bl));
    first = 0;
    start = c->nblk_cached;
  }
  for (long gb0 = start; gb0 < c->nblk; gb0 += c->tile_blk) {
    const long nt = std::min(c->tile_blk, c->nblk - gb0);
    {
      PhaseScope ps(c, PH_TAU_BUILD);
      BSE_TRY(tau_build_range(c, orbr, gb0, nt, c->rebuild_buf, nt, 0, mask));
    }
    PhaseScope ps(c, PH_TAU_TILE);
    int row0 = 0, rows = 0;  // the first launch writes every band of y
    if (!first) tile_rows(c, gb0, nt, &row0, &rows);
    BSE_TRY(tau_stream(c->rebuild_buf, nt, nt, c->blkIJ + gb0, c->R, a, y, nb, c->nv, nr,
                       first ? 0 : 1, c->max_lds, c->st, nullptr, c->tau_bl, row0, rows));
    first = 0;
  }
  return BSE_OK;
}

int ensure_apply_work(bse_ctx* c, int nbc) {
  if (c->nbc >= nbc) return BSE_OK;
  ctx_release(c, c->A_s);
  ctx_release(c, c->Zs);
  ctx_release(c, c->A_rot);
  ctx_release(c, c->agrid);
  ctx_release(c, c->drho);
  c->A_s = c->Zs = c->A_rot = nullptr;
  c->agrid = c->drho = nullptr;
  c->nbc = 0;
  const size_t npw = c->basis.npw, nr = c->basis.nr;
  BSE_TRY(ctx_alloc_t(c, &c->A_s, (size_t)nbc * c->nv * npw));
  BSE_TRY(ctx_alloc_t(c, &c->Zs, (size_t)nbc * c->nv * npw));
  if (c->loc) BSE_TRY(ctx_alloc_t(c, &c->A_rot, (size_t)nbc * c->nv * npw));
  BSE_TRY(ctx_alloc_t(c, &c->agrid, (size_t)nbc * c->nvh * nr));
  BSE_TRY(ctx_alloc_t(c, &c->drho, (size_t)((nbc + 1) / 2) * nr));
  c->nbc = nbc;
  if (c->ygrid) {  // keep the accumulation buffer as large as the chunk
    ctx_release(c, c->ygrid);
    c->ygrid = nullptr;
    BSE_TRY(ensure_ygrid(c));
  }
  return BSE_OK;
}

int ensure_ygrid(bse_ctx* c) {
  if (c->ygrid) return BSE_OK;
  return ctx_alloc_t(c, &c->ygrid, (size_t)c->nbc * c->nvh * c->basis.nr);
}

// out_v += scale sum_w L_w (v_c * (M_w x_v)) for the nx real grid functions
// x_v (packed two per complex grid, like out); L and M hold the nv occupied-
// sized functions of the exact-exchange terms (SM Sec. I).  One Poisson solve
// per (w, v) pair, batched over w.
int exchange_like(bse_ctx* c, const double2* L, const double2* M, const double2* x, int nx,
                  double2* out, double scale) {
  const long nr = c->basis.nr;
  if (!c->xpair) BSE_TRY(ctx_alloc_t(c, &c->xpair, (size_t)c->nvh * nr));
  double2* P = c->xpair;
  for (int v = 0; v < nx; ++v) {
    BSE_TRY(pair_times(M, c->nv, x + (long)(v >> 1) * nr, v & 1, nr, P, c->st));
    BSE_TRY(fft3d(c->fft, P, c->nvh, -1, c->st));
    BSE_TRY(mul_real_field(P, c->nvh, nr, c->vc, 1.0 / (double)nr, c->st));
    BSE_TRY(fft3d(c->fft, P, c->nvh, +1, c->st));
    BSE_TRY(contract_pairs(L, P, c->nv, nr, out + (long)(v >> 1) * nr, v & 1, scale, c->st));
  }
  return BSE_OK;
}

// band index of nb vector sets into the localised frame (out_b = U^T A_b)
// or back (out_b = U A_b)
int rotate_bands(bse_ctx* c, int nb, const double* A, double* out, bool back) {
  const long npw = c->basis.npw, L = (long)c->nv * npw;
  for (int b = 0; b < nb; ++b)
    BSE_TRY(dgemm(back ? 0 : 1, 0, c->nv, npw, c->nv, 1.0, c->Uloc, c->nv, A + b * L, npw, 0.0,
                  out + b * L, npw, c->st));
  return BSE_OK;
}

// the gathered grid part Zg (in the kernel frame) plus the diagonal of D on
// A, projected: Y = P_c (Zg + (T - eps_v + Delta) A); in a localised frame
// Zg is rotated back first and the diagonal added in the canonical frame
static int finish_apply(bse_ctx* c, int nb, const double* A, int with_v, double* Y) {
  if (c->loc) {
    BSE_TRY(rotate_bands(c, nb, c->Zs, c->A_rot, true));
    if (with_v)
      BSE_TRY(diag_axpy(A, c->T, c->eps_d, c->scissor, c->nv, c->basis.npw, nb, c->A_rot, c->st));
    return proj_c(c, c->A_rot, Y, nb);
  }
  return proj_c(c, c->Zs, Y, nb);
}

// out_v += scale sum_w L_w [W (M_w x_v)] for the nx real grid functions x_v
// (packed like out): the exchange form of W, the bare Coulomb part and, by
// the kernel mask, the PDEP part of Eq. 3 (two GEMMs on the sphere
// coefficients of the nv pair densities of each v).
static int w_exchange_like(bse_ctx* c, const double2* L, const double2* M, const double2* x,
                           int nx, double2* out, double scale) {
  const long nr = c->basis.nr, npw = c->basis.npw;
  const int nv = c->nv;
  const bool bare = (c->kmask & BSE_K_1D_BARE) != 0;
  const bool pdep = (c->kmask & BSE_K_1D_PDEP) && c->npdep > 0;
  if (!c->xpair) BSE_TRY(ctx_alloc_t(c, &c->xpair, (size_t)c->nvh * nr));
  if (pdep && !c->wx_RS) {
    BSE_TRY(ctx_alloc_t(c, &c->wx_RS, (size_t)nv * npw));
    BSE_TRY(ctx_alloc_t(c, &c->wx_T, (size_t)nv * c->npdep));
    BSE_TRY(ctx_alloc_t(c, &c->wx_F, (size_t)nv * npw));
    BSE_TRY(ctx_alloc_t(c, &c->wx_cmp, (size_t)c->nvh * npw));
  }
  double2* P = c->xpair;
  SphereMap m = c->map;
  const bool fused = w_fused_on(), pairs = w_pairs_on(c, false);
  for (int v = 0; v < nx; ++v) {
    const double2* xv = x + (long)(v >> 1) * nr;
    if (pairs) {
      BSE_TRY(fft3d_fwd_times(c->fft, c->sp, M, c->nvh, xv, v & 1, P, bare ? c->vc : nullptr,
                              1.0 / (double)nr, pdep ? c->wx_cmp : nullptr, c->st));
    } else {
      BSE_TRY(pair_times(M, nv, xv, v & 1, nr, P, c->st));
      if (fused)
        BSE_TRY(fft3d_fwd_w(c->fft, c->sp, P, c->nvh, bare ? c->vc : nullptr, 1.0 / (double)nr,
                            pdep ? c->wx_cmp : nullptr, c->st));
      else
        BSE_TRY(fft3d(c->fft, P, c->nvh, -1, c->st));
    }
    if (pdep) {
      BSE_TRY(gather_sets(fused ? c->cmap : m, fused ? c->wx_cmp : P, nv, 1, 1.0 / (double)nr,
                          nullptr, nullptr, nullptr, 0.0, 0.0, c->wx_RS, c->st));
      BSE_TRY(gemm(c, 0, 0, nv, c->npdep, npw, 1.0, c->wx_RS, npw, c->Pt, c->npdep, 0.0,
                   c->wx_T, c->npdep));
      BSE_TRY(dgemm(0, 1, nv, npw, c->npdep, 1.0, c->wx_T, c->npdep, c->Ptc, c->npdep, 0.0,
                    c->wx_F, npw, c->st));
    }
    if (!fused && bare)
      BSE_TRY(mul_real_field(P, c->nvh, nr, c->vc, 1.0 / (double)nr, c->st));
    else if (!fused)
      BSE_TRY(zero_fill(reinterpret_cast<double*>(P), 2L * c->nvh * nr, c->st));
    if (pdep) BSE_TRY(scatter_sets(m, c->wx_F, nv, 1, P, 1, c->st));
    BSE_TRY(fft3d(c->fft, P, c->nvh, +1, c->st));
    BSE_TRY(contract_pairs(L, P, nv, nr, out + (long)(v >> 1) * nr, v & 1, scale, c->st));
  }
  return BSE_OK;
}

// Coupling beyond the TDA (SM Sec. I), real orbitals:
//   Y = P_c (s K2e - K2d) P_c X,  (K2e A)_v = P_c [v_c * sum a_v' phi_v'] phi_v,
//   (K2d A)_v = P_c sum_v' [W (a_v' phi_v)] phi_v',
// in FP64 and in the canonical frame, chunks of at most c->nbc vectors.
int apply_coupling(bse_ctx* c, int nb, const double* X, double* Y) {
  const long nr = c->basis.nr, L = (long)c->nv * c->basis.npw, gs = (long)c->nvh * nr;
  BSE_TRY(ensure_ygrid(c));
  for (int i0 = 0; i0 < nb; i0 += c->nbc) {
    const int k = std::min(c->nbc, nb - i0);
    BSE_TRY(proj_c(c, X + i0 * L, c->A_s, k));
    BSE_TRY(to_grid(c, c->A_s, c->nv, k, c->agrid));
    double2* z = c->ygrid;
    if (c->kmask & BSE_K_1E) {
      const long nbh = (k + 1) / 2;
      BSE_TRY(transition_density(c->phir, c->agrid, c->nv, k, nr, c->drho, c->st));
      BSE_TRY(fft3d(c->fft, c->drho, nbh, -1, c->st));
      BSE_TRY(mul_real_field(c->drho, nbh, nr, c->vc, 1.0 / (double)nr, c->st));
      BSE_TRY(fft3d(c->fft, c->drho, nbh, +1, c->st));
      BSE_TRY(combine(c->agrid, c->phir, c->Vr, c->drho, nullptr, z, c->nv, k, nr, c->spin, 0,
                      c->st));
    } else {
      BSE_TRY(zero_fill(reinterpret_cast<double*>(z), 2 * k * gs, c->st));
    }
    if (c->kmask & (BSE_K_1D_BARE | BSE_K_1D_PDEP))
      for (int b = 0; b < k; ++b)
        BSE_TRY(w_exchange_like(c, c->phir, c->agrid + b * gs, c->phir, c->nv, z + b * gs, -1.0));
    BSE_TRY(from_grid(c, z, c->nv, k, nullptr, nullptr, 0.0, c->Zs));
    BSE_TRY(proj_c(c, c->Zs, Y + i0 * L, k));
  }
  return BSE_OK;
}

// Y = P_c (D + s K1e - K1d) P_c X for nb <= c->nbc vectors; in a localised
// frame the grid part runs on A~ = U^T A with the localised orbitals
int apply_chunk(bse_ctx* c, int nb, const double* X, double* Y) {
  const long nr = c->basis.nr;
  const double* A = c->in_pc ? X : c->A_s;
  if (!c->in_pc) BSE_TRY(proj_c(c, X, c->A_s, nb));
  const double* Ag = A;
  if (c->loc) {
    BSE_TRY(rotate_bands(c, nb, A, c->A_rot, false));
    Ag = c->A_rot;
  }
  BSE_TRY(to_grid(c, Ag, c->nv, nb, c->agrid));
  const double2* vdrho = nullptr;
  if (c->kmask & BSE_K_1E) {
    PhaseScope ps(c, PH_K1E);
    const long nbh = (nb + 1) / 2;
    BSE_TRY(transition_density(c->phik, c->agrid, c->nv, nb, nr, c->drho, c->st));
    BSE_TRY(fft3d(c->fft, c->drho, nbh, -1, c->st));
    BSE_TRY(mul_real_field(c->drho, nbh, nr, c->vc, 1.0 / (double)nr, c->st));
    BSE_TRY(fft3d(c->fft, c->drho, nbh, +1, c->st));
    vdrho = c->drho;
  }
  const int with_v = (c->kmask & BSE_K_D) ? 1 : 0;
  double2* zg = c->agrid;
  // exact-exchange part of H_KS in D: -alpha K_x a_v, K_x a = sum_w phi_w v_c*(phi_w a)
  // (taken before the stream, which may overwrite a(r) with z)
  const long gs = (long)c->nvh * nr;
  if (c->alpha != 0.0 && with_v) {
    if (!c->xgrid || c->xgrid_sets < nb) {
      ctx_release(c, c->xgrid);
      c->xgrid = nullptr;
      BSE_TRY(ctx_alloc_t(c, &c->xgrid, (size_t)c->nbc * gs));
      c->xgrid_sets = c->nbc;
    }
    BSE_TRY(zero_fill(reinterpret_cast<double*>(c->xgrid), 2 * nb * gs, c->st));
    for (int b = 0; b < nb; ++b)
      BSE_TRY(exchange_like(c, c->phir, c->phir, c->agrid + b * gs, c->nv, c->xgrid + b * gs,
                            -c->alpha));
  }
  if (c->kmask & (BSE_K_1D_BARE | BSE_K_1D_PDEP)) {
    if (c->nblk_cached == c->nblk) {
      // whole tau cached: one launch, combine fused, z written over a(r)
      FuseArgs f{c->Vr, vdrho, c->phik, c->spin, with_v};
      BSE_TRY(tau_contract(c, c->phik, c->agrid, c->agrid, nb, c->kmask, true, &f));
    } else {
      BSE_TRY(ensure_ygrid(c));
      BSE_TRY(tau_contract(c, c->phik, c->agrid, c->ygrid, nb, c->kmask, true));
      PhaseScope ps(c, PH_COMBINE);
      BSE_TRY(combine(c->agrid, c->phik, c->Vr, vdrho, c->ygrid, c->ygrid, c->nv, nb, nr, c->spin,
                      with_v, c->st));
      zg = c->ygrid;
    }
  } else {
    PhaseScope ps(c, PH_COMBINE);
    BSE_TRY(combine(c->agrid, c->phik, c->Vr, vdrho, nullptr, c->agrid, c->nv, nb, nr, c->spin,
                    with_v, c->st));
  }
  if (c->alpha != 0.0 && with_v)
    BSE_TRY(axpby(1.0, reinterpret_cast<const double*>(c->xgrid), 1.0,
                  reinterpret_cast<double*>(zg), 2 * nb * gs, c->st));
  const bool diag_here = with_v && !c->loc;
  BSE_TRY(from_grid(c, zg, c->nv, nb, diag_here ? A : nullptr, c->eps_d, c->scissor, c->Zs));
  return finish_apply(c, nb, A, with_v, Y);
}

// kernel part of the operator on one exciton, before P_c, gathered:
//   Kt_v = <e| s (v_c*Drho) phi_v - sum_v' tau_{v'v} a_v' >
// a(r) in agrid set 0; set 1 is scratch; drho keeps v_c*Drho afterwards.
// A mixed context contracts with its whole FP32 tau cache (a and the sum
// pass through FP32 grids) instead of rebuilding the blocks its FP64 cache
// lacks.
int kernel_part(bse_ctx* c, const double2* agrid, double* Kt) {
  const long nr = c->basis.nr;
  double2* y = c->agrid + (long)c->nvh * nr;
  const double2* vdrho = nullptr;
  if (c->kmask & BSE_K_1E) {
    BSE_TRY(transition_density(c->phik, agrid, c->nv, 1, nr, c->drho, c->st));
    BSE_TRY(fft3d(c->fft, c->drho, 1, -1, c->st));
    BSE_TRY(mul_real_field(c->drho, 1, nr, c->vc, 1.0 / (double)nr, c->st));
    BSE_TRY(fft3d(c->fft, c->drho, 1, +1, c->st));
    vdrho = c->drho;
  }
  const double2* yk = nullptr;
  if ((c->kmask & (BSE_K_1D_BARE | BSE_K_1D_PDEP)) && c->active == BSE_MIXED && c->tau_f) {
    BSE_TRY(ensure_mixed_work(c, 2));
    const long ng = (long)c->nvh * nr;
    float2* af = c->agrid_f;
    float2* yf = c->agrid_f + ng;
    BSE_TRY(to_f32(reinterpret_cast<const double*>(agrid), reinterpret_cast<float*>(af), 2 * ng,
                   c->st));
    {
      PhaseScope ps(c, PH_TAU_STREAM);
      BSE_TRY(tau_stream(c->tau_f, c->nblk, c->nblk, c->blkIJ, c->Rf, af, yf, 1, c->nv, nr, 0,
                         c->max_lds, c->st, nullptr, c->tau_bl));
    }
    BSE_TRY(to_f64(reinterpret_cast<const float*>(yf), reinterpret_cast<double*>(y), 2 * ng,
                   c->st));
    yk = y;
  } else if (c->kmask & (BSE_K_1D_BARE | BSE_K_1D_PDEP)) {
    BSE_TRY(tau_contract(c, c->phik, agrid, y, 1, c->kmask, true));
    yk = y;
  }
  BSE_TRY(combine(agrid, c->phik, c->Vr, vdrho, yk, y, c->nv, 1, nr, c->spin, 0, c->st));
  BSE_TRY(from_grid(c, y, c->nv, 1, nullptr, nullptr, 0.0, Kt));
  return BSE_OK;
}

// sigma term of U:  y_v = sum_v' W(a_v' a_v) phi_v'  (sigma built from a,
// contracted with phi), tiles rebuilt for every block.  A mixed context
// builds and contracts the tiles in FP32 (a and the sum pass through FP32
// grids).
int sigma_phi(bse_ctx* c, const double2* agrid, double2* y) {
  if (!(c->active == BSE_MIXED && c->vc_f && c->phik_f))
    return tau_contract(c, agrid, c->phik, y, 1, c->kmask, false);
  const long nr = c->basis.nr, ng = (long)c->nvh * nr;
  BSE_TRY(ensure_mixed_work(c, 2));
  float2* af = c->agrid_f;
  float2* yf = c->agrid_f + ng;
  BSE_TRY(to_f32(reinterpret_cast<const double*>(agrid), reinterpret_cast<float*>(af), 2 * ng,
                 c->st));
  float* buf = reinterpret_cast<float*>(c->rebuild_buf);
  for (long gb0 = 0; gb0 < c->nblk; gb0 += c->tile_blk) {
    const long nt = std::min(c->tile_blk, c->nblk - gb0);
    {
      PhaseScope ps(c, PH_TAU_BUILD);
      BSE_TRY(tau_build_range_f(c, af, gb0, nt, buf, nt, 0, c->kmask));
    }
    PhaseScope ps(c, PH_TAU_TILE);
    int row0 = 0, rows = 0;  // the first launch writes every band of y
    if (gb0 > 0) tile_rows(c, gb0, nt, &row0, &rows);
    BSE_TRY(tau_stream(buf, nt, nt, c->blkIJ + gb0, c->Rf, c->phik_f, yf, 1, c->nv, nr,
                       gb0 == 0 ? 0 : 1, c->max_lds, c->st, nullptr, c->tau_bl, row0, rows));
  }
  return to_f64(reinterpret_cast<const float*>(yf), reinterpret_cast<double*>(y), 2 * ng, c->st);
}

// ---------------------------------------------------------------------------
// mixed precision: FP32 grids, transforms, K1e and tau contraction; the
// projector, the diagonal (T - eps + Delta) A and everything in G space stay
// FP64
// ---------------------------------------------------------------------------
int ensure_mixed_work(bse_ctx* c, int nbc) {
  if (c->nbc_f >= nbc) return BSE_OK;
  ctx_release(c, c->agrid_f);
  ctx_release(c, c->drho_f);
  c->agrid_f = c->drho_f = nullptr;
  c->nbc_f = 0;
  const size_t nr = c->basis.nr;
  BSE_TRY(ctx_alloc_t(c, &c->agrid_f, (size_t)nbc * c->nvh * nr));
  BSE_TRY(ctx_alloc_t(c, &c->drho_f, (size_t)((nbc + 1) / 2) * nr));
  c->nbc_f = nbc;
  return BSE_OK;
}

static int ensure_compact_f(bse_ctx* c, long ngrids) {
  if (c->compact_f_grids >= ngrids) return BSE_OK;
  ctx_release(c, c->compact_f);
  c->compact_f = nullptr;
  c->compact_f_grids = 0;
  BSE_TRY(ctx_alloc_t(c, &c->compact_f, (size_t)ngrids * c->basis.npw));
  c->compact_f_grids = ngrids;
  return BSE_OK;
}

static int from_grid_f(bse_ctx* c, float2* grids, int nvs, int nset, const double* A,
                       const double* eps, double shift, double* Y) {
  PhaseScope ps(c, PH_FFT_FWD);
  const long ng = (long)nset * ((nvs + 1) / 2);
  BSE_TRY(ensure_compact_f(c, ng));
  BSE_TRY(grid_to_compact(c->fft, c->sp, grids, ng, c->compact_f, c->st));
  return gather_sets(c->cmap, c->compact_f, nvs, nset, 1.0 / (double)c->basis.nr, A, c->T, eps,
                     shift, 0.0, Y, c->st);
}

int apply_chunk_mixed(bse_ctx* c, int nb, const double* X, double* Y) {
  const long nr = c->basis.nr;
  BSE_TRY(ensure_mixed_work(c, c->nbc));
  const double* A = c->in_pc ? X : c->A_s;
  if (!c->in_pc) BSE_TRY(proj_c(c, X, c->A_s, nb));
  const double* Ag = A;
  if (c->loc) {
    BSE_TRY(rotate_bands(c, nb, A, c->A_rot, false));
    Ag = c->A_rot;
  }
  {
    PhaseScope ps(c, PH_FFT_INV);
    BSE_TRY(sphere_to_grid(c->fft, c->sp, c->basis.omega, Ag, c->nv, nb, c->agrid_f, c->st));
  }
  const float2* vdrho = nullptr;
  if (c->kmask & BSE_K_1E) {
    PhaseScope ps(c, PH_K1E);
    const long nbh = (nb + 1) / 2;
    BSE_TRY(transition_density(c->phik_f, c->agrid_f, c->nv, nb, nr, c->drho_f, c->st));
    BSE_TRY(fft3d(c->fft, c->drho_f, nbh, -1, c->st));
    BSE_TRY(mul_real_field(c->drho_f, nbh, nr, c->vc_f, 1.0f / (float)nr, c->st));
    BSE_TRY(fft3d(c->fft, c->drho_f, nbh, +1, c->st));
    vdrho = c->drho_f;
  }
  const int with_v = (c->kmask & BSE_K_D) ? 1 : 0;
  if (c->kmask & (BSE_K_1D_BARE | BSE_K_1D_PDEP)) {
    PhaseScope ps(c, PH_TAU_STREAM);
    FuseArgsF f{c->Vr_f, vdrho, c->phik_f, c->spin, with_v};
    BSE_TRY(tau_stream(c->tau_f, c->nblk, c->nblk, c->blkIJ, c->Rf, c->agrid_f, c->agrid_f, nb,
                       c->nv, nr, 0, c->max_lds, c->st, &f, c->tau_bl));
  } else {
    PhaseScope ps(c, PH_COMBINE);
    BSE_TRY(combine(c->agrid_f, c->phik_f, c->Vr_f, vdrho, nullptr, c->agrid_f, c->nv, nb, nr,
                    c->spin, with_v, c->st));
  }
  const bool diag_here = with_v && !c->loc;
  BSE_TRY(from_grid_f(c, c->agrid_f, c->nv, nb, diag_here ? A : nullptr, c->eps_d, c->scissor,
                      c->Zs));
  return finish_apply(c, nb, A, with_v, Y);
}

int apply_any(bse_ctx* c, int nb, const double* X, double* Y) {
  if (c->active == BSE_MIXED) return apply_chunk_mixed(c, nb, X, Y);
  return apply_chunk(c, nb, X, Y);
}

// (T + shift - eps_v) X + <e| V(r) x(r)> with the grid part in FP32
int apply_H_f(bse_ctx* c, int nvs, int nset, const double* X, double* Y, double shift,
              const double* eps, int project) {
  const long ng = (long)nset * ((nvs + 1) / 2);
  if (ng > (long)c->nbc_f * c->nvh) return fail(BSE_EINVAL, "FP32 grid work too small");
  {
    PhaseScope ps(c, PH_FFT_INV);
    BSE_TRY(sphere_to_grid(c->fft, c->sp, c->basis.omega, X, nvs, nset, c->agrid_f, c->st));
  }
  BSE_TRY(mul_real_field(c->agrid_f, ng, c->basis.nr, c->Vr_f, 1.0f, c->st));
  BSE_TRY(from_grid_f(c, c->agrid_f, nvs, nset, X, eps, shift, Y));
  if (project) BSE_TRY(proj_c(c, Y, Y, nset));
  return BSE_OK;
}

}  // namespace bsex

namespace bsex {

// ---------------------------------------------------------------------------
// HIP graphs of the block apply
// ---------------------------------------------------------------------------
void graphs_destroy(bse_ctx* c) {
  if (c->graphs.empty()) return;
  if (c->st) (void)hipStreamSynchronize(c->st);
  for (auto& g : c->graphs) (void)hipGraphExecDestroy(g.second);
  c->graphs.clear();
  c->graph_bufs.clear();
}

int graph_apply(bse_ctx* c, int nb, const double* X, double* Y) {
  const long L = (long)c->nv * c->basis.npw;
  if (nb < 1 || nb > c->nbc) return fail(BSE_EINVAL, "graph apply: block of %d", nb);
  const int key = nb * 4 + c->active + (c->in_pc ? 2 : 0);
  for (auto& g : c->graphs)
    if (g.first == key) {
      BSE_HIP(hipMemcpyAsync(c->gX, X, sizeof(double) * nb * L, hipMemcpyDeviceToDevice, c->st));
      BSE_HIP(hipGraphLaunch(g.second, c->st));
      BSE_HIP(hipMemcpyAsync(Y, c->gY, sizeof(double) * nb * L, hipMemcpyDeviceToDevice, c->st));
      return BSE_OK;
    }
  if (!c->gX) {
    BSE_TRY(ctx_alloc_t(c, &c->gX, (size_t)c->nbc * L));
    BSE_TRY(ctx_alloc_t(c, &c->gY, (size_t)c->nbc * L));
  }
  // eager run first: it sizes every lazily allocated buffer and gives Y
  BSE_HIP(hipMemcpyAsync(c->gX, X, sizeof(double) * nb * L, hipMemcpyDeviceToDevice, c->st));
  BSE_TRY(apply_any(c, nb, c->gX, c->gY));
  BSE_HIP(hipMemcpyAsync(Y, c->gY, sizeof(double) * nb * L, hipMemcpyDeviceToDevice, c->st));
  BSE_HIP(hipStreamSynchronize(c->st));
  const size_t n_alloc = c->allocs.size();
  // capture on a private stream (the context's may be the legacy null stream,
  // which cannot be captured); nothing runs during capture
  if (!c->cap_st) BSE_HIP(hipStreamCreateWithFlags(&c->cap_st, hipStreamNonBlocking));
  hipGraph_t graph = nullptr;
  BSE_HIP(hipStreamBeginCapture(c->cap_st, hipStreamCaptureModeThreadLocal));
  hipStream_t keep = c->st;
  c->st = c->cap_st;
  const int rc = apply_any(c, nb, c->gX, c->gY);
  c->st = keep;
  const hipError_t e = hipStreamEndCapture(c->cap_st, &graph);
  if (rc != BSE_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc;
  }
  if (e != hipSuccess || !graph)
    return fail(BSE_EHIP, "graph capture failed: %s", hipGetErrorString(e));
  if (c->allocs.size() != n_alloc) {  // cannot happen after the eager run
    (void)hipGraphDestroy(graph);
    return fail(BSE_ESTATE, "graph capture allocated");
  }
  hipGraphExec_t exec = nullptr;
  const hipError_t e2 = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e2 != hipSuccess) return fail(BSE_EHIP, "graph instantiate: %s", hipGetErrorString(e2));
  c->graphs.push_back({key, exec});
  // every buffer of the context may be referenced by the graph
  c->graph_bufs.clear();
  for (auto& b : c->allocs) c->graph_bufs.push_back(b.p);
  return BSE_OK;
}

}  // namespace bsex
