// Uneven batches of independent systems: a host scheduler (batch_sched.h) keeps up
// to n_streams systems in flight, each on its own HIP stream and host thread,
// largest first, admitting a system only while its device-memory estimate
// fits the batch budget.  Per shape (grid, N_v, precision, block) an
// autotuner times the Davidson block apply under each kernel variant and
// caches the fastest; Davidson applies can replay captured HIP graphs.  Each
// system is solved exactly as by the single-system calls: ground state, the
// lowest exciton, the Z-vector and the forces of Eqs. 4-7.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <string>
#include <map>
#include <mutex>
#include <numeric>
#include <thread>
#include <tuple>
#include <vector>

#include "context.h"
#include "batch_sched.h"

namespace bsex {
const char* last_error();

namespace {

// stack of each slot thread (solver host code, HIP runtime, profiler callbacks)
constexpr size_t kSlotStack = (size_t)64 << 20;

// variant bits: 1 = runtime-length FFT kernels, 2 = the tau stream whose four
// lanes per grid point each read whole blocks (instead of quad-shared loads)
void set_variant(bse_ctx* c, int v) {
  fft_plan_set_runtime(&c->fft, (v & 1) != 0);
  c->tau_bl = (v & 2) ? 4 : 1;
}

using TuneKey = std::tuple<int, int, int, int, int, int>;
std::mutex g_tune_mu;
std::map<TuneKey, int> g_tune;

int time_variant(bse_ctx* c, int nb, double* X, double* Y, int reps, double* ms) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  BSE_HIP(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(BSE_EHIP, "event create failed");
  }
  int rc = BSE_OK;
  if (hipEventRecord(e0, c->st) != hipSuccess) rc = fail(BSE_EHIP, "event record failed");
  for (int r = 0; r < reps && rc == BSE_OK; ++r) rc = apply_any(c, nb, X, Y);
  float t = 0.0f;
  if (rc == BSE_OK && (hipEventRecord(e1, c->st) != hipSuccess ||
                       hipEventSynchronize(e1) != hipSuccess ||
                       hipEventElapsedTime(&t, e0, e1) != hipSuccess))
    rc = fail(BSE_EHIP, "event timing failed");
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *ms = t / reps;
  return rc;
}

// shape class of a system: grid, band count in buckets of 64, precision and
// Davidson block (the variants' ranking follows the grid and the band scale)
TuneKey tune_key(const int grid[3], int nv, int precision, int nb) {
  return TuneKey{grid[0], grid[1], grid[2], (nv + 63) / 64, precision, nb};
}

// pick (and cache) the fastest variant for this context's shape class: one
// warm-up apply, then two timed applies per variant
int autotune(bse_ctx* c, int nb, int* chosen, double* best_ms) {
  const TuneKey key = tune_key(c->basis.grid, c->nv, c->active, nb);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(key);
    if (it != g_tune.end()) {
      set_variant(c, it->second);
      *chosen = it->second;
      *best_ms = -1.0;
      return BSE_OK;
    }
  }
  const long L = (long)c->nv * c->basis.npw;
  double *X = nullptr, *Y = nullptr;
  BSE_TRY(ctx_alloc_t(c, &X, (size_t)nb * L));
  int rc = ctx_alloc_t(c, &Y, (size_t)nb * L);
  if (rc == BSE_OK) rc = zero_fill(X, (long)nb * L, c->st);
  const bool ct = c->fft.ct_plane_ok[0] || c->fft.ct_axis_ok[0] || c->fft.ct_plane_ok[1] ||
                  c->fft.ct_axis_ok[1];
  int best = 0;
  double bms = 1e300;
  if (rc == BSE_OK) rc = apply_any(c, nb, X, Y);  // warm-up (and lazy buffers)
  for (int v = 0; v < 4 && rc == BSE_OK; ++v) {
    if ((v & 1) && !ct) continue;  // no compile-time FFT to switch off
    set_variant(c, v);
    double ms = 0.0;
    rc = time_variant(c, nb, X, Y, 2, &ms);
    if (rc == BSE_OK && ms < bms) {
      bms = ms;
      best = v;
    }
  }
  ctx_release(c, X);
  ctx_release(c, Y);
  BSE_TRY(rc);
  set_variant(c, best);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[key] = best;
  }
  *chosen = best;
  *best_ms = bms;
  return BSE_OK;
}

// device bytes one system holds at its peak (tau cache, apply and solver
// buffers, ground-state block), an estimate for admission only
double estimate_bytes(const bse_system_desc& d, int prec, long npw, double* tau_bytes) {
  const double nr = (double)d.grid[0] * d.grid[1] * d.grid[2];
  const double nv = d.n_val, nvh = (d.n_val + 1) / 2;
  const double nB = (d.n_val + 7) / 8;
  const double nblk = nB * (nB + 1) / 2;
  *tau_bytes = nblk * 64 * nr * (prec == BSE_MIXED ? 4.0 : 8.0);
  const double L = nv * npw * 8.0;
  const double grids = 8 * nvh * nr * 16.0 * (prec == BSE_MIXED ? 2.5 : 2.0);
  const double tiles = 4 * 64 * (2.0 * nr + 2.0 * npw + std::max(d.n_pdep, 1)) * 8.0;
  const double solver = (2 * 16 * 5 + 4 * 5 + 8) * L;  // Davidson of one state: 5-vector blocks
  const double gs = (d.n_val + 56) * npw * 8.0 * 8;
  return *tau_bytes + grids + tiles + solver + gs + 0.5e9;
}

int run_one(const bse_system_desc& d0, const bse_batch_opts& o, hipStream_t st, double tau_bytes,
            bool tune, bse_batch_result* r) {
  using clk = std::chrono::steady_clock;
  auto ms_since = [](clk::time_point t) {
    return std::chrono::duration<double, std::milli>(clk::now() - t).count();
  };
  bse_system_desc d = d0;
  d.stream = st;
  d.precision = o.precision;
  if (d.tau_policy == BSE_TAU_AUTO) d.tau_budget_bytes = (int64_t)(tau_bytes * 1.02) + (1 << 20);
  auto t0 = clk::now();
  bse_ctx* c = nullptr;
  BSE_TRY(bse_init_system(&d, &c));
  r->t_init_ms = ms_since(t0);
  const long L = (long)c->nv * c->basis.npw;
  double *X = nullptr, *Z = nullptr;
  int rc = ctx_alloc_t(c, &X, (size_t)L);
  if (rc == BSE_OK) rc = ctx_alloc_t(c, &Z, (size_t)L);
  bse_solver_opts so{};
  so.tol = o.tol > 0 ? o.tol : 1e-6;
  const int block = 5;  // Davidson block for one state
  if (rc == BSE_OK && tune) {
    double ms = 0;
    rc = autotune(c, block, &r->variant, &ms);
  }
  if (rc == BSE_OK && o.use_graph) c->use_graph = true;
  bse_solver_stats ds{}, zs{};
  if (rc == BSE_OK) {
    auto t1 = clk::now();
    rc = bse_davidson(c, 1, &so, &r->omega, X, &ds);
    r->t_davidson_ms = ms_since(t1);
    r->davidson_iters = ds.iters;
  }
  if (rc == BSE_OK) {
    auto t2 = clk::now();
    rc = bse_zvector_solve(c, X, &so, Z, &zs);
    r->t_z_ms = ms_since(t2);
    r->z_iters = zs.iters;
  }
  if (rc == BSE_OK && r->dwdR_host) {
    auto t3 = clk::now();
    rc = bse_forces(c, X, Z, r->dwdR_host);
    r->t_force_ms = ms_since(t3);
  }
  if (rc != BSE_OK) {
    std::string keep = last_error();
    bse_free(c);
    set_error("%s", keep.c_str());
    return rc;
  }
  bse_free(c);
  return BSE_OK;
}

}  // namespace
}  // namespace bsex

using namespace bsex;

extern "C" int bse_batch_run(const bse_system_desc* descs, int32_t n, const bse_batch_opts* opts,
                             bse_batch_result* results) {
  if (n < 0 || (n > 0 && (!descs || !results))) return fail(BSE_EINVAL, "NULL argument");
  if (n == 0) return BSE_OK;
  bse_batch_opts o{};
  if (opts) o = *opts;
  if (o.precision != BSE_FP64 && o.precision != BSE_MIXED)
    return fail(BSE_EINVAL, "precision %d unknown", o.precision);
  const int ns = o.n_streams > 0 ? std::min(o.n_streams, 8) : 4;
  int dev = 0;
  BSE_HIP(hipGetDevice(&dev));
  size_t freeb = 0, totalb = 0;
  BSE_HIP(hipMemGetInfo(&freeb, &totalb));
  const double budget = o.mem_budget > 0 ? (double)o.mem_budget : 0.85 * (double)freeb;
  std::vector<double> est(n), taub(n);
  for (int i = 0; i < n; ++i) {
    int32_t npw = 0;
    const int rc = bse_basis_size(descs[i].cell, descs[i].grid, descs[i].ecut, &npw);
    if (rc != BSE_OK) return rc;
    est[i] = estimate_bytes(descs[i], o.precision, npw, &taub[i]);
    results[i].status = -1;
    results[i].omega = 0.0;
    results[i].davidson_iters = results[i].z_iters = 0;
    results[i].t_init_ms = results[i].t_davidson_ms = results[i].t_z_ms = results[i].t_force_ms = 0;
    results[i].variant = -1;
    results[i].stream_slot = -1;
    results[i].message[0] = 0;
  }
  // tuning pays only for shape classes that recur in the batch
  std::map<TuneKey, int> classes;
  for (int i = 0; i < n; ++i)
    ++classes[tune_key(descs[i].grid, descs[i].n_val, o.precision, 5)];
  // one stream per slot thread, created and destroyed on that thread
  std::vector<hipStream_t> streams(ns, nullptr);
  BatchHooks hooks;
  hooks.slot_begin = [&](int slot) {
    (void)hipSetDevice(dev);
    if (hipStreamCreateWithFlags(&streams[slot], hipStreamNonBlocking) != hipSuccess)
      streams[slot] = nullptr;
  };
  hooks.run = [&](int slot, int pick) {
    bse_batch_result* r = &results[pick];
    r->stream_slot = slot;
    hipStream_t st = streams[slot];
    int rc = st ? BSE_OK : fail(BSE_EHIP, "stream creation failed");
    if (rc == BSE_OK) {
      try {
        const bool tune =
            o.autotune && classes.at(tune_key(descs[pick].grid, descs[pick].n_val, o.precision, 5)) > 1;
        rc = run_one(descs[pick], o, st, taub[pick], tune, r);
      } catch (...) {
        rc = fail(BSE_ENOMEM, "host allocation failed");
      }
    }
    r->status = rc;
    if (rc != BSE_OK) {
      std::strncpy(r->message, bse_last_error(), sizeof(r->message) - 1);
      r->message[sizeof(r->message) - 1] = 0;
    }
  };
  hooks.slot_end = [&](int slot) {
    if (streams[slot]) {
      (void)hipStreamSynchronize(streams[slot]);
      (void)hipStreamDestroy(streams[slot]);
    }
  };
  if (schedule_batch(n, est, budget, ns, kSlotStack, hooks) != 0)
    return fail(BSE_EINVAL, "no batch worker thread could be started");
  for (int i = 0; i < n; ++i)
    if (results[i].status != BSE_OK)
      return fail(results[i].status, "system %d: %s", i, results[i].message);
  return BSE_OK;
}

extern "C" int bse_tune_cache_clear(void) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune.clear();
  return BSE_OK;
}
