// d omega / d R without any allocation: bse_forces_noalloc.
//
// For callers that cannot allocate device memory (code under HIP graph
// capture, tight serving loops).  The scratch the force contraction needs
// beyond the context's own buffers (the occupied overlaps, the projector's
// overlap and the per-site partial sums) lives in one file-scope device
// array of kScratchDoubles doubles per device.  Its device address is looked
// up once per device when a context is initialised on it (bse_init_system)
// and kept in g_scratch; host code never passes the array's own name to a
// kernel.  All calls on a device share its array, which keeps the last
// call's contents: every part used is written before it is read, and calls
// that overlap on one device race.
#include <mutex>

#include "context.h"

namespace bsex {

namespace {
constexpr long kScratchDoubles = 8L << 20;  // 64 MiB per device
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch[kMaxDevices] = {nullptr};
}  // namespace

static __device__ __align__(256) double scratch[kScratchDoubles];

// With `dev` current: record the device address of this device's scratch.
int noalloc_setup(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return fail(BSE_EINVAL, "device %d out of range", dev);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch[dev]) return BSE_OK;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p)
    return fail(BSE_EHIP, "scratch address lookup failed: %s", hipGetErrorString(e));
  g_scratch[dev] = static_cast<double*>(p);
  return BSE_OK;
}

long noalloc_scratch_doubles() { return kScratchDoubles; }

}  // namespace bsex

using namespace bsex;

extern "C" int bse_forces_noalloc(bse_ctx* c, const double* Xs, const double* Zin,
                                  double* dwdR_dev) {
  if (!c || !Xs || !Zin) return fail(BSE_EINVAL, "NULL argument");
  if (c->nsites > 0 && !dwdR_dev) return fail(BSE_EINVAL, "dwdR_dev is NULL");
  double* s = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (c->dev >= 0 && c->dev < kMaxDevices) s = g_scratch[c->dev];
  }
  if (!s) return fail(BSE_ESTATE, "no scratch address for device %d", c->dev);
  if (c->nbc < 3 || !c->A_s || !c->agrid || !c->drho)
    return fail(BSE_ESTATE, "the context's apply buffers hold fewer than 3 vector sets");
  const long npw = c->basis.npw, nv = c->nv, L = nv * npw, nr = c->basis.nr;
  const long n_o = nv * nv, pl = c->nsites > 0 ? force_reduce_work(c->nsites, nr) : 0;
  const long base = 2 * n_o + pl;
  if (base > kScratchDoubles)
    return fail(BSE_EINVAL, "forces need %ld doubles of scratch; the limit is %ld", base,
                kScratchDoubles);
  // split-K work of the overlap product when it fits, a single pass otherwise
  const long tall = dgemm_tall_work(nv, nv, npw);
  const bool use_tall = base + tall <= kScratchDoubles;
  double* O = s;            // [nv][nv]  <a_v|a_v'>
  double* Ov = O + n_o;     // [nv][nv]  projector overlap
  double* part = Ov + n_o;  // per-site partial sums
  double* tw = part + pl;   // overlap split-K work
  double* A = c->A_s;       // P_c X
  double* Pt = c->A_s + L;  // O Phi
  double* Zp = c->A_s + 2 * L;
  const hipStream_t st = c->st;
  // P_c on the exciton and on Z (Eq. 5-6 take both in the unoccupied space)
  BSE_TRY(dgemm(0, 1, nv, nv, npw, 1.0, c->Phi, npw, Xs, npw, 0.0, Ov, nv, st));
  BSE_TRY(dgemm_from(1, 0, nv, npw, nv, -1.0, Ov, nv, c->Phi, npw, 1.0, Xs, A, npw, st));
  BSE_TRY(dgemm(0, 1, nv, nv, npw, 1.0, c->Phi, npw, Zin, npw, 0.0, Ov, nv, st));
  BSE_TRY(dgemm_from(1, 0, nv, npw, nv, -1.0, Ov, nv, c->Phi, npw, 1.0, Zin, Zp, npw, st));
  if (use_tall)
    BSE_TRY(dgemm_tall(nv, nv, npw, 1.0, A, npw, A, npw, 0.0, O, nv, tw, tall, st));
  else
    BSE_TRY(dgemm(0, 1, nv, nv, npw, 1.0, A, npw, A, npw, 0.0, O, nv, st));
  BSE_TRY(dgemm(0, 0, nv, npw, nv, 1.0, O, nv, c->Phi, npw, 0.0, Pt, npw, st));
  const long gs = (long)c->nvh * nr;
  const double om = c->basis.omega;
  BSE_TRY(sphere_to_grid(c->fft, c->sp, om, A, c->nv, 1, c->agrid, st));
  BSE_TRY(sphere_to_grid(c->fft, c->sp, om, Pt, c->nv, 1, c->agrid + gs, st));
  BSE_TRY(sphere_to_grid(c->fft, c->sp, om, Zp, c->nv, 1, c->agrid + 2 * gs, st));
  BSE_TRY(force_density(c->agrid, c->agrid + gs, c->agrid + 2 * gs, c->phir, c->nv, nr, c->drho,
                        st));
  BSE_TRY(fft3d(c->fft, c->drho, 1, -1, st));
  if (c->nsites > 0)
    BSE_TRY(force_reduce(c->drho, c->sites, c->sites + 3 * c->nsites, c->sites + 4 * c->nsites,
                         c->nsites, c->basis.grid, c->basis.cell, part, pl, dwdR_dev, st));
  return BSE_OK;
}
