// Batched in-place 3-D complex FFT (FP64) for gfx950.
//
// Two kernels per transform of [batch][N1][N2][N3] (N3 contiguous):
//  * a plane kernel holds one N2 x N3 plane (fixed i1) in LDS (83 KB at
//    72 x 72) and transforms both in-plane axes, lines going through small
//    ping-pong scratch buffers in LDS;
//  * an axis kernel transforms along N1, L neighbouring lines per workgroup
//    (the N2 * N3 lines of a grid taken as one range) so every global access
//    touches L consecutive values.
// Both run mixed-radix Stockham passes (autosort, no bit reversal) with
// twiddles from a per-axis table exp(-2 pi i k/n) computed on the host in
// long double: radices 2, 3, 4, 5 in the kernels for any length, and 8 and 9
// first (then 4, 2, 3, 5) in the compile-time kernels for the grid lengths
// in use, so 72 = 8 x 9 and 64 = 8 x 8 take two passes.
//
// Transforms between the wavefunction sphere and the grid are pruned: only
// the planes |n1| <= n1max that meet the sphere are built (the sphere scatter
// is fused into the plane kernel) or kept (the forward plane kernel writes
// only sphere entries, into a compact n_pw-per-grid array).
#include <cmath>
#include <cstdlib>
#include <cstring>

#include "common.h"

namespace bsex {

namespace f64 {
using real = double;
using cplx = double2;
__host__ __device__ __forceinline__ cplx mk(real a, real b) { return make_double2(a, b); }
#define BSEX_FFT_PREC 0
#define BSEX_FFT_TW(a) ((const cplx*)(a).tw)
#include "fft_impl.h"
#undef BSEX_FFT_PREC
#undef BSEX_FFT_TW
}  // namespace f64

namespace f32 {
using real = float;
using cplx = float2;
__host__ __device__ __forceinline__ cplx mk(real a, real b) { return make_float2(a, b); }
#define BSEX_FFT_PREC 1
#define BSEX_FFT_TW(a) ((const cplx*)(a).twf)
#include "fft_impl.h"
#undef BSEX_FFT_PREC
#undef BSEX_FFT_TW
}  // namespace f32

int fft_plan_init(FftPlan* p, const int grid[3]) {
  p->nr = 1;
  for (int a = 0; a < 3; ++a) {
    const int n = grid[a];
    if (n < 2 || n > 512) return fail(BSE_EINVAL, "FFT length %d unsupported", n);
    FftAxis& ax = p->ax[a];
    ax.n = n;
    ax.nrad = 0;
    int m = n;
    for (int r : {4, 2, 3, 5})
      while (m % r == 0) {
        if (ax.nrad >= 8) return fail(BSE_EINVAL, "FFT length %d has too many factors", n);
        ax.rad[ax.nrad++] = r;
        m /= r;
      }
    if (m != 1) return fail(BSE_EINVAL, "FFT length %d is not a product of 2, 3, 5", n);
    std::vector<double2> tw(n);
    std::vector<float2> twf(n);
    for (int k = 0; k < n; ++k) {
      const long double ang = -2.0L * 3.141592653589793238462643383279502884L * k / n;
      tw[k] = make_double2((double)cosl(ang), (double)sinl(ang));
      twf[k] = make_float2((float)cosl(ang), (float)sinl(ang));
    }
    BSE_HIP(hipMalloc(&ax.tw, sizeof(double2) * n));
    BSE_HIP(hipMalloc(&ax.twf, sizeof(float2) * n));
    HostStage hs;
    int rc = stage_h2d(&hs, tw.data(), ax.tw, sizeof(double2) * n, nullptr);
    if (rc == BSE_OK) rc = stage_h2d(&hs, twf.data(), ax.twf, sizeof(float2) * n, nullptr);
    stage_free(&hs);
    BSE_TRY(rc);
    p->N[a] = n;
    p->nr *= n;
  }
  int dev = 0;
  BSE_HIP(hipGetDevice(&dev));
  hipDeviceProp_t prop;
  BSE_HIP(hipGetDeviceProperties(&prop, dev));
  p->max_lds = prop.sharedMemPerBlock;
  BSE_TRY(f64::init_kernels(p));
  BSE_TRY(f32::init_kernels(p));
  return BSE_OK;
}

void fft_plan_set_runtime(FftPlan* p, bool runtime) {
  for (int q = 0; q < 2; ++q) {
    p->ct_plane[q] = p->ct_plane_ok[q] && !runtime;
    p->ct_axis[q] = p->ct_axis_ok[q] && !runtime;
  }
}

void fft_plan_free(FftPlan* p) {
  for (int a = 0; a < 3; ++a) {
    if (p->ax[a].tw) (void)hipFree(p->ax[a].tw);
    if (p->ax[a].twf) (void)hipFree(p->ax[a].twf);
    p->ax[a].tw = nullptr;
    p->ax[a].twf = nullptr;
  }
}

int sphere_plan_build(const FftPlan& p, const Basis& b, SpherePlan* sp) {
  const int N1 = p.N[0], N2 = p.N[1], N3 = p.N[2];
  const long np2 = (long)N2 * N3;
  struct Ent {
    int i1, pos, code;
  };
  std::vector<Ent> ents;
  ents.push_back({0, 0, 0});
  for (int k = 0; k < b.nhalf; ++k) {
    ents.push_back({(int)(b.idx_p[k] / np2), (int)(b.idx_p[k] % np2), k + 1});
    ents.push_back({(int)(b.idx_m[k] / np2), (int)(b.idx_m[k] % np2), -(k + 1)});
  }
  std::stable_sort(ents.begin(), ents.end(), [](const Ent& x, const Ent& y) {
    return x.i1 != y.i1 ? x.i1 < y.i1 : x.pos < y.pos;
  });
  std::vector<int> planes, off, pos(ents.size()), code(ents.size());
  std::vector<int> eplus(b.nhalf), eminus(b.nhalf), plane_sp(N1, -1);
  int ezero = 0, nmax1 = 0;
  sp->m2 = sp->m3 = 0;
  for (size_t e = 0; e < ents.size(); ++e) {
    if (planes.empty() || planes.back() != ents[e].i1) {
      plane_sp[ents[e].i1] = (int)planes.size();
      planes.push_back(ents[e].i1);
      off.push_back((int)e);
      const int n1 = (ents[e].i1 < (N1 + 1) / 2) ? ents[e].i1 : ents[e].i1 - N1;
      nmax1 = std::max(nmax1, std::abs(n1));
    }
    pos[e] = ents[e].pos;
    code[e] = ents[e].code;
    const int i2 = ents[e].pos / N3, i3 = ents[e].pos % N3;
    sp->m2 = std::max(sp->m2, std::abs(i2 < (N2 + 1) / 2 ? i2 : i2 - N2));
    sp->m3 = std::max(sp->m3, std::abs(i3 < (N3 + 1) / 2 ? i3 : i3 - N3));
    if (ents[e].code == 0) ezero = (int)e;
    else if (ents[e].code > 0) eplus[ents[e].code - 1] = (int)e;
    else eminus[-ents[e].code - 1] = (int)e;
  }
  off.push_back((int)ents.size());
  sp->nplanes = (int)planes.size();
  sp->nent = (int)ents.size();
  sp->e_zero = ezero;
  sp->nmax1 = nmax1;
  auto up = [](int** d, const std::vector<int>& h) -> int {
    BSE_HIP(hipMalloc(d, sizeof(int) * std::max<size_t>(h.size(), 1)));
    HostStage hs;
    const int rc = stage_h2d(&hs, h.data(), *d, sizeof(int) * h.size(), nullptr);
    stage_free(&hs);
    return rc;
  };
  BSE_TRY(up(&sp->plane_i1, planes));
  BSE_TRY(up(&sp->plane_off, off));
  BSE_TRY(up(&sp->ent_pos, pos));
  BSE_TRY(up(&sp->ent_code, code));
  BSE_TRY(up(&sp->e_plus, eplus));
  BSE_TRY(up(&sp->e_minus, eminus));
  BSE_TRY(up(&sp->plane_sp, plane_sp));
  return BSE_OK;
}

void sphere_plan_free(SpherePlan* sp) {
  int** ptrs[] = {&sp->plane_i1, &sp->plane_off, &sp->ent_pos, &sp->ent_code, &sp->e_plus,
                  &sp->e_minus, &sp->plane_sp};
  for (int** q : ptrs) {
    if (*q) (void)hipFree(*q);
    *q = nullptr;
  }
}

int fft3d(const FftPlan& p, double2* data, long batch, int dir, hipStream_t st) {
  return f64::fft3d(p, data, batch, dir, st);
}
int fft3d(const FftPlan& p, float2* data, long batch, int dir, hipStream_t st) {
  return f32::fft3d(p, data, batch, dir, st);
}
int fft3d_fwd_w(const FftPlan& p, const SpherePlan& sp, double2* data, long batch,
                const double* f, double s, double2* compact, hipStream_t st) {
  return f64::fft3d_fwd_w(p, sp, data, batch, f, s, compact, st);
}
int fft3d_fwd_w(const FftPlan& p, const SpherePlan& sp, float2* data, long batch, const float* f,
                float s, float2* compact, hipStream_t st) {
  return f32::fft3d_fwd_w(p, sp, data, batch, f, s, compact, st);
}
bool fwd_pairs_supported(const FftPlan& p, bool f32) {
  return f32 ? f32::fwd_pairs_supported(p) : f64::fwd_pairs_supported(p);
}
int fft3d_fwd_pairs(const FftPlan& p, const SpherePlan& sp, const double2* orb, int nv,
                    const int2* IJ, long nblk, double2* data, const double* f, double s,
                    double2* compact, hipStream_t st) {
  return f64::fft3d_fwd_pairs(p, sp, orb, nv, IJ, nblk, data, f, s, compact, st);
}
int fft3d_fwd_times(const FftPlan& p, const SpherePlan& sp, const double2* M, long nm,
                    const double2* x2, int xc, double2* data, const double* f, double s,
                    double2* compact, hipStream_t st) {
  return f64::fft3d_fwd_times(p, sp, M, nm, x2, xc, data, f, s, compact, st);
}
int fft3d_fwd_pairs(const FftPlan& p, const SpherePlan& sp, const float2* orb, int nv,
                    const int2* IJ, long nblk, float2* data, const float* f, float s,
                    float2* compact, hipStream_t st) {
  return f32::fft3d_fwd_pairs(p, sp, orb, nv, IJ, nblk, data, f, s, compact, st);
}
int sphere_to_grid(const FftPlan& p, const SpherePlan& sp, double omega, const double* X, int nv,
                   int nset, double2* grid, hipStream_t st) {
  return f64::sphere_to_grid(p, sp, omega, X, nv, nset, grid, st);
}
int sphere_to_grid(const FftPlan& p, const SpherePlan& sp, double omega, const double* X, int nv,
                   int nset, float2* grid, hipStream_t st) {
  return f32::sphere_to_grid(p, sp, omega, X, nv, nset, grid, st);
}
int grid_to_compact(const FftPlan& p, const SpherePlan& sp, double2* grid, long batch,
                    double2* compact, hipStream_t st) {
  return f64::grid_to_compact(p, sp, grid, batch, compact, st);
}
int grid_to_compact(const FftPlan& p, const SpherePlan& sp, float2* grid, long batch,
                    float2* compact, hipStream_t st) {
  return f32::grid_to_compact(p, sp, grid, batch, compact, st);
}

}  // namespace bsex
