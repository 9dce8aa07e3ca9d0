// Precision-generic part of the batched 3-D FFT.  Included once per
// precision inside a namespace that defines `real`, `cplx`, `mk(re, im)`,
// BSEX_FFT_PREC (0 FP64, 1 FP32) and BSEX_FFT_TW(axis) (its twiddle table).
namespace {

constexpr int kThreads = 256;
constexpr int kMaxN = 512;

struct AxisArgs {
  int n;
  int nrad;
  int rad[8];
  const cplx* tw;
};

#include "fft_codelets.h"

// One Stockham pass of radix R over L lines: element k of line l is read
// at in[k*iks + l*ils] and written at out[k*oks + l*ols].  Lines l >= nl
// are skipped.
template <int R, int DIR>
__device__ __forceinline__ void spass(const cplx* __restrict__ in, int iks, int ils,
                                      cplx* __restrict__ out, int oks, int ols, int n, int L,
                                      int nl, int ns, const cplx* __restrict__ tw, int nthr) {
  const int nq = n / R;
  const int tstride = n / (ns * R);
  for (int u = threadIdx.x; u < nq * L; u += nthr) {
    const int l = u % L;
    if (l >= nl) continue;
    const int j = u / L;
    const int k = j % ns;
    cplx v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      cplx x = in[(j + r * nq) * iks + l * ils];
      if (r > 0 && k > 0) {
        cplx w = tw[k * r * tstride];
        if (DIR > 0) w.y = -w.y;
        x = cmul(x, w);
      }
      v[r] = x;
    }
    if (R == 2) dft2<DIR>(v);
    if (R == 3) dft3<DIR>(v);
    if (R == 4) dft4<DIR>(v);
    if (R == 5) dft5<DIR>(v);
    const int base = (j / ns) * ns * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) out[(base + r * ns) * oks + l * ols] = v[r];
  }
}

template <int DIR>
__device__ __forceinline__ void spass_any(int R, const cplx* in, int iks, int ils, cplx* out,
                                          int oks, int ols, int n, int L, int nl, int ns,
                                          const cplx* tw, int nthr) {
  if (R == 4)
    spass<4, DIR>(in, iks, ils, out, oks, ols, n, L, nl, ns, tw, nthr);
  else if (R == 2)
    spass<2, DIR>(in, iks, ils, out, oks, ols, n, L, nl, ns, tw, nthr);
  else if (R == 3)
    spass<3, DIR>(in, iks, ils, out, oks, ols, n, L, nl, ns, tw, nthr);
  else
    spass<5, DIR>(in, iks, ils, out, oks, ols, n, L, nl, ns, tw, nthr);
}

// Transform all nlines lines of a plane held in LDS (element k of line l at
// P[k*ks + l*ls]), LB lines at a time: the first pass reads P, the middle
// passes ping-pong between the scratch buffers S0/S1 ([k][l] layout) and the
// last pass writes back into P.
template <int DIR>
__device__ void plane_lines(cplx* P, int ks, int ls, int nlines, const AxisArgs& ax,
                            cplx* S0, cplx* S1, int LB, int nthr) {
  const int n = ax.n;
  for (int l0 = 0; l0 < nlines; l0 += LB) {
    const int nl = min(LB, nlines - l0);
    cplx* base = P + l0 * ls;
    int ns = 1;
    const cplx* src = base;
    int iks = ks, ils = ls;
    cplx* bufs[2] = {S0, S1};
    int which = 0;
    for (int p = 0; p < ax.nrad; ++p) {
      const bool last = (p == ax.nrad - 1);
      cplx* dst = last ? base : bufs[which];
      const int oks = last ? ks : LB, ols = last ? ls : 1;
      if (ax.nrad == 1) {  // single pass cannot run in place: go through S0
        spass_any<DIR>(ax.rad[p], src, iks, ils, S0, LB, 1, n, LB, nl, ns, ax.tw, nthr);
        __syncthreads();
        for (int e = threadIdx.x; e < n * LB; e += nthr) {
          const int k = e / LB, l = e % LB;
          if (l < nl) base[k * ks + l * ls] = S0[e];
        }
        __syncthreads();
        break;
      }
      spass_any<DIR>(ax.rad[p], src, iks, ils, dst, oks, ols, n, LB, nl, ns, ax.tw, nthr);
      __syncthreads();
      ns *= ax.rad[p];
      src = dst;
      iks = LB;
      ils = 1;
      which ^= 1;
    }
  }
}

// Strided single-axis pass.  Lines: base = o1 * s_o1 + o2 * s_o2 + inner * s_in,
// elements at base + k * es.  A workgroup takes L consecutive inner lines of
// one (o1, o2).  Elements with |n(k)| > ld_lim are not read (taken as zero)
// and elements with |n(k)| > st_lim are not written (n = minimum image of k).
template <int DIR>
__global__ __launch_bounds__(kThreads) void k_fft_axis(cplx* __restrict__ data, AxisArgs ax,
                                                       int es, int n_inner, long s_in, int n_o2,
                                                       long s_o2, long s_o1, int L, int ld_lim,
                                                       int st_lim) {
  extern __shared__ cplx lds[];
  const int n = ax.n;
  cplx* b0 = lds;
  cplx* b1 = lds + (long)n * L;
  const int tiles = (n_inner + L - 1) / L;
  long w = blockIdx.x;
  const int tile = (int)(w % tiles);
  w /= tiles;
  const int o2 = (int)(w % n_o2);
  const long o1 = w / n_o2;
  const int i0 = tile * L;
  const int nl = min(L, n_inner - i0);
  cplx* base = data + o1 * s_o1 + (long)o2 * s_o2 + (long)i0 * s_in;
  const bool contiguous = (es == 1);
  for (int e = threadIdx.x; e < n * L; e += kThreads) {
    int k, l;
    if (contiguous) {
      l = e / n;
      k = e % n;
    } else {
      k = e / L;
      l = e % L;
    }
    const int nk = (k < (n + 1) / 2) ? k : k - n;
    cplx x = mk(0.0, 0.0);
    if (l < nl && abs(nk) <= ld_lim) x = base[(long)l * s_in + (long)k * es];
    b0[k * L + l] = x;
  }
  __syncthreads();
  int ns = 1;
  cplx* src = b0;
  cplx* dst = b1;
  for (int p = 0; p < ax.nrad; ++p) {
    spass_any<DIR>(ax.rad[p], src, L, 1, dst, L, 1, n, L, L, ns, ax.tw, kThreads);
    ns *= ax.rad[p];
    __syncthreads();
    cplx* t = src;
    src = dst;
    dst = t;
  }
  for (int e = threadIdx.x; e < n * L; e += kThreads) {
    int k, l;
    if (contiguous) {
      l = e / n;
      k = e % n;
    } else {
      k = e / L;
      l = e % L;
    }
    const int nk = (k < (n + 1) / 2) ? k : k - n;
    if (l < nl && abs(nk) <= st_lim) base[(long)l * s_in + (long)k * es] = src[k * L + l];
  }
}

// Both in-plane axes (2 and 3) of one N2 x N3 plane (fixed i1) in LDS.
// IN = 0: the plane is read from the grid; IN = 1: it is built from sphere
// coefficients (two real orbitals per grid, entries of this plane only).
// OUT = 0: the plane is written back; OUT = 1: only its sphere entries are
// written to the compact array (n_pw complex values per grid).
constexpr int kPlaneThreads = 512;

struct PlaneArgs {
  int N1, N2, N3;
  long nr;
  int nplanes;            // planes per grid processed
  const int* plane_i1;    // NULL: plane p is i1 = p
  const int* plane_off;   // [nplanes + 1] entry ranges (sphere modes)
  const int* ent_pos;     // in-plane position i2 * N3 + i3
  const int* ent_code;    // 0: G = 0; k + 1: +G_k; -(k + 1): -G_k
  int nent;               // entries per grid (= n_pw)
  const double* X;        // sphere input [set][nv][npw]
  int nv, nvh, npw;
  double s0, s1;          // 1/sqrt(Omega), 1/sqrt(2 Omega)
  cplx* compact;       // [grid][nent]
  int LB;                 // lines per scratch batch
  int m2, m3;             // the sphere's modes have |n2| <= m2 and |n3| <= m3
  long batch;             // grids (pruned inverse kernel: workgroups beyond are idle)
  int group;              // pruned inverse kernel: the planes of a grid on one XCD
  const int* plane_sp;    // OUT == 2: [N1] sphere plane of grid plane i1 (-1: none)
  const real* mulf;       // OUT == 2: real field the plane leaves multiplied by (NULL: 0)
  real muls;              //           and its scale
};

// OUT == 2 (forward transform of a W build): the finished plane P of grid g
// goes back times mulf * muls, and its sphere entries, unscaled, to the
// compact output when one is set
__device__ __forceinline__ void plane_store_w(const cplx* P, cplx* gp, const PlaneArgs& pa,
                                              long g, int i1, int np2, int nt) {
  const real* f = pa.mulf ? pa.mulf + (long)i1 * np2 : nullptr;
  for (int e = threadIdx.x; e < np2; e += nt) {
    cplx x = mk(0.0, 0.0);  // no bare part: exact zeros, as a fill would leave
    if (f) {
      const real m = f[e] * pa.muls;
      x = P[e];
      x.x *= m;
      x.y *= m;
    }
    gp[e] = x;
  }
  if (pa.compact) {
    const int sp = pa.plane_sp[i1];
    if (sp >= 0) {
      cplx* cg = pa.compact + g * (long)pa.nent;
      for (int e = pa.plane_off[sp] + threadIdx.x; e < pa.plane_off[sp + 1]; e += nt)
        cg[e] = P[pa.ent_pos[e]];
    }
  }
}

template <int DIR, int IN, int OUT>
__global__ __launch_bounds__(kPlaneThreads) void k_fft_plane(cplx* data, PlaneArgs pa,
                                                              AxisArgs ay, AxisArgs az) {
  extern __shared__ cplx lds[];
  const int N2 = pa.N2, N3 = pa.N3, np2 = N2 * N3;
  cplx* P = lds;
  const int nmax = max(N2, N3);
  cplx* S0 = P + np2;
  cplx* S1 = S0 + (long)pa.LB * nmax;
  const long g = blockIdx.x / pa.nplanes;
  const int pl = (int)(blockIdx.x % pa.nplanes);
  const int i1 = pa.plane_i1 ? pa.plane_i1[pl] : pl;
  cplx* gp = data + g * pa.nr + (long)i1 * np2;
  if (IN == 0) {
    for (int e = threadIdx.x; e < np2; e += kPlaneThreads) P[e] = gp[e];
  } else {
    for (int e = threadIdx.x; e < np2; e += kPlaneThreads) P[e] = mk(0.0, 0.0);
    __syncthreads();
    const long set = g / pa.nvh;
    const int p = (int)(g % pa.nvh);
    const double* x1 = pa.X + (set * pa.nv + 2 * p) * (long)pa.npw;
    const double* x2 = (2 * p + 1 < pa.nv) ? x1 + pa.npw : nullptr;
    for (int e = pa.plane_off[pl] + threadIdx.x; e < pa.plane_off[pl + 1]; e += kPlaneThreads) {
      const int code = pa.ent_code[e];
      cplx h;
      if (code == 0) {
        h = mk(x1[0] * pa.s0, x2 ? x2[0] * pa.s0 : 0.0);
      } else {
        const int k = abs(code) - 1;
        const double c1 = x1[1 + 2 * k], q1 = x1[2 + 2 * k];
        const double c2 = x2 ? x2[1 + 2 * k] : 0.0, q2 = x2 ? x2[2 + 2 * k] : 0.0;
        h = code > 0 ? mk((c1 + q2) * pa.s1, (c2 - q1) * pa.s1)
                     : mk((c1 - q2) * pa.s1, (q1 + c2) * pa.s1);
      }
      P[pa.ent_pos[e]] = h;
    }
  }
  __syncthreads();
  // axis 3 (rows, contiguous) and axis 2 (columns, stride N3)
  plane_lines<DIR>(P, 1, N3, N2, az, S0, S1, pa.LB, kPlaneThreads);
  plane_lines<DIR>(P, N3, 1, N3, ay, S0, S1, pa.LB, kPlaneThreads);
  if (OUT == 0) {
    for (int e = threadIdx.x; e < np2; e += kPlaneThreads) gp[e] = P[e];
  } else if (OUT == 2) {
    plane_store_w(P, gp, pa, g, i1, np2, kPlaneThreads);
  } else {
    cplx* cg = pa.compact + g * (long)pa.nent;
    for (int e = pa.plane_off[pl] + threadIdx.x; e < pa.plane_off[pl + 1]; e += kPlaneThreads)
      cg[e] = P[pa.ent_pos[e]];
  }
}

// ---------------------------------------------------------------------------
// Compile-time versions for the grid lengths in use: the factorisation,
// pass strides, line counts and LDS strides are constants, so all index
// arithmetic reduces to shifts and constant multiplies.
// ---------------------------------------------------------------------------
struct Fac {
  int n;
  int r[8];
};
constexpr Fac factor(int N) {
  Fac f{0, {0, 0, 0, 0, 0, 0, 0, 0}};
  int m = N;
  // radix 8 and 9 first: fewer passes through LDS (72 = 8 x 9, 64 = 8 x 8)
  const int rs[6] = {8, 4, 2, 9, 3, 5};
  for (int q = 0; q < 6; ++q)
    while (m % rs[q] == 0) {
      f.r[f.n++] = rs[q];
      m /= rs[q];
    }
  return f;
}

template <int R, int DIR, int N, int NS, int L, int IKS, int ILS, int OKS, int OLS, int NT>
__device__ __forceinline__ void spass_ct(const cplx* __restrict__ in, cplx* __restrict__ out,
                                         int nl, const cplx* __restrict__ tw) {
  constexpr int NQ = N / R;
  constexpr int TS = N / (NS * R);
#pragma unroll 2
  for (int u = threadIdx.x; u < NQ * L; u += NT) {
    const int l = u % L;
    if (l >= nl) continue;
    const int j = u / L;
    const int k = j % NS;
    cplx v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      cplx x = in[(j + r * NQ) * IKS + l * ILS];
      if (r > 0 && NS > 1) {
        cplx w = tw[k * r * TS];
        if (DIR > 0) w.y = -w.y;
        x = cmul(x, w);
      }
      v[r] = x;
    }
    if (R == 2) dft2<DIR>(v);
    if (R == 3) dft3<DIR>(v);
    if (R == 4) dft4<DIR>(v);
    if (R == 5) dft5<DIR>(v);
    if (R == 8) dft8<DIR>(v);
    if (R == 9) dft9<DIR>(v);
    const int base = (j / NS) * NS * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) out[(base + r * NS) * OKS + l * OLS] = v[r];
  }
}

// Passes P.. of a length-N transform of L lines: the first reads `src`
// with strides (IKS, ILS); intermediate results ping-pong between S0 and S1
// ([k][l] layout); the last pass writes `dst` with strides (OKS, OLS).
template <int N, int DIR, int L, int NT, int P, int NS, int IKS, int ILS, int OKS, int OLS>
__device__ __forceinline__ void ct_passes(const cplx* src, cplx* S0, cplx* S1,
                                          cplx* dst, int nl, const cplx* tw) {
  constexpr Fac F = factor(N);
  if constexpr (P < F.n) {
    constexpr int R = F.r[P];
    constexpr bool last = (P == F.n - 1);
    constexpr int oks = last ? OKS : L;
    constexpr int ols = last ? OLS : 1;
    cplx* out = last ? dst : ((P % 2 == 0) ? S0 : S1);
    spass_ct<R, DIR, N, NS, L, IKS, ILS, oks, ols, NT>(src, out, nl, tw);
    __syncthreads();
    ct_passes<N, DIR, L, NT, P + 1, NS * R, L, 1, OKS, OLS>(out, S0, S1, dst, nl, tw);
  }
}

// Scratch buffers of a plane: line transforms of at most two passes go
// P -> S0 -> P, longer ones also use S1.
template <int N2, int N3>
constexpr int plane_nscratch() {
  return (factor(N2).n <= 2 && factor(N3).n <= 2) ? 1 : 2;
}

template <int N2, int N3>
constexpr int plane_lb() {
  const int nmax = N2 > N3 ? N2 : N3;
  const int ns = plane_nscratch<N2, N3>();
  if (N2 == N3 && ns == 1) {
    // one scratch buffer: the largest divisor of N (at most 64) whose batch
    // fits 160 KB in FP64 and 80 KB in FP32 (two workgroups per CU), so a
    // plane takes few equal batches (72: 2 x 36)
    const int budget = sizeof(cplx) == 16 ? 163840 : 81920;
    for (int d = 64; d >= 4; --d)
      if (N2 % d == 0 && (int)sizeof(cplx) * (N2 * N3 + d * nmax) <= budget) return d;
  }
  // lines per scratch batch: largest power of two (<= 32) fitting 160 KB; in
  // FP32 at least 16 lines within 80 KB when that fits, for two workgroups
  // per CU (48 x 120: 16 lines, 77 KB, instead of 32 lines, 107 KB)
  if (sizeof(cplx) == 8 && (int)sizeof(cplx) * (N2 * N3 + ns * 16 * nmax) <= 81920) {
    int lb = 32;
    while (lb > 16 && (int)sizeof(cplx) * (N2 * N3 + ns * lb * nmax) > 81920) lb /= 2;
    return lb;
  }
  int lb = 32;
  while (lb > 4 && (int)sizeof(cplx) * (N2 * N3 + ns * lb * nmax) > 163840) lb /= 2;
  return lb;
}

template <int N2, int N3>
constexpr int plane_lds_bytes() {
  const int nmax = N2 > N3 ? N2 : N3;
  return (int)sizeof(cplx) * (N2 * N3 + plane_nscratch<N2, N3>() * plane_lb<N2, N3>() * nmax);
}

template <int N2, int N3, int DIR, int IN, int OUT>
__global__ __launch_bounds__(kPlaneThreads) void k_fft_plane_ct(cplx* data, PlaneArgs pa,
                                                                 AxisArgs ay, AxisArgs az) {
  constexpr int NP2 = N2 * N3;
  constexpr int LB = plane_lb<N2, N3>();
  constexpr int NM = N2 > N3 ? N2 : N3;
  constexpr int NT = kPlaneThreads;
  static_assert(factor(N2).n >= 2 && factor(N3).n >= 2, "plane lengths need two passes");
  extern __shared__ cplx lds[];
  cplx* P = lds;
  cplx* S0 = P + NP2;
  // with one scratch buffer S1 is never used: alias it to S0
  cplx* S1 = plane_nscratch<N2, N3>() == 2 ? S0 + LB * NM : S0;
  const long g = blockIdx.x / pa.nplanes;
  const int pl = (int)(blockIdx.x % pa.nplanes);
  const int i1 = pa.plane_i1 ? pa.plane_i1[pl] : pl;
  cplx* gp = data + g * pa.nr + (long)i1 * NP2;
  if (IN == 0) {
#pragma unroll 4
    for (int e = threadIdx.x; e < NP2; e += NT) P[e] = gp[e];
  } else {
    for (int e = threadIdx.x; e < NP2; e += NT) P[e] = mk(0.0, 0.0);
    __syncthreads();
    const long set = g / pa.nvh;
    const int p = (int)(g % pa.nvh);
    const double* x1 = pa.X + (set * pa.nv + 2 * p) * (long)pa.npw;
    const double* x2 = (2 * p + 1 < pa.nv) ? x1 + pa.npw : nullptr;
    for (int e = pa.plane_off[pl] + threadIdx.x; e < pa.plane_off[pl + 1]; e += NT) {
      const int code = pa.ent_code[e];
      cplx h;
      if (code == 0) {
        h = mk(x1[0] * pa.s0, x2 ? x2[0] * pa.s0 : 0.0);
      } else {
        const int k = abs(code) - 1;
        const double c1 = x1[1 + 2 * k], q1 = x1[2 + 2 * k];
        const double c2 = x2 ? x2[1 + 2 * k] : 0.0, q2 = x2 ? x2[2 + 2 * k] : 0.0;
        h = code > 0 ? mk((c1 + q2) * pa.s1, (c2 - q1) * pa.s1)
                     : mk((c1 - q2) * pa.s1, (q1 + c2) * pa.s1);
      }
      P[pa.ent_pos[e]] = h;
    }
  }
  __syncthreads();
  // rows (axis 3): element stride 1, line stride N3
#pragma unroll 1
  for (int l0 = 0; l0 < N2; l0 += LB)
    ct_passes<N3, DIR, LB, NT, 0, 1, 1, N3, 1, N3>(P + l0 * N3, S0, S1, P + l0 * N3,
                                                  min(LB, N2 - l0), az.tw);
  // columns (axis 2): element stride N3, line stride 1
#pragma unroll 1
  for (int l0 = 0; l0 < N3; l0 += LB)
    ct_passes<N2, DIR, LB, NT, 0, 1, N3, 1, N3, 1>(P + l0, S0, S1, P + l0, min(LB, N3 - l0), ay.tw);
  if (OUT == 0) {
#pragma unroll 4
    for (int e = threadIdx.x; e < NP2; e += NT) gp[e] = P[e];
  } else if (OUT == 2) {
    plane_store_w(P, gp, pa, g, i1, NP2, NT);
  } else {
    cplx* cg = pa.compact + g * (long)pa.nent;
    for (int e = pa.plane_off[pl] + threadIdx.x; e < pa.plane_off[pl + 1]; e += NT)
      cg[e] = P[pa.ent_pos[e]];
  }
}

// ---------------------------------------------------------------------------
// Pruned sphere-plane transforms (compile-time lengths).  The sphere's modes
// occupy rows |n2| <= m2 and columns |n3| <= m3 of a plane, so
//  inverse (sphere -> plane): row transforms only on the 2 m2 + 1 rows that
//    hold modes, kept in a compact block Q; then every column is transformed
//    reading Q (zeros elsewhere) and its last pass writes the plane straight
//    to memory, LB adjacent columns per batch (coalesced rows of LB values);
//  forward (plane -> sphere): rows staged from memory in batches by
//    coalesced copies and transformed, keeping only the 2 m3 + 1 columns that
//    hold modes in Q; then those columns are transformed in place and the
//    plane's modes gathered from Q.
// Q holds (2 m2 + 1) x N3 or N2 x (2 m3 + 1) values instead of the whole
// plane, so at 72 x 72 in FP64 two workgroups share a CU.
// ---------------------------------------------------------------------------
// one Stockham pass with functor access: element k of line l is read by
// ld(k, l) and written by st(k, l, value)
template <int R, int DIR, int N, int NS, int L, int NT, class LD, class ST>
__device__ __forceinline__ void spass_fn(LD ld, ST st, int nl, const cplx* __restrict__ tw) {
  constexpr int NQ = N / R;
  constexpr int TS = N / (NS * R);
#pragma unroll 2
  for (int u = threadIdx.x; u < NQ * L; u += NT) {
    const int l = u % L;
    if (l >= nl) continue;
    const int j = u / L;
    const int k = j % NS;
    cplx v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      cplx x = ld(j + r * NQ, l);
      if (r > 0 && NS > 1) {
        cplx w = tw[k * r * TS];
        if (DIR > 0) w.y = -w.y;
        x = cmul(x, w);
      }
      v[r] = x;
    }
    if (R == 2) dft2<DIR>(v);
    if (R == 3) dft3<DIR>(v);
    if (R == 4) dft4<DIR>(v);
    if (R == 5) dft5<DIR>(v);
    if (R == 8) dft8<DIR>(v);
    if (R == 9) dft9<DIR>(v);
    const int base = (j / NS) * NS * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) st(base + r * NS, l, v[r]);
  }
}

// passes P.. of a length-N transform of L lines: the first reads through ld,
// intermediate results ping-pong between S0 and S1 ([k][l] layout), the last
// writes through st
template <int N, int DIR, int L, int NT, int P, int NS, class LD, class ST>
__device__ __forceinline__ void fn_passes(LD ld, ST st, cplx* S0, cplx* S1, int nl,
                                          const cplx* tw) {
  constexpr Fac F = factor(N);
  if constexpr (P < F.n) {
    constexpr int R = F.r[P];
    if constexpr (P == F.n - 1) {
      spass_fn<R, DIR, N, NS, L, NT>(ld, st, nl, tw);
      __syncthreads();
    } else {
      cplx* out = (P % 2 == 0) ? S0 : S1;
      spass_fn<R, DIR, N, NS, L, NT>(
          ld, [out](int k, int l, cplx v) { out[k * L + l] = v; }, nl, tw);
      __syncthreads();
      fn_passes<N, DIR, L, NT, P + 1, NS * R>(
          [out](int k, int l) { return out[k * L + l]; }, st, S0, S1, nl, tw);
    }
  }
}

__device__ __forceinline__ int min_img(int i, int n) { return i < (n + 1) / 2 ? i : i - n; }

// lines per batch of the pruned kernels: three candidates per precision for
// the inverse pass, the first two for the forward pass (the launch scores
// them, below)
constexpr int kSphereLB[3] = {sizeof(cplx) == 16 ? 16 : 32, sizeof(cplx) == 16 ? 18 : 36,
                              sizeof(cplx) == 16 ? 36 : 56};

// LDS of the pruned kernels for sphere extents m2, m3 and batch LB
template <int N2, int N3>
size_t sphere_inv_lds(int m2, int lb) {
  constexpr int nm = N2 > N3 ? N2 : N3;
  return sizeof(cplx) * ((size_t)(2 * m2 + 1) * N3 + (size_t)plane_nscratch<N2, N3>() * nm * lb);
}
template <int N2, int N3>
size_t sphere_fwd_whole_lds(int lb) {
  constexpr int nm = N2 > N3 ? N2 : N3;
  return sizeof(cplx) * ((size_t)N2 * N3 + (size_t)plane_nscratch<N2, N3>() * nm * lb);
}
template <int N2, int N3>
size_t sphere_fwd_lds(int m3, int lb) {
  constexpr int nm = N2 > N3 ? N2 : N3;
  return sizeof(cplx) * ((size_t)N2 * (2 * m3 + 1) + (size_t)plane_nscratch<N2, N3>() * nm * lb +
                         (size_t)lb * N3);
}

template <int N2, int N3, int DIR, int LB>
__global__ __launch_bounds__(kPlaneThreads) void k_sphere_inv_ct(cplx* data, PlaneArgs pa,
                                                                  AxisArgs ay, AxisArgs az) {
  constexpr int NM = N2 > N3 ? N2 : N3;
  constexpr int NT = kPlaneThreads;
  static_assert(factor(N2).n >= 2 && factor(N3).n >= 2, "plane lengths need two passes");
  extern __shared__ cplx lds[];
  const int m2 = pa.m2, K2 = 2 * pa.m2 + 1;
  cplx* Q = lds;                       // [K2][N3]
  cplx* S0 = Q + K2 * N3;
  cplx* S1 = plane_nscratch<N2, N3>() == 2 ? S0 + NM * LB : S0;
  // the planes of one grid share its coefficient rows: with pa.group they
  // run on one XCD and read those rows into one L2
  long g;
  int pl;
  xcd_item(blockIdx.x, pa.nplanes, pa.group != 0, g, pl);
  if (g >= pa.batch) return;
  const int i1 = pa.plane_i1[pl];
  cplx* gp = data + g * pa.nr + (long)i1 * (N2 * N3);
  for (int e = threadIdx.x; e < K2 * N3; e += NT) Q[e] = mk(0.0, 0.0);
  __syncthreads();
  {
    const long set = g / pa.nvh;
    const int p = (int)(g % pa.nvh);
    const double* x1 = pa.X + (set * pa.nv + 2 * p) * (long)pa.npw;
    const double* x2 = (2 * p + 1 < pa.nv) ? x1 + pa.npw : nullptr;
    for (int e = pa.plane_off[pl] + threadIdx.x; e < pa.plane_off[pl + 1]; e += NT) {
      const int code = pa.ent_code[e];
      cplx h;
      if (code == 0) {
        h = mk(x1[0] * pa.s0, x2 ? x2[0] * pa.s0 : 0.0);
      } else {
        const int k = abs(code) - 1;
        const double c1 = x1[1 + 2 * k], q1 = x1[2 + 2 * k];
        const double c2 = x2 ? x2[1 + 2 * k] : 0.0, q2 = x2 ? x2[2 + 2 * k] : 0.0;
        h = code > 0 ? mk((c1 + q2) * pa.s1, (c2 - q1) * pa.s1)
                     : mk((c1 - q2) * pa.s1, (q1 + c2) * pa.s1);
      }
      const int pos = pa.ent_pos[e];
      const int q = min_img(pos / N3, N2) + m2;
      Q[q * N3 + pos % N3] = h;
    }
  }
  __syncthreads();
  // rows holding modes (axis 3), in place in Q
#pragma unroll 1
  for (int l0 = 0; l0 < K2; l0 += LB)
    ct_passes<N3, DIR, LB, NT, 0, 1, 1, N3, 1, N3>(Q + l0 * N3, S0, S1, Q + l0 * N3,
                                                  min(LB, K2 - l0), az.tw);
  // every column (axis 2) from Q, zeros outside its rows; the last pass
  // writes the plane
#pragma unroll 1
  for (int l0 = 0; l0 < N3; l0 += LB) {
    auto ld = [=](int k, int l) -> cplx {
      const int q = min_img(k, N2) + m2;
      return (q >= 0 && q < K2) ? Q[q * N3 + l0 + l] : mk(0.0, 0.0);
    };
    auto st = [=](int k, int l, cplx v) { gp[k * N3 + l0 + l] = v; };
    fn_passes<N2, DIR, LB, NT, 0, 1>(ld, st, S0, S1, min(LB, N3 - l0), ay.tw);
  }
}

template <int N2, int N3, int DIR, int LB>
__global__ __launch_bounds__(kPlaneThreads) void k_sphere_fwd_ct(cplx* data, PlaneArgs pa,
                                                                  AxisArgs ay, AxisArgs az) {
  constexpr int NM = N2 > N3 ? N2 : N3;
  constexpr int NT = kPlaneThreads;
  static_assert(factor(N2).n >= 2 && factor(N3).n >= 2, "plane lengths need two passes");
  extern __shared__ cplx lds[];
  const int m3 = pa.m3, K3 = 2 * pa.m3 + 1;
  cplx* Q = lds;                       // [N2][K3]
  cplx* S0 = Q + N2 * K3;
  cplx* S1 = plane_nscratch<N2, N3>() == 2 ? S0 + NM * LB : S0;
  cplx* R0 = S0 + plane_nscratch<N2, N3>() * NM * LB;  // staged rows [LB][N3]
  const long g = blockIdx.x / pa.nplanes;
  const int pl = (int)(blockIdx.x % pa.nplanes);
  const int i1 = pa.plane_i1[pl];
  const cplx* gp = data + g * pa.nr + (long)i1 * (N2 * N3);
  // rows (axis 3): staged by coalesced copies, only the columns holding
  // modes kept
#pragma unroll 1
  for (int l0 = 0; l0 < N2; l0 += LB) {
    const int nl = min(LB, N2 - l0);
    for (int e = threadIdx.x; e < nl * N3; e += NT) R0[e] = gp[l0 * N3 + e];
    __syncthreads();
    auto ld = [=](int k, int l) { return R0[l * N3 + k]; };
    auto st = [=](int k, int l, cplx v) {
      const int q = min_img(k, N3) + m3;
      if (q >= 0 && q < K3) Q[(l0 + l) * K3 + q] = v;
    };
    fn_passes<N3, DIR, LB, NT, 0, 1>(ld, st, S0, S1, nl, az.tw);
  }
  // the kept columns (axis 2), in place in Q
#pragma unroll 1
  for (int l0 = 0; l0 < K3; l0 += LB) {
    auto ld = [=](int k, int l) { return Q[k * K3 + l0 + l]; };
    auto st = [=](int k, int l, cplx v) { Q[k * K3 + l0 + l] = v; };
    fn_passes<N2, DIR, LB, NT, 0, 1>(ld, st, S0, S1, min(LB, K3 - l0), ay.tw);
  }
  cplx* cg = pa.compact + g * (long)pa.nent;
  for (int e = pa.plane_off[pl] + threadIdx.x; e < pa.plane_off[pl + 1]; e += NT) {
    const int pos = pa.ent_pos[e];
    cg[e] = Q[(pos / N3) * K3 + min_img(pos % N3, N3) + m3];
  }
}

// The forward pass with the whole plane in LDS (one coalesced load of all
// rows, row transforms in place), then only the 2 m3 + 1 columns that hold
// modes transformed in place: for planes whose LDS fits two workgroups per
// CU this beats staging rows in batches.
template <int N2, int N3, int DIR, int LB>
__global__ __launch_bounds__(kPlaneThreads) void k_sphere_fwd_whole(cplx* data, PlaneArgs pa,
                                                                     AxisArgs ay, AxisArgs az) {
  constexpr int NP2 = N2 * N3;
  constexpr int NM = N2 > N3 ? N2 : N3;
  constexpr int NT = kPlaneThreads;
  static_assert(factor(N2).n >= 2 && factor(N3).n >= 2, "plane lengths need two passes");
  extern __shared__ cplx lds[];
  const int m3 = pa.m3, K3 = 2 * pa.m3 + 1;
  cplx* P = lds;
  cplx* S0 = P + NP2;
  cplx* S1 = plane_nscratch<N2, N3>() == 2 ? S0 + NM * LB : S0;
  const long g = blockIdx.x / pa.nplanes;
  const int pl = (int)(blockIdx.x % pa.nplanes);
  const int i1 = pa.plane_i1[pl];
  const cplx* gp = data + g * pa.nr + (long)i1 * NP2;
#pragma unroll 4
  for (int e = threadIdx.x; e < NP2; e += NT) P[e] = gp[e];
  __syncthreads();
#pragma unroll 1
  for (int l0 = 0; l0 < N2; l0 += LB)
    ct_passes<N3, DIR, LB, NT, 0, 1, 1, N3, 1, N3>(P + l0 * N3, S0, S1, P + l0 * N3,
                                                  min(LB, N2 - l0), az.tw);
  // column l of the kept set is n3 = l - m3, stored at index (l - m3) mod N3
#pragma unroll 1
  for (int l0 = 0; l0 < K3; l0 += LB) {
    auto col = [=](int l) { const int n = l0 + l - m3; return n < 0 ? n + N3 : n; };
    auto ld = [=](int k, int l) { return P[k * N3 + col(l)]; };
    auto st = [=](int k, int l, cplx v) { P[k * N3 + col(l)] = v; };
    fn_passes<N2, DIR, LB, NT, 0, 1>(ld, st, S0, S1, min(LB, K3 - l0), ay.tw);
  }
  cplx* cg = pa.compact + g * (long)pa.nent;
  for (int e = pa.plane_off[pl] + threadIdx.x; e < pa.plane_off[pl + 1]; e += NT)
    cg[e] = P[pa.ent_pos[e]];
}

template <int N>
constexpr int axis_l() {
  int L = 32;
  while (L > 4 && 2 * (int)sizeof(cplx) * N * L > 40960) L /= 2;
  return L;
}

template <int N, int DIR>
__global__ __launch_bounds__(kThreads) void k_fft_axis_ct(cplx* __restrict__ data, AxisArgs ax,
                                                          int es, int n_inner, long s_in, int n_o2,
                                                          long s_o2, long s_o1, int ld_lim,
                                                          int st_lim) {
  constexpr int L = axis_l<N>();
  constexpr Fac F = factor(N);
  static_assert(F.n >= 1, "");
  extern __shared__ cplx lds[];
  cplx* b0 = lds;
  cplx* b1 = lds + N * L;
  const int tiles = (n_inner + L - 1) / L;
  long w = blockIdx.x;
  const int tile = (int)(w % tiles);
  w /= tiles;
  const int o2 = (int)(w % n_o2);
  const long o1 = w / n_o2;
  const int i0 = tile * L;
  const int nl = min(L, n_inner - i0);
  cplx* base = data + o1 * s_o1 + (long)o2 * s_o2 + (long)i0 * s_in;
#pragma unroll 4
  for (int e = threadIdx.x; e < N * L; e += kThreads) {
    const int k = e / L, l = e % L;
    const int nk = (k < (N + 1) / 2) ? k : k - N;
    cplx x = mk(0.0, 0.0);
    if (l < nl && abs(nk) <= ld_lim) x = base[(long)l * s_in + (long)k * es];
    b0[e] = x;
  }
  __syncthreads();
  // passes ping-pong b0 -> b1 -> b0 ...; the result lands in b0 or b1
  cplx* res = (F.n % 2 == 1) ? b1 : b0;
  cplx* other = (F.n % 2 == 1) ? b0 : b1;
  // all passes use the [k][l] layout; the last writes `res`
  ct_passes<N, DIR, L, kThreads, 0, 1, L, 1, L, 1>(b0, b1, b0, res, L, ax.tw);
  (void)other;
#pragma unroll 4
  for (int e = threadIdx.x; e < N * L; e += kThreads) {
    const int k = e / L, l = e % L;
    const int nk = (k < (N + 1) / 2) ? k : k - N;
    if (l < nl && abs(nk) <= st_lim) base[(long)l * s_in + (long)k * es] = res[e];
  }
}

// Axis pass with direct memory access: the first Stockham pass reads the
// grid and the last writes it, so only the intermediate results pass through
// LDS (one buffer for a two-pass length).  Lines per workgroup: the largest
// power of two (at most 32) that gives every thread at most one butterfly of
// the first pass.  In place is safe: every element of the tile is read in the
// first pass, which a barrier separates from the last.  Lengths of one pass
// keep the staged kernel.
template <int N>
constexpr int axis_gd_l() {
  constexpr Fac F = factor(N);
  int L = 32;
  while (L > 4 && (N / F.r[0]) * L > kThreads) L /= 2;
  return L;
}
template <int N>
constexpr bool axis_gd_ok() {
  return factor(N).n >= 2;
}
template <int N>
constexpr size_t axis_gd_lds() {
  return (factor(N).n >= 3 ? 2 : 1) * sizeof(cplx) * (size_t)N * axis_gd_l<N>();
}

template <int N, int DIR>
__global__ __launch_bounds__(kThreads) void k_fft_axis_gd(cplx* __restrict__ data, AxisArgs ax,
                                                          int es, int n_inner, long s_in, int n_o2,
                                                          long s_o2, long s_o1, int ld_lim,
                                                          int st_lim) {
  constexpr int L = axis_gd_l<N>();
  static_assert(factor(N).n >= 2, "");
  extern __shared__ cplx lds[];
  cplx* S0 = lds;
  cplx* S1 = lds + N * L;
  const int tiles = (n_inner + L - 1) / L;
  long w = blockIdx.x;
  const int tile = (int)(w % tiles);
  w /= tiles;
  const int o2 = (int)(w % n_o2);
  const long o1 = w / n_o2;
  const int i0 = tile * L;
  const int nl = min(L, n_inner - i0);
  cplx* base = data + o1 * s_o1 + (long)o2 * s_o2 + (long)i0 * s_in;
  auto ld = [=](int k, int l) {
    const int nk = (k < (N + 1) / 2) ? k : k - N;
    cplx x = mk(0.0, 0.0);
    if (abs(nk) <= ld_lim) x = base[(long)l * s_in + (long)k * es];
    return x;
  };
  auto st = [=](int k, int l, cplx v) {
    const int nk = (k < (N + 1) / 2) ? k : k - N;
    if (abs(nk) <= st_lim) base[(long)l * s_in + (long)k * es] = v;
  };
  fn_passes<N, DIR, L, kThreads, 0, 1>(ld, st, S0, S1, nl, ax.tw);
}

// Forward axis-1 pass over the pair grids of a W build (Eqs. 2c, 3) with the
// pair products formed in its first pass, so the pair grids are never
// written before their transform.  Two sources:
//  * IJ set (tau build): grid q = 32 blk + 4 j + m of block blk = (I, J)
//    holds phi_{8I+2m} phi_{8J+j} + i phi_{8I+2m+1} phi_{8J+j} (the tile
//    layout of the pair-density kernel); orbital v is the real (v even) or
//    imaginary (v odd) part of packed grid v / 2 of orb, zero for v >= nv;
//  * IJ NULL (exchange-like terms): grid q < ngrid holds orb[q] times the
//    real field x (component xc of the packed grid x2).
// The 32 grids of one group of 32 and one line tile run on one XCD
// (xcd_item), where they share their common factors' lines in L2.
template <int N>
__global__ __launch_bounds__(kThreads) void k_fft_axis_pairs(cplx* __restrict__ data, AxisArgs ax,
                                                             const cplx* __restrict__ orb, int nv,
                                                             const int2* __restrict__ IJ,
                                                             const cplx* __restrict__ x2, int xc,
                                                             long ngrid, int np2, long nr,
                                                             int group) {
  constexpr int L = axis_gd_l<N>();
  static_assert(factor(N).n >= 2, "");
  extern __shared__ cplx lds[];
  cplx* S0 = lds;
  cplx* S1 = lds + N * L;
  const int tiles = (np2 + L - 1) / L;
  const long nblk = (ngrid + 31) / 32;
  long item;
  int sub;
  xcd_item(blockIdx.x, 32, group != 0, item, sub);
  if (item >= nblk * tiles) return;
  const int tile = (int)(item % tiles);
  const long blk = item / tiles;
  const long q = blk * 32 + sub;
  if (q >= ngrid) return;
  const int i0 = tile * L;
  const int nl = min(L, np2 - i0);
  const cplx *oa, *ow;
  bool a_ok = true, a1_ok = true, w_ok = true, w_im = xc != 0;
  if (IJ) {
    const int2 b = IJ[blk];
    const int va = 8 * b.x + 2 * (sub & 3), vw = 8 * b.y + (sub >> 2);
    a_ok = va < nv;
    a1_ok = va + 1 < nv;
    w_ok = vw < nv;
    w_im = (vw & 1) != 0;
    // va is even: phi_va and phi_va+1 are the two parts of one packed grid
    oa = orb + (long)(va >> 1) * nr + i0;
    ow = orb + (long)(vw >> 1) * nr + i0;
  } else {
    oa = orb + q * nr + i0;
    ow = x2 + i0;
  }
  cplx* out = data + q * nr + i0;
  auto ld = [=](int k, int l) {
    const long r = (long)k * np2 + l;
    const cplx a = a_ok ? oa[r] : mk(0.0, 0.0);
    const cplx wv = w_ok ? ow[r] : mk(0.0, 0.0);
    const real w = w_im ? wv.y : wv.x;
    return mk(a.x * w, a1_ok ? a.y * w : (real)0);
  };
  auto st = [=](int k, int l, cplx v) { out[(long)k * np2 + l] = v; };
  fn_passes<N, -1, L, kThreads, 0, 1>(ld, st, S0, S1, nl, ax.tw);
}

int lines_per_group(int n) {
  // about 16 KB of LDS per buffer; at least 4 lines
  int L = 16384 / ((int)sizeof(cplx) * n);
  if (L < 4) L = 4;
  if (L > 32) L = 32;
  return L;
}

AxisArgs axis_args(const FftAxis& a) {
  AxisArgs ax;
  ax.n = a.n;
  ax.nrad = a.nrad;
  for (int i = 0; i < 8; ++i) ax.rad[i] = a.rad[i];
  ax.tw = BSEX_FFT_TW(a);
  return ax;
}

#define BSEX_AXIS_SIZES(X) \
  X(8) X(12) X(16) X(20) X(24) X(30) X(32) X(36) X(40) X(48) X(60) X(64) X(72) X(80) X(96) X(120) X(128)
#define BSEX_PLANE_SIZES(X) \
  X(12, 12) X(16, 16) X(24, 24) X(32, 32) X(40, 40) X(48, 48) X(64, 64) X(72, 72) X(48, 120) X(120, 120)

bool axis_ct_supported(int n) {
#define C(N) \
  if (n == N) return true;
  BSEX_AXIS_SIZES(C)
#undef C
  return false;
}

bool plane_ct_supported(int n2, int n3) {
#define C(A, B) \
  if (n2 == A && n3 == B) return true;
  BSEX_PLANE_SIZES(C)
#undef C
  return false;
}

size_t plane_ct_lds(int n2, int n3) {
#define C(A, B) \
  if (n2 == A && n3 == B) return (size_t)plane_lds_bytes<A, B>();
  BSEX_PLANE_SIZES(C)
#undef C
  return 0;
}

bool axis_gd_supported(int n) {
#define C(N) \
  if (n == N) return axis_gd_ok<N>();
  BSEX_AXIS_SIZES(C)
#undef C
  return false;
}

size_t axis_gd_lds_of(int n) {
#define C(N) \
  if (n == N) return axis_gd_lds<N>();
  BSEX_AXIS_SIZES(C)
#undef C
  return 0;
}

int axis_gd_lines(int n) {
#define C(N) \
  if (n == N) return axis_gd_l<N>();
  BSEX_AXIS_SIZES(C)
#undef C
  return 0;
}

size_t axis_ct_lds(int n) {
#define C(N) \
  if (n == N) return 2 * sizeof(cplx) * (size_t)N * axis_l<N>();
  BSEX_AXIS_SIZES(C)
#undef C
  return 0;
}

int axis_ct_lines(int n) {
#define C(N) \
  if (n == N) return axis_l<N>();
  BSEX_AXIS_SIZES(C)
#undef C
  return 0;
}

void launch_axis_ct(int n, int dir, dim3 grid, size_t shm, hipStream_t st, cplx* data,
                    AxisArgs ax, int es, int n_inner, long s_in, int n_o2, long s_o2, long s_o1,
                    int ld_lim, int st_lim) {
#define C(N)                                                                                 \
  if (n == N) {                                                                              \
    if (dir < 0)                                                                             \
      hipLaunchKernelGGL((k_fft_axis_ct<N, -1>), grid, dim3(kThreads), shm, st, data, ax, es, \
                         n_inner, s_in, n_o2, s_o2, s_o1, ld_lim, st_lim);                    \
    else                                                                                     \
      hipLaunchKernelGGL((k_fft_axis_ct<N, 1>), grid, dim3(kThreads), shm, st, data, ax, es,  \
                         n_inner, s_in, n_o2, s_o2, s_o1, ld_lim, st_lim);                    \
    return;                                                                                  \
  }
  BSEX_AXIS_SIZES(C)
#undef C
}

template <int N>
bool launch_axis_gd_n(int n, int dir, dim3 grid, size_t shm, hipStream_t st, cplx* data,
                      AxisArgs ax, int es, int n_inner, long s_in, int n_o2, long s_o2,
                      long s_o1, int ld_lim, int st_lim) {
  if constexpr (axis_gd_ok<N>()) {
    if (n != N) return false;
    if (dir < 0)
      hipLaunchKernelGGL((k_fft_axis_gd<N, -1>), grid, dim3(kThreads), shm, st, data, ax, es,
                         n_inner, s_in, n_o2, s_o2, s_o1, ld_lim, st_lim);
    else
      hipLaunchKernelGGL((k_fft_axis_gd<N, 1>), grid, dim3(kThreads), shm, st, data, ax, es,
                         n_inner, s_in, n_o2, s_o2, s_o1, ld_lim, st_lim);
    return true;
  }
  return false;
}

template <int N>
bool launch_axis_pairs_n(int n, dim3 grid, size_t shm, hipStream_t st, cplx* data, AxisArgs ax,
                         const cplx* orb, int nv, const int2* IJ, const cplx* x2, int xc,
                         long ngrid, int np2, long nr, int group) {
  if constexpr (axis_gd_ok<N>()) {
    if (n != N) return false;
    hipLaunchKernelGGL((k_fft_axis_pairs<N>), grid, dim3(kThreads), shm, st, data, ax, orb, nv,
                       IJ, x2, xc, ngrid, np2, nr, group);
    return true;
  }
  return false;
}

void launch_axis_gd(int n, int dir, dim3 grid, size_t shm, hipStream_t st, cplx* data,
                    AxisArgs ax, int es, int n_inner, long s_in, int n_o2, long s_o2, long s_o1,
                    int ld_lim, int st_lim) {
#define C(N)                                                                               \
  if (launch_axis_gd_n<N>(n, dir, grid, shm, st, data, ax, es, n_inner, s_in, n_o2, s_o2, \
                          s_o1, ld_lim, st_lim))                                           \
    return;
  BSEX_AXIS_SIZES(C)
#undef C
}

template <int N>
int set_axis_gd_lds() {
  if constexpr (axis_gd_ok<N>()) {
    const int g = (int)axis_gd_lds<N>();
    BSE_HIP(hipFuncSetAttribute((const void*)k_fft_axis_gd<N, -1>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, g));
    BSE_HIP(hipFuncSetAttribute((const void*)k_fft_axis_gd<N, 1>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, g));
    BSE_HIP(hipFuncSetAttribute((const void*)k_fft_axis_pairs<N>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, g));
  }
  return BSE_OK;
}

template <int DIR, int IN, int OUT>
void launch_plane_ct(int n2, int n3, dim3 grid, size_t shm, hipStream_t st, cplx* data,
                     PlaneArgs pa, AxisArgs ay, AxisArgs az) {
#define C(A, B)                                                                               \
  if (n2 == A && n3 == B) {                                                                   \
    hipLaunchKernelGGL((k_fft_plane_ct<A, B, DIR, IN, OUT>), grid, dim3(kPlaneThreads), shm,  \
                       st, data, pa, ay, az);                                                 \
    return;                                                                                   \
  }
  BSEX_PLANE_SIZES(C)
#undef C
}

int set_ct_lds_limits(int n2, int n3, int n1) {
#define C(A, B)                                                                                  \
  if (n2 == A && n3 == B) {                                                                      \
    const int need = (int)plane_ct_lds(A, B);                                                    \
    const void* fns[] = {(const void*)k_fft_plane_ct<A, B, -1, 0, 0>,                            \
                         (const void*)k_fft_plane_ct<A, B, 1, 0, 0>,                             \
                         (const void*)k_fft_plane_ct<A, B, 1, 1, 0>,                             \
                         (const void*)k_fft_plane_ct<A, B, -1, 0, 1>,                            \
                         (const void*)k_fft_plane_ct<A, B, -1, 0, 2>};                           \
    for (const void* f : fns)                                                                    \
      BSE_HIP(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, need));         \
  }
  BSEX_PLANE_SIZES(C)
#undef C
#define C(N)                                                                                    \
  if (n1 == N) {                                                                                \
    const int need = (int)axis_ct_lds(N);                                                       \
    BSE_HIP(hipFuncSetAttribute((const void*)k_fft_axis_ct<N, -1>,                              \
                                hipFuncAttributeMaxDynamicSharedMemorySize, need));             \
    BSE_HIP(hipFuncSetAttribute((const void*)k_fft_axis_ct<N, 1>,                               \
                                hipFuncAttributeMaxDynamicSharedMemorySize, need));             \
    BSE_TRY(set_axis_gd_lds<N>());                                                              \
  }
  BSEX_AXIS_SIZES(C)
#undef C
  return BSE_OK;
}

// padded lines of the pruned kernels' batches (same line counts as below)
inline long sphere_padded(int nrow, int ncol, int lb) {
  return (long)((nrow + lb - 1) / lb + (ncol + lb - 1) / lb) * lb;
}
// rounds of butterflies (at most one per thread each) of the line
// transforms of length n in batches of lb lines
inline long pass_rounds(int n, int lb) {
  const Fac f = factor(n);
  long r = 0;
  for (int p = 0; p < f.n; ++p) r += ((long)(n / f.r[p]) * lb + kPlaneThreads - 1) / kPlaneThreads;
  return r;
}
// rounds of the pruned kernels: nrow row transforms of length lrow, then
// ncol column transforms of length lcol (inverse: K2 rows of N3, N3 columns
// of N2; forward: N2 rows of N3, K3 columns of N2)
inline long sphere_rounds(int nrow, int lrow, int ncol, int lcol, int lb) {
  return (long)((nrow + lb - 1) / lb) * pass_rounds(lrow, lb) +
         (long)((ncol + lb - 1) / lb) * pass_rounds(lcol, lb);
}

// pruned sphere-plane launches: false when the size has no compiled kernel
// or the LDS the extents need exceeds the device's
bool launch_sphere_ct(int n2, int n3, bool inverse, int m, size_t max_lds, dim3 grid,
                      hipStream_t st, cplx* data, PlaneArgs pa, AxisArgs ay, AxisArgs az) {
  // inverse pass: batch size k in {0, 1, 2}, scored by the rounds of
  // butterflies over the workgroup's threads (each ending at a barrier),
  // tripled when two workgroups do not fit a CU.  Forward pass: batch size k
  // in {0, 1} and the staged (w = 0) or whole-plane (w = 1) kernel, scored by
  // the padded line count, doubled when two workgroups do not fit a CU (the
  // choices measured fastest at the grids in use).  Ties go to the
  // whole-plane kernel and the smaller batch.
#define C(A, B)                                                                               \
  if (n2 == A && n3 == B) {                                                                   \
    int pick = -1, pw = 0;                                                                    \
    long best = 0;                                                                            \
    size_t shm = 0;                                                                           \
    for (int w = inverse ? 0 : 1; w >= 0; --w)                                                \
      for (int k = 0; k < (inverse ? 3 : 2); ++k) {                                           \
        const int lb = kSphereLB[k];                                                          \
        const size_t need = inverse ? sphere_inv_lds<A, B>(m, lb)                             \
                            : w ? sphere_fwd_whole_lds<A, B>(lb) : sphere_fwd_lds<A, B>(m, lb); \
        if (need > max_lds) continue;                                                         \
        const long score = inverse                                                            \
            ? sphere_rounds(2 * m + 1, B, B, A, lb) * (need <= 81920 ? 1 : 3)                 \
            : sphere_padded(A, 2 * m + 1, lb) * (need <= 81920 ? 1 : 2);                      \
        if (pick < 0 || score < best) {                                                       \
          pick = k;                                                                           \
          pw = w;                                                                             \
          best = score;                                                                       \
          shm = need;                                                                         \
        }                                                                                     \
      }                                                                                       \
    if (pick < 0) return false;                                                               \
    if (inverse) {                                                                            \
      if (pick == 0)                                                                          \
        hipLaunchKernelGGL((k_sphere_inv_ct<A, B, 1, kSphereLB[0]>), grid, dim3(kPlaneThreads), \
                           shm, st, data, pa, ay, az);                                        \
      else if (pick == 1)                                                                     \
        hipLaunchKernelGGL((k_sphere_inv_ct<A, B, 1, kSphereLB[1]>), grid, dim3(kPlaneThreads), \
                           shm, st, data, pa, ay, az);                                        \
      else                                                                                    \
        hipLaunchKernelGGL((k_sphere_inv_ct<A, B, 1, kSphereLB[2]>), grid, dim3(kPlaneThreads), \
                           shm, st, data, pa, ay, az);                                        \
    } else if (pw) {                                                                          \
      if (pick == 0)                                                                          \
        hipLaunchKernelGGL((k_sphere_fwd_whole<A, B, -1, kSphereLB[0]>), grid,                \
                           dim3(kPlaneThreads), shm, st, data, pa, ay, az);                   \
      else                                                                                    \
        hipLaunchKernelGGL((k_sphere_fwd_whole<A, B, -1, kSphereLB[1]>), grid,                \
                           dim3(kPlaneThreads), shm, st, data, pa, ay, az);                   \
    } else {                                                                                  \
      if (pick == 0)                                                                          \
        hipLaunchKernelGGL((k_sphere_fwd_ct<A, B, -1, kSphereLB[0]>), grid,                   \
                           dim3(kPlaneThreads), shm, st, data, pa, ay, az);                   \
      else                                                                                    \
        hipLaunchKernelGGL((k_sphere_fwd_ct<A, B, -1, kSphereLB[1]>), grid,                   \
                           dim3(kPlaneThreads), shm, st, data, pa, ay, az);                   \
    }                                                                                         \
    return true;                                                                              \
  }
  BSEX_PLANE_SIZES(C)
#undef C
  return false;
}

// the pruned kernels may use up to the device's LDS (extents are known only
// with a sphere)
int set_sphere_lds_limits(int n2, int n3, size_t max_lds) {
#define C(A, B)                                                                               \
  if (n2 == A && n3 == B) {                                                                   \
    const int lim = (int)max_lds;                                                             \
    const void* fns[] = {(const void*)k_sphere_inv_ct<A, B, 1, kSphereLB[0]>,                 \
                         (const void*)k_sphere_inv_ct<A, B, 1, kSphereLB[1]>,                 \
                         (const void*)k_sphere_inv_ct<A, B, 1, kSphereLB[2]>,                 \
                         (const void*)k_sphere_fwd_ct<A, B, -1, kSphereLB[0]>,                \
                         (const void*)k_sphere_fwd_ct<A, B, -1, kSphereLB[1]>,                \
                         (const void*)k_sphere_fwd_whole<A, B, -1, kSphereLB[0]>,             \
                         (const void*)k_sphere_fwd_whole<A, B, -1, kSphereLB[1]>};            \
    for (const void* f : fns)                                                                 \
      BSE_HIP(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lim));       \
  }
  BSEX_PLANE_SIZES(C)
#undef C
  return BSE_OK;
}

}  // namespace

size_t fft_plane_lds(const FftPlan& p, int* LB) {
  const size_t plane = sizeof(cplx) * (size_t)p.N[1] * p.N[2];
  const int nmax = std::max(p.N[1], p.N[2]);
  int lb = 32;
  while (lb > 4 && plane + 2 * sizeof(cplx) * (size_t)lb * nmax > p.max_lds) lb /= 2;
  if (LB) *LB = lb;
  return plane + 2 * sizeof(cplx) * (size_t)lb * nmax;
}

static int launch_axis(const FftAxis& a, cplx* data, int dir, int es, int n_inner, long s_in,
                       int n_o2, long s_o2, long n_o1, long s_o1, int ld_lim, int st_lim,
                       hipStream_t st, bool ct, bool gd = false) {
  const AxisArgs ax = axis_args(a);
  if (ct && gd && axis_gd_supported(a.n)) {
    const int L = axis_gd_lines(a.n);
    const long tiles = (n_inner + L - 1) / L;
    const long groups = tiles * n_o2 * n_o1;
    if (groups <= 0) return BSE_OK;
    if (groups > 0x7fffffffL) return fail(BSE_EINVAL, "FFT batch too large");
    launch_axis_gd(a.n, dir, dim3((unsigned)groups), axis_gd_lds_of(a.n), st, data, ax, es,
                   n_inner, s_in, n_o2, s_o2, s_o1, ld_lim, st_lim);
    BSE_HIP(hipGetLastError());
    return BSE_OK;
  }
  if (ct) {
    const int L = axis_ct_lines(a.n);
    const long tiles = (n_inner + L - 1) / L;
    const long groups = tiles * n_o2 * n_o1;
    if (groups <= 0) return BSE_OK;
    if (groups > 0x7fffffffL) return fail(BSE_EINVAL, "FFT batch too large");
    launch_axis_ct(a.n, dir, dim3((unsigned)groups), axis_ct_lds(a.n), st, data, ax, es, n_inner,
                   s_in, n_o2, s_o2, s_o1, ld_lim, st_lim);
    BSE_HIP(hipGetLastError());
    return BSE_OK;
  }
  const int L = lines_per_group(a.n);
  const long tiles = (n_inner + L - 1) / L;
  const long groups = tiles * n_o2 * n_o1;
  if (groups <= 0) return BSE_OK;
  if (groups > 0x7fffffffL) return fail(BSE_EINVAL, "FFT batch too large");
  const size_t shm = 2 * sizeof(cplx) * a.n * L;
  if (dir < 0)
    hipLaunchKernelGGL(k_fft_axis<-1>, dim3((unsigned)groups), dim3(kThreads), shm, st, data, ax,
                       es, n_inner, s_in, n_o2, s_o2, s_o1, L, ld_lim, st_lim);
  else
    hipLaunchKernelGGL(k_fft_axis<1>, dim3((unsigned)groups), dim3(kThreads), shm, st, data, ax,
                       es, n_inner, s_in, n_o2, s_o2, s_o1, L, ld_lim, st_lim);
  BSE_HIP(hipGetLastError());
  return BSE_OK;
}

// axis-1 pass over [batch][N1][N2][N3]: the N2 * N3 lines of one grid start
// at consecutive addresses, so they are tiled as a single range and no tile
// is left partly empty at the end of each row of N3 lines
static int x_pass(const FftPlan& p, cplx* data, long batch, int dir, int ld_lim, int st_lim,
                  hipStream_t st) {
  const int np2 = p.N[1] * p.N[2];
  return launch_axis(p.ax[0], data, dir, np2, np2, 1, 1, 0, batch, p.nr, ld_lim, st_lim, st,
                     p.ct_axis[BSEX_FFT_PREC], p.axis_direct[BSEX_FFT_PREC]);
}

template <int DIR, int IN, int OUT>
static int launch_plane(const FftPlan& p, cplx* data, long batch, PlaneArgs pa, hipStream_t st) {
  int lb = 0;
  const size_t shm = fft_plane_lds(p, &lb);
  pa.N1 = p.N[0];
  pa.N2 = p.N[1];
  pa.N3 = p.N[2];
  pa.nr = p.nr;
  pa.LB = lb;
  const long groups = batch * pa.nplanes;
  if (groups <= 0) return BSE_OK;
  if (groups > 0x7fffffffL) return fail(BSE_EINVAL, "FFT batch too large");
  if (p.ct_plane[BSEX_FFT_PREC])
    launch_plane_ct<DIR, IN, OUT>(p.N[1], p.N[2], dim3((unsigned)groups), plane_ct_lds(p.N[1], p.N[2]),
                                  st, data, pa, axis_args(p.ax[1]), axis_args(p.ax[2]));
  else
    hipLaunchKernelGGL((k_fft_plane<DIR, IN, OUT>), dim3((unsigned)groups), dim3(kPlaneThreads),
                       shm, st, data, pa, axis_args(p.ax[1]), axis_args(p.ax[2]));
  BSE_HIP(hipGetLastError());
  return BSE_OK;
}

// the sphere-plane passes through the pruned kernels, when they apply
static bool launch_sphere(const FftPlan& p, const SpherePlan& sp, bool inverse, cplx* data,
                          long batch, PlaneArgs pa, hipStream_t st) {
  if (!p.prune[BSEX_FFT_PREC]) return false;
  pa.group = inverse && xcd_group_on() ? 1 : 0;
  pa.batch = batch;
  const long groups = (pa.group ? round8(batch) : batch) * pa.nplanes;
  if (groups <= 0 || groups > 0x7fffffffL) return false;
  pa.N1 = p.N[0];
  pa.N2 = p.N[1];
  pa.N3 = p.N[2];
  pa.nr = p.nr;
  pa.m2 = sp.m2;
  pa.m3 = sp.m3;
  return launch_sphere_ct(p.N[1], p.N[2], inverse, inverse ? sp.m2 : sp.m3, p.max_lds,
                          dim3((unsigned)groups), st, data, pa, axis_args(p.ax[1]),
                          axis_args(p.ax[2]));
}

int init_kernels(FftPlan* p) {
  int lb = 0;
  const size_t need = fft_plane_lds(*p, &lb);
  if (need > p->max_lds)
    return fail(BSE_EINVAL, "FFT plane %dx%d does not fit the device LDS", p->N[1], p->N[2]);
  const void* fns[] = {(const void*)k_fft_plane<-1, 0, 0>, (const void*)k_fft_plane<1, 0, 0>,
                       (const void*)k_fft_plane<1, 1, 0>, (const void*)k_fft_plane<-1, 0, 1>,
                       (const void*)k_fft_plane<-1, 0, 2>};
  for (const void* f : fns)
    BSE_HIP(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)need));
  bool ctp = plane_ct_supported(p->N[1], p->N[2]) && plane_ct_lds(p->N[1], p->N[2]) <= p->max_lds;
  bool cta = axis_ct_supported(p->N[0]);
  if (const char* e = getenv("BSEX_FFT_RUNTIME")) {
    if (atoi(e)) ctp = cta = false;
  }
  p->ct_plane[BSEX_FFT_PREC] = p->ct_plane_ok[BSEX_FFT_PREC] = ctp;
  p->ct_axis[BSEX_FFT_PREC] = p->ct_axis_ok[BSEX_FFT_PREC] = cta;
  bool prune = plane_ct_supported(p->N[1], p->N[2]);
  if (const char* e = getenv("BSEX_FFT_PRUNE")) prune = prune && atoi(e) != 0;
  p->prune[BSEX_FFT_PREC] = prune;
  bool direct = true;
  if (const char* e = getenv("BSEX_FFT_AXIS_DIRECT")) direct = atoi(e) != 0;
  p->axis_direct[BSEX_FFT_PREC] = direct;
  if (prune) BSE_TRY(set_sphere_lds_limits(p->N[1], p->N[2], p->max_lds));
  return set_ct_lds_limits(ctp ? p->N[1] : -1, ctp ? p->N[2] : -1, cta ? p->N[0] : -1);
}

int fft3d(const FftPlan& p, cplx* data, long batch, int dir, hipStream_t st) {
  if (batch <= 0) return BSE_OK;
  PlaneArgs pa{};
  pa.nplanes = p.N[0];
  const int all = p.N[0];
  if (dir > 0) {
    BSE_TRY((launch_plane<1, 0, 0>(p, data, batch, pa, st)));
    BSE_TRY(x_pass(p, data, batch, +1, all, all, st));
  } else {
    BSE_TRY(x_pass(p, data, batch, -1, all, all, st));
    BSE_TRY((launch_plane<-1, 0, 0>(p, data, batch, pa, st)));
  }
  return BSE_OK;
}

// the plane pass of a W build's forward transform (OUT == 2)
static int plane_fwd_w(const FftPlan& p, const SpherePlan& sp, cplx* data, long batch,
                       const real* f, real s, cplx* compact, hipStream_t st) {
  if (compact && !sp.plane_sp) return fail(BSE_EINVAL, "fused W transform: no sphere plan");
  const int all = p.N[0];
  PlaneArgs pa{};
  pa.nplanes = all;
  pa.plane_sp = sp.plane_sp;
  pa.plane_off = sp.plane_off;
  pa.ent_pos = sp.ent_pos;
  pa.nent = sp.nent;
  pa.compact = compact;
  pa.mulf = f;
  pa.muls = s;
  return launch_plane<-1, 0, 2>(p, data, batch, pa, st);
}

int fft3d_fwd_w(const FftPlan& p, const SpherePlan& sp, cplx* data, long batch, const real* f,
                real s, cplx* compact, hipStream_t st) {
  if (batch <= 0) return BSE_OK;
  BSE_TRY(x_pass(p, data, batch, -1, p.N[0], p.N[0], st));
  return plane_fwd_w(p, sp, data, batch, f, s, compact, st);
}

bool fwd_pairs_supported(const FftPlan& p) {
  return p.ct_axis[BSEX_FFT_PREC] && p.axis_direct[BSEX_FFT_PREC] && axis_gd_supported(p.N[0]);
}

// first pass of fft3d_fwd_pairs / fft3d_fwd_times (k_fft_axis_pairs)
static int axis_pairs(const FftPlan& p, const cplx* orb, int nv, const int2* IJ, const cplx* x2,
                      int xc, long ngrid, cplx* data, hipStream_t st) {
  if (!fwd_pairs_supported(p))
    return fail(BSE_EINVAL, "pair-forming transform: axis length %d", p.N[0]);
  const int np2 = p.N[1] * p.N[2];
  const long tiles = (np2 + axis_gd_lines(p.N[0]) - 1) / axis_gd_lines(p.N[0]);
  const long items = (ngrid + 31) / 32 * tiles;
  const int group = xcd_group_on() ? 1 : 0;
  const long groups = 32 * (group ? round8(items) : items);
  if (groups > 0x7fffffffL) return fail(BSE_EINVAL, "FFT batch too large");
  const AxisArgs ax = axis_args(p.ax[0]);
  const dim3 grid((unsigned)groups);
  const size_t shm = axis_gd_lds_of(p.N[0]);
  const int n1 = p.N[0];
  bool done = false;
#define C(K)                                                                               \
  if (!done)                                                                               \
    done = launch_axis_pairs_n<K>(n1, grid, shm, st, data, ax, orb, nv, IJ, x2, xc, ngrid, \
                                  np2, p.nr, group);
  BSEX_AXIS_SIZES(C)
#undef C
  if (!done) return fail(BSE_EINVAL, "pair-forming transform: axis length %d", p.N[0]);
  BSE_HIP(hipGetLastError());
  return BSE_OK;
}

int fft3d_fwd_pairs(const FftPlan& p, const SpherePlan& sp, const cplx* orb, int nv,
                    const int2* IJ, long nblk, cplx* data, const real* f, real s, cplx* compact,
                    hipStream_t st) {
  if (nblk <= 0) return BSE_OK;
  BSE_TRY(axis_pairs(p, orb, nv, IJ, nullptr, 0, nblk * 32, data, st));
  return plane_fwd_w(p, sp, data, nblk * 32, f, s, compact, st);
}

int fft3d_fwd_times(const FftPlan& p, const SpherePlan& sp, const cplx* M, long nm,
                    const cplx* x2, int xc, cplx* data, const real* f, real s, cplx* compact,
                    hipStream_t st) {
  if (nm <= 0) return BSE_OK;
  BSE_TRY(axis_pairs(p, M, 0, nullptr, x2, xc, nm, data, st));
  return plane_fwd_w(p, sp, data, nm, f, s, compact, st);
}

int sphere_to_grid(const FftPlan& p, const SpherePlan& sp, double omega, const double* X, int nv,
                   int nset, cplx* grid, hipStream_t st) {
  const int nvh = (nv + 1) / 2;
  const long batch = (long)nset * nvh;
  if (batch <= 0) return BSE_OK;
  PlaneArgs pa{};
  pa.nplanes = sp.nplanes;
  pa.plane_i1 = sp.plane_i1;
  pa.plane_off = sp.plane_off;
  pa.ent_pos = sp.ent_pos;
  pa.ent_code = sp.ent_code;
  pa.nent = sp.nent;
  pa.X = X;
  pa.nv = nv;
  pa.nvh = nvh;
  pa.npw = sp.nent;
  pa.s0 = 1.0 / std::sqrt(omega);
  pa.s1 = 1.0 / std::sqrt(2.0 * omega);
  if (!launch_sphere(p, sp, true, grid, batch, pa, st))
    BSE_TRY((launch_plane<1, 1, 0>(p, grid, batch, pa, st)));
  BSE_HIP(hipGetLastError());
  return x_pass(p, grid, batch, +1, sp.nmax1, p.N[0], st);
}

int grid_to_compact(const FftPlan& p, const SpherePlan& sp, cplx* grid, long batch,
                    cplx* compact, hipStream_t st) {
  if (batch <= 0) return BSE_OK;
  BSE_TRY(x_pass(p, grid, batch, -1, p.N[0], sp.nmax1, st));
  PlaneArgs pa{};
  pa.nplanes = sp.nplanes;
  pa.plane_i1 = sp.plane_i1;
  pa.plane_off = sp.plane_off;
  pa.ent_pos = sp.ent_pos;
  pa.ent_code = sp.ent_code;
  pa.nent = sp.nent;
  pa.compact = compact;
  if (launch_sphere(p, sp, false, grid, batch, pa, st)) {
    BSE_HIP(hipGetLastError());
    return BSE_OK;
  }
  return launch_plane<-1, 0, 1>(p, grid, batch, pa, st);
}

