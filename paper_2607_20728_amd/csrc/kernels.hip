// Element-wise, sphere<->grid and tau kernels of the DMPT BSE operator (FP64).
#include <cmath>
#include <cstdlib>

#include "kernels.h"

namespace bsex {

bool xcd_group_on() {
  static const bool on = [] {
    const char* e = getenv("BSEX_XCD_GROUP");
    return !e || atoi(e) != 0;
  }();
  return on;
}

namespace {

constexpr int TPB = 256;

inline unsigned nblocks(long n, int tpb = TPB) {
  long b = (n + tpb - 1) / tpb;
  if (b > 1048576) b = 1048576;  // grid-stride loops cover the rest
  if (b < 1) b = 1;
  return (unsigned)b;
}

__device__ __forceinline__ long gtid() { return (long)blockIdx.x * blockDim.x + threadIdx.x; }
__device__ __forceinline__ long gstride() { return (long)gridDim.x * blockDim.x; }

// ---------------------------------------------------------------------------
// sphere <-> grid (two real orbitals per complex grid)
//   f(0) = x0/sqrt(Omega), f(+G) = (xc - i xs)/sqrt(2 Omega), f(-G) = conj(f(+G));
//   grid of orbitals u (real part) and w (imaginary part): H = U + i W.
// ---------------------------------------------------------------------------
template <typename V2>
__device__ __forceinline__ V2 make2(double x, double y) {
  V2 v;
  v.x = x;
  v.y = y;
  return v;
}

// one workgroup per (grid, range of modes); the workgroups of one grid run on
// one XCD (xcd_item), so the scattered updates of a grid meet in one L2
template <typename V2, typename XT>
__global__ void k_scatter(const int* __restrict__ idx_p, const int* __restrict__ idx_m, int nhalf,
                          int npw, long nr, long zero, const XT* __restrict__ X, int nv,
                          int nvh, long ngrid, int nbx, int group, V2* __restrict__ grid, int acc,
                          double s0, double s1) {
  long g;
  int bx;
  xcd_item(blockIdx.x, nbx, group != 0, g, bx);
  const int t = bx * blockDim.x + threadIdx.x;
  if (t > nhalf || g >= ngrid) return;
  {
    const long set = g / nvh;
    const int p = (int)(g % nvh);
    const int v1 = 2 * p, v2 = 2 * p + 1;
    const XT* x1 = X + (set * nv + v1) * (long)npw;
    const XT* x2 = (v2 < nv) ? X + (set * nv + v2) * (long)npw : nullptr;
    V2* G = grid + g * nr;
    if (t == 0) {
      double2 h = make_double2(x1[0] * s0, x2 ? x2[0] * s0 : 0.0);
      if (acc) {
        h.x += G[zero].x;
        h.y += G[zero].y;
      }
      G[zero] = make2<V2>(h.x, h.y);
    } else {
      const int k = t - 1;
      const double c1 = x1[1 + 2 * k], q1 = x1[2 + 2 * k];
      const double c2 = x2 ? x2[1 + 2 * k] : 0.0, q2 = x2 ? x2[2 + 2 * k] : 0.0;
      double2 hp = make_double2((c1 + q2) * s1, (c2 - q1) * s1);
      double2 hm = make_double2((c1 - q2) * s1, (q1 + c2) * s1);
      const int ip = idx_p[k], im = idx_m[k];
      if (acc) {
        const V2 op = G[ip], om = G[im];
        hp.x += op.x;
        hp.y += op.y;
        hm.x += om.x;
        hm.y += om.y;
      }
      G[ip] = make2<V2>(hp.x, hp.y);
      G[im] = make2<V2>(hm.x, hm.y);
    }
  }
}

// one workgroup per (grid, range of modes); the workgroups of one grid run on
// one XCD (xcd_item), which then holds that grid's entries in its L2
template <typename V2, typename YT>
__global__ void k_gather(const int* __restrict__ idx_p, const int* __restrict__ idx_m, int nhalf,
                         int npw, long nr, long zero, const V2* __restrict__ grid, int nv,
                         int nvh, long ngrid, int nbx, int group, double c0, double c1,
                         const double* __restrict__ A, const double* __restrict__ T,
                         const double* __restrict__ eps, double shift, double beta,
                         YT* __restrict__ Y) {
  long g;
  int bx;
  xcd_item(blockIdx.x, nbx, group != 0, g, bx);
  const int t = bx * blockDim.x + threadIdx.x;
  if (t > nhalf || g >= ngrid) return;
  {
    const long set = g / nvh;
    const int p = (int)(g % nvh);
    const int v1 = 2 * p, v2 = 2 * p + 1;
    const V2* G = grid + g * nr;
    double a1, b1, a2 = 0, b2 = 0;  // (cos, sin) or (G0, unused)
    int j1, j2;
    if (t == 0) {
      const V2 hv = G[zero];
      const double2 h = make_double2(hv.x, hv.y);
      a1 = c0 * h.x;
      a2 = c0 * h.y;
      j1 = 0;
      j2 = -1;
    } else {
      const int k = t - 1;
      const V2 hpv = G[idx_p[k]], hmv = G[idx_m[k]];
      const double2 hp = make_double2(hpv.x, hpv.y), hm = make_double2(hmv.x, hmv.y);
      a1 = 0.5 * c1 * (hp.x + hm.x);    // orbital 1, cos
      b1 = -0.5 * c1 * (hp.y - hm.y);   // orbital 1, sin
      a2 = 0.5 * c1 * (hp.y + hm.y);    // orbital 2, cos
      b2 = 0.5 * c1 * (hp.x - hm.x);    // orbital 2, sin
      j1 = 1 + 2 * k;
      j2 = 2 + 2 * k;
    }
    for (int o = 0; o < 2; ++o) {
      const int v = o ? v2 : v1;
      if (v >= nv) break;
      const long row = (set * nv + v) * (long)npw;
      const double va = o ? a2 : a1;
      const double vb = o ? b2 : b1;
      for (int q = 0; q < 2; ++q) {
        const int j = q ? j2 : j1;
        if (j < 0) break;
        double val = q ? vb : va;
        if (A) val += (T[j] + shift - (eps ? eps[v] : 0.0)) * A[row + j];
        if (beta != 0.0) val += beta * (double)Y[row + j];
        Y[row + j] = (YT)val;
      }
    }
  }
}

template <typename V2, typename R>
__global__ void k_mul_real(V2* __restrict__ g, long n, long nr, const R* __restrict__ f, R scale) {
  for (long e = gtid(); e < n; e += gstride()) {
    const R m = f[e % nr] * scale;
    V2 x = g[e];
    x.x *= m;
    x.y *= m;
    g[e] = x;
  }
}

__global__ void k_real_part(const double2* __restrict__ g, long nr, double* __restrict__ out) {
  for (long e = gtid(); e < nr; e += gstride()) out[e] = g[e].x;
}

// A thread owns one grid point and a group of up to TD_B vectors, so each
// phi_v(r) is read once per group rather than once per pair of vectors.
constexpr int TD_B = 8;

template <typename V2, typename R>
__global__ void k_transition_density(const V2* __restrict__ phir, const V2* __restrict__ a,
                                     int nvh, int nb, long nr, V2* __restrict__ drho) {
  const long ngroups = (nb + TD_B - 1) / TD_B;
  for (long e = gtid(); e < ngroups * nr; e += gstride()) {
    const long r = e % nr;
    const int b0 = (int)(e / nr) * TD_B;
    const int nbg = min(TD_B, nb - b0);
    R s[TD_B];
#pragma unroll
    for (int o = 0; o < TD_B; ++o) s[o] = 0;
    for (int p = 0; p < nvh; ++p) {
      const V2 f = phir[(long)p * nr + r];
#pragma unroll
      for (int o = 0; o < TD_B; ++o) {
        if (o < nbg) {
          const V2 x = a[((long)(b0 + o) * nvh + p) * nr + r];
          s[o] += f.x * x.x + f.y * x.y;
        }
      }
    }
#pragma unroll
    for (int o = 0; o < TD_B; o += 2) {
      if (o < nbg) {
        V2 out;
        out.x = s[o];
        out.y = (o + 1 < nbg) ? s[o + 1] : (R)0;
        drho[(long)((b0 + o) / 2) * nr + r] = out;
      }
    }
  }
}

template <typename V2, typename R>
__global__ void k_combine(const V2* __restrict__ a, const V2* __restrict__ phir,
                          const R* __restrict__ V, const V2* __restrict__ vdrho, const V2* y,
                          V2* out, int nvh, int nb, long nr, R s, int with_v) {
  const long n = (long)nb * nvh * nr;
  for (long e = gtid(); e < n; e += gstride()) {
    const long r = e % nr;
    const long bp = e / nr;
    const int p = (int)(bp % nvh);
    const int b = (int)(bp / nvh);
    V2 z;
    z.x = 0;
    z.y = 0;
    if (with_v) {
      const R v = V[r];
      const V2 x = a[e];
      z.x = v * x.x;
      z.y = v * x.y;
    }
    if (vdrho) {
      const V2 d = vdrho[(long)(b >> 1) * nr + r];
      const R w = s * ((b & 1) ? d.y : d.x);
      const V2 f = phir[(long)p * nr + r];
      z.x += w * f.x;
      z.y += w * f.y;
    }
    if (y) {
      const V2 q = y[e];
      z.x -= q.x;
      z.y -= q.y;
    }
    out[e] = z;
  }
}

template <typename V2>
__device__ __forceinline__ double orb_at(const V2* __restrict__ phir, int v, int nv, long nr,
                                         long r) {
  if (v >= nv) return 0.0;
  const V2 f = phir[(long)(v >> 1) * nr + r];
  return (v & 1) ? f.y : f.x;
}

// grid q of a tile holds elements 2q, 2q+1 of the 64 per block, element
// e = j*8 + i is the pair (8I + i, 8J + j)
template <typename V2>
__global__ void k_pair_density(const V2* __restrict__ phir, int nv, const int2* __restrict__ IJ,
                               long nblk, long nr, V2* __restrict__ grids) {
  const long n = nblk * 32 * nr;
  for (long e = gtid(); e < n; e += gstride()) {
    const long r = e % nr;
    const long q = e / nr;
    const long blk = q / 32;
    const int qq = (int)(q % 32);
    const int j = qq >> 2;
    const int i0 = 2 * (qq & 3);
    const int2 b = IJ[blk];
    const double w = orb_at(phir, 8 * b.y + j, nv, nr, r);
    const double u0 = orb_at(phir, 8 * b.x + i0, nv, nr, r);
    const double u1 = orb_at(phir, 8 * b.x + i0 + 1, nv, nr, r);
    grids[e] = make2<V2>(u0 * w, u1 * w);
  }
}

// dst[rb][dst_blk0 + blk][j][ri][i] from the packed tile
template <typename G2, typename TD>
__global__ void k_tau_store(const G2* __restrict__ grids, const int2* __restrict__ IJ,
                            long nblk, long nr, int R, TD* __restrict__ dst, long dst_nblk,
                            long dst_blk0) {
  const long per_rb = nblk * 64 * R;
  const long nrb = nr / R;
  const long n = nrb * per_rb;
  for (long e = gtid(); e < n; e += gstride()) {
    const long rb = e / per_rb;
    long w = e % per_rb;
    const int i = (int)(w % 8);
    w /= 8;
    const int ri = (int)(w % R);
    w /= R;
    const int j = (int)(w % 8);
    const long blk = w / 8;
    const long el = blk * 64 + j * 8 + i;
    const G2 g = grids[(el >> 1) * nr + rb * R + ri];
    double v = (el & 1) ? g.y : g.x;
    const int2 b = IJ[blk];
    if (b.x == b.y) {
      if (i > j)
        v = 0.0;
      else if (i == j)
        v *= 0.5;
    }
    dst[rb * dst_nblk * 64 * R + (dst_blk0 + blk) * 64 * R + (j * R + ri) * 8 + i] = (TD)v;
  }
}

// The same store through LDS: a workgroup takes TS_P consecutive grid points
// and TS_NB blocks (TS_NB * 32 complex grids), reads each grid's points as
// one contiguous run into LDS and writes, for every point block rb, the
// TS_NB blocks' contiguous 64 R values of the cache layout.  Both the reads
// and the writes are coalesced; k_tau_store reads 16-byte pieces of 16
// different grids per wave.
constexpr int TS_P = 64, TS_NB = 2;
template <typename G2, typename TD, int R>
__global__ __launch_bounds__(256) void k_tau_store_lds(const G2* __restrict__ grids,
                                                       const int2* __restrict__ IJ, long nblk,
                                                       long nr, TD* __restrict__ dst,
                                                       long dst_nblk, long dst_blk0) {
  constexpr int NG = TS_NB * 32;  // complex grids of a workgroup
  constexpr int RB = TS_P / R;    // point blocks of a workgroup
  __shared__ G2 buf[NG][TS_P + 1];
  const long nrb = nr / R;
  const long npg = (nrb + RB - 1) / RB;
  const long pg = blockIdx.x % npg;
  const long blk0 = (blockIdx.x / npg) * TS_NB;
  const long p0 = pg * TS_P;                  // first point
  const long ngrid = nblk * 32;
  for (int e = threadIdx.x; e < NG * TS_P; e += 256) {
    const int g = e / TS_P, p = e % TS_P;
    const long gg = blk0 * 32 + g, pp = p0 + p;
    G2 v;
    v.x = 0;
    v.y = 0;
    if (gg < ngrid && pp < nrb * R) v = grids[gg * nr + pp];
    buf[g][p] = v;
  }
  __syncthreads();
  constexpr int PER_RB = TS_NB * 64 * R;
  for (int e = threadIdx.x; e < RB * PER_RB; e += 256) {
    const int rbl = e / PER_RB;
    const int rem = e % PER_RB;
    const int bl = rem / (64 * R);
    const int w = rem % (64 * R);
    const int i = w % 8, ri = (w / 8) % R, j = w / (8 * R);
    const long rb = pg * RB + rbl, blk = blk0 + bl;
    if (rb >= nrb || blk >= nblk) continue;
    const int el = bl * 64 + j * 8 + i;
    const G2 g = buf[el >> 1][rbl * R + ri];
    double v = (el & 1) ? g.y : g.x;
    const int2 b = IJ[blk];
    if (b.x == b.y) {
      if (i > j)
        v = 0.0;
      else if (i == j)
        v *= 0.5;
    }
    dst[rb * dst_nblk * 64 * R + (dst_blk0 + blk) * 64 * R + w] = (TD)v;
  }
}

// ---------------------------------------------------------------------------
// tau stream: for every grid point r, y[b][v](r) += sum_v' tau_{vv'}(r) a[b][v'](r)
// with tau stored once per unordered pair as 8x8 blocks (diagonal blocks hold
// the upper triangle with the diagonal halved), blocks in row-major order of
// the block triangle.  A workgroup owns R grid points; a and the y
// accumulators of those points live in LDS.  The NBT = 8 trial vectors are
// split over BL adjacent lanes; a unit of BL lanes owns one grid point and a
// contiguous run of blocks, so along a run the row block I changes rarely:
// its accumulator y[I] and a[I] stay in registers and are flushed to LDS only
// when I changes, while the transposed contribution y[J] goes to LDS with one
// atomic add per (j, b).
// ---------------------------------------------------------------------------
constexpr int NBT = 8;
constexpr int NSLOT = 128;

// FUSE: the epilogue writes z = V a + s (v_c*Drho_b) phi - y instead of y
// (into `y`, which may alias `a`: every workgroup reads its points of a into
// LDS before any write and no other workgroup touches them).
template <typename T>
struct vec2_of;
template <>
struct vec2_of<double> {
  using type = double2;
};
template <>
struct vec2_of<float> {
  using type = float2;
};

// LDS rows (one per orbital v) hold NBT * R values plus SPAD of padding: the
// slots of a wave work on unrelated rows, and an unpadded row of 16 words
// would put the same word of every row in the same bank.  A launch stages the
// rows row0 .. row0 + nrows - 1 only: the bands its blocks touch (a rebuilt
// tile late in the block order touches only the last bands).
constexpr int SPAD = 1;

// T: storage and arithmetic type of tau, a and y.  The LDS accumulators of y
// are FP64 for both types: the LDS FP32 atomic add is several times slower
// than the FP64 one on gfx950, and FP64 sums lose nothing.
template <int R, int BL, bool FUSE, typename T>
__global__ __launch_bounds__(NSLOT * R * BL) void k_tau_stream(
    const T* __restrict__ tau, long rb_stride, long nblk, const int2* __restrict__ IJ,
    const typename vec2_of<T>::type* a, typename vec2_of<T>::type* y, int nb, int nv, int nvh,
    long nr, int row0, int nrows, int accumulate, const T* __restrict__ V,
    const typename vec2_of<T>::type* __restrict__ vdrho,
    const typename vec2_of<T>::type* __restrict__ phir, T s, int with_v) {
  using V2 = typename vec2_of<T>::type;
  constexpr int NT = NSLOT * R * BL;
  constexpr int NBL = NBT / BL;
  constexpr int RS = NBT * R + SPAD;
  // rows of a tau block loaded ahead of their use: the whole block in FP32
  // (64 registers), two rows in FP64
  constexpr int JU = sizeof(T) == 4 ? 8 : 2;
  extern __shared__ char lds_raw[];
  T* as = reinterpret_cast<T*>(lds_raw);
  double* ys = reinterpret_cast<double*>(as + (long)nrows * RS);
  const long rb = blockIdx.x;
  const long r0 = rb * R;
  const int n_el = nrows * NBT * R;
  for (int e = threadIdx.x; e < n_el; e += NT) {
    const int ri = e % R;
    const int b = (e / R) % NBT;
    const int vl = e / (R * NBT);
    const int v = row0 + vl;
    T av = 0;
    double yv = 0;
    if (v < nv && b < nb) {
      const long gi = ((long)b * nvh + (v >> 1)) * nr + r0 + ri;
      av = reinterpret_cast<const T*>(a + gi)[v & 1];
      if (accumulate) yv = reinterpret_cast<const T*>(y + gi)[v & 1];
    }
    const int li = vl * RS + b * R + ri;
    as[li] = av;
    ys[li] = yv;
  }
  __syncthreads();
  const int bl = threadIdx.x % BL;
  const int ri = (threadIdx.x / BL) % R;
  const int slot = threadIdx.x / (BL * R);
  const long b0 = nblk * slot / NSLOT, b1 = nblk * (slot + 1) / NSLOT;
  const T* tb = tau + rb * rb_stride + ri * 8;
  const int lo = bl * NBL * R + ri;  // lane offset inside an LDS row
  int curI = -1;
  T aI[8][NBL], acc[8][NBL];
  for (long blk = b0; blk < b1; ++blk) {
    const int2 bij = IJ[blk];
    if (bij.x != curI) {
      if (curI >= 0) {
#pragma unroll
        for (int i = 0; i < 8; ++i)
#pragma unroll
          for (int b = 0; b < NBL; ++b)
            atomicAdd(&ys[(curI * 8 + i - row0) * RS + lo + b * R], (double)acc[i][b]);
      }
      curI = bij.x;
#pragma unroll
      for (int i = 0; i < 8; ++i)
#pragma unroll
        for (int b = 0; b < NBL; ++b) {
          aI[i][b] = as[(curI * 8 + i - row0) * RS + lo + b * R];
          acc[i][b] = 0;
        }
    }
    const T* tp = tb + blk * 64 * R;
#pragma unroll 1
    for (int j0 = 0; j0 < 8; j0 += JU) {
      T t[JU][8];
#pragma unroll
      for (int jj = 0; jj < JU; ++jj)
#pragma unroll
        for (int i = 0; i < 8; ++i) t[jj][i] = tp[(j0 + jj) * 8 * R + i];
#pragma unroll
      for (int jj = 0; jj < JU; ++jj) {
        const int wv = bij.y * 8 + j0 + jj - row0;
        T aj[NBL], tr[NBL];
#pragma unroll
        for (int b = 0; b < NBL; ++b) {
          aj[b] = as[wv * RS + lo + b * R];
          tr[b] = 0;
        }
#pragma unroll
        for (int i = 0; i < 8; ++i)
#pragma unroll
          for (int b = 0; b < NBL; ++b) {
            acc[i][b] = fma(t[jj][i], aj[b], acc[i][b]);
            tr[b] = fma(t[jj][i], aI[i][b], tr[b]);
          }
#pragma unroll
        for (int b = 0; b < NBL; ++b) atomicAdd(&ys[wv * RS + lo + b * R], (double)tr[b]);
      }
    }
  }
  if (curI >= 0) {
#pragma unroll
    for (int i = 0; i < 8; ++i)
#pragma unroll
      for (int b = 0; b < NBL; ++b)
        atomicAdd(&ys[(curI * 8 + i - row0) * RS + lo + b * R], (double)acc[i][b]);
  }
  __syncthreads();
  for (int e = threadIdx.x; e < n_el; e += NT) {
    const int rr = e % R;
    const int b = (e / R) % NBT;
    const int vl = e / (R * NBT);
    const int v = row0 + vl;
    if (v < nv && b < nb) {
      const long gi = ((long)b * nvh + (v >> 1)) * nr + r0 + rr;
      const int li = vl * RS + b * R + rr;
      T out = (T)ys[li];
      if (FUSE) {
        const long r = r0 + rr;
        T z = -out;
        if (with_v) z += V[r] * as[li];
        if (vdrho) {
          const T d = reinterpret_cast<const T*>(vdrho + (long)(b >> 1) * nr + r)[b & 1];
          const T f = reinterpret_cast<const T*>(phir + (long)(v >> 1) * nr + r)[v & 1];
          z += s * d * f;
        }
        out = z;
      }
      reinterpret_cast<T*>(y + gi)[v & 1] = out;
    }
  }
}

// ---------------------------------------------------------------------------
// Quad-shared tau stream (the default).  The work layout of k_tau_stream with
// four lanes per grid point (lane bl takes trial vectors 2bl, 2bl+1), but each
// lane reads only columns 2bl and 2bl+1 of a block from memory and the block's
// eight columns reach all four lanes of the quad by DPP broadcasts: every tau
// value leaves the cache once, and the LDS traffic is that of k_tau_stream.
// ---------------------------------------------------------------------------
constexpr int QS_BL = 4;

// Workgroup i runs on XCD i mod 8 (round-robin dispatch).  Give each XCD a
// contiguous range of grid-point blocks, in order, so the workgroups whose
// points share a 128-byte line of a(r) and z(r) run on the same XCD and meet
// in its L2.  A bijection of [0, n) for any n.
__device__ __forceinline__ long xcd_order(long i, long n) {
  constexpr int NX = 8;
  const long q = n / NX, rem = n % NX;
  const long x = i % NX, k = i / NX;
  return x * q + (x < rem ? x : rem) + k;
}

// value of lane `src` of this lane's quad (quad permutation [src x 4])
template <int SRC>
__device__ __forceinline__ float quad_bcast(float x) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), SRC * 0x55, 0xF, 0xF, true));
}
template <int SRC>
__device__ __forceinline__ double quad_bcast(double x) {
  const long long u = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_mov_dpp((int)(u & 0xffffffffLL), SRC * 0x55, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(u >> 32), SRC * 0x55, 0xF, 0xF, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ void load8(double (&v)[8], const double* p) {
  const double2* q = reinterpret_cast<const double2*>(p);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const double2 w = q[k];
    v[2 * k] = w.x;
    v[2 * k + 1] = w.y;
  }
}
__device__ __forceinline__ void load8(float (&v)[8], const float* p) {
  const float4* q = reinterpret_cast<const float4*>(p);
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const float4 w = q[k];
    v[4 * k] = w.x;
    v[4 * k + 1] = w.y;
    v[4 * k + 2] = w.z;
    v[4 * k + 3] = w.w;
  }
}

// one column j of the current block: t[i] = tau[i][j] from the quad lane that
// read it, then acc (row block I) and the transposed contribution to row j
template <int J, int R, typename T>
__device__ __forceinline__ void qs_column(const T (&own)[2][8], T (&acc)[8][2],
                                          const T (&aI)[8][2], const T* as, double* ys,
                                          int rowJ, int lo) {
  constexpr int NBL = 2;
  constexpr int RS = NBT * R + SPAD;
  T t[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) t[i] = quad_bcast<J / 2>(own[J % 2][i]);
  const int wv = rowJ + J;
  T aj[NBL], tr[NBL];
#pragma unroll
  for (int b = 0; b < NBL; ++b) {
    aj[b] = as[wv * RS + lo + b * R];
    tr[b] = 0;
  }
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int b = 0; b < NBL; ++b) {
      acc[i][b] = fma(t[i], aj[b], acc[i][b]);
      tr[b] = fma(t[i], aI[i][b], tr[b]);
    }
#pragma unroll
  for (int b = 0; b < NBL; ++b) atomicAdd(&ys[wv * RS + lo + b * R], (double)tr[b]);
}

template <int R, bool FUSE, typename T>
__global__ __launch_bounds__(NSLOT * R * QS_BL) void k_tau_stream_qs(
    const T* __restrict__ tau, long rb_stride, long nblk, const int2* __restrict__ IJ,
    const typename vec2_of<T>::type* a, typename vec2_of<T>::type* y, int nb, int nv, int nvh,
    long nr, int row0, int nrows, int accumulate, const T* __restrict__ V,
    const typename vec2_of<T>::type* __restrict__ vdrho,
    const typename vec2_of<T>::type* __restrict__ phir, T s, int with_v) {
  constexpr int NT = NSLOT * R * QS_BL;
  constexpr int NBL = NBT / QS_BL;
  constexpr int RS = NBT * R + SPAD;
  extern __shared__ char lds_raw[];
  T* as = reinterpret_cast<T*>(lds_raw);
  double* ys = reinterpret_cast<double*>(as + (long)nrows * RS);
  const long rb = xcd_order(blockIdx.x, gridDim.x);
  const long r0 = rb * R;
  const int n_el = nrows * NBT * R;
  for (int e = threadIdx.x; e < n_el; e += NT) {
    const int ri = e % R;
    const int b = (e / R) % NBT;
    const int vl = e / (R * NBT);
    const int v = row0 + vl;
    T av = 0;
    double yv = 0;
    if (v < nv && b < nb) {
      const long gi = ((long)b * nvh + (v >> 1)) * nr + r0 + ri;
      av = reinterpret_cast<const T*>(a + gi)[v & 1];
      if (accumulate) yv = reinterpret_cast<const T*>(y + gi)[v & 1];
    }
    const int li = vl * RS + b * R + ri;
    as[li] = av;
    ys[li] = yv;
  }
  __syncthreads();
  const int bl = threadIdx.x % QS_BL;
  const int ri = (threadIdx.x / QS_BL) % R;
  const int slot = threadIdx.x / (QS_BL * R);
  const long b0 = nblk * slot / NSLOT, b1 = nblk * (slot + 1) / NSLOT;
  // this lane's two columns (2 bl, 2 bl + 1) of block 0 for its grid point
  const T* tcol = tau + rb * rb_stride + (2 * bl * R + ri) * 8;
  const int lo = bl * NBL * R + ri;  // lane offset inside an LDS row
  int curI = -1;
  T aI[8][NBL], acc[8][NBL];
  // FP32 lanes have the registers to read the next block's columns while the
  // current block is in use; FP64 lanes read each block when they reach it
  constexpr bool PF = sizeof(T) == 4;
  T nxt[2][8];
  if (PF && b0 < b1) {
    load8(nxt[0], tcol + b0 * 64 * R);
    load8(nxt[1], tcol + b0 * 64 * R + 8 * R);
  }
#pragma unroll 1
  for (long blk = b0; blk < b1; ++blk) {
    const int2 bij = IJ[blk];
    T own[2][8];
    if (PF) {
#pragma unroll
      for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int i = 0; i < 8; ++i) own[q][i] = nxt[q][i];
      if (blk + 1 < b1) {
        load8(nxt[0], tcol + (blk + 1) * 64 * R);
        load8(nxt[1], tcol + (blk + 1) * 64 * R + 8 * R);
      }
    } else {
      const T* tp = tcol + blk * 64 * R;
      load8(own[0], tp);
      load8(own[1], tp + 8 * R);
    }
    if (bij.x != curI) {
      if (curI >= 0) {
#pragma unroll
        for (int i = 0; i < 8; ++i)
#pragma unroll
          for (int b = 0; b < NBL; ++b)
            atomicAdd(&ys[(curI * 8 + i - row0) * RS + lo + b * R], (double)acc[i][b]);
      }
      curI = bij.x;
#pragma unroll
      for (int i = 0; i < 8; ++i)
#pragma unroll
        for (int b = 0; b < NBL; ++b) {
          aI[i][b] = as[(curI * 8 + i - row0) * RS + lo + b * R];
          acc[i][b] = 0;
        }
    }
    const int rowJ = bij.y * 8 - row0;
    qs_column<0, R>(own, acc, aI, as, ys, rowJ, lo);
    qs_column<1, R>(own, acc, aI, as, ys, rowJ, lo);
    qs_column<2, R>(own, acc, aI, as, ys, rowJ, lo);
    qs_column<3, R>(own, acc, aI, as, ys, rowJ, lo);
    qs_column<4, R>(own, acc, aI, as, ys, rowJ, lo);
    qs_column<5, R>(own, acc, aI, as, ys, rowJ, lo);
    qs_column<6, R>(own, acc, aI, as, ys, rowJ, lo);
    qs_column<7, R>(own, acc, aI, as, ys, rowJ, lo);
  }
  if (curI >= 0) {
#pragma unroll
    for (int i = 0; i < 8; ++i)
#pragma unroll
      for (int b = 0; b < NBL; ++b)
        atomicAdd(&ys[(curI * 8 + i - row0) * RS + lo + b * R], (double)acc[i][b]);
  }
  __syncthreads();
  for (int e = threadIdx.x; e < n_el; e += NT) {
    const int rr = e % R;
    const int b = (e / R) % NBT;
    const int vl = e / (R * NBT);
    const int v = row0 + vl;
    if (v < nv && b < nb) {
      const long gi = ((long)b * nvh + (v >> 1)) * nr + r0 + rr;
      const int li = vl * RS + b * R + rr;
      T out = (T)ys[li];
      if (FUSE) {
        const long r = r0 + rr;
        T z = -out;
        if (with_v) z += V[r] * as[li];
        if (vdrho) {
          const T d = reinterpret_cast<const T*>(vdrho + (long)(b >> 1) * nr + r)[b & 1];
          const T f = reinterpret_cast<const T*>(phir + (long)(v >> 1) * nr + r)[v & 1];
          z += s * d * f;
        }
        out = z;
      }
      reinterpret_cast<T*>(y + gi)[v & 1] = out;
    }
  }
}

// ---------------------------------------------------------------------------
// potential, Coulomb kernel, forces
// ---------------------------------------------------------------------------
__device__ __forceinline__ int min_image(int i, int n) { return (i < (n + 1) / 2) ? i : i - n; }

__global__ void k_site_potential(const double* __restrict__ xyz, const double* __restrict__ depth,
                                 const double* __restrict__ width, int nsites, int N1, int N2,
                                 int N3, double L1, double L2, double L3, double omega,
                                 double2* __restrict__ out) {
  const long nr = (long)N1 * N2 * N3;
  const double tp = 6.283185307179586477;
  for (long e = gtid(); e < nr; e += gstride()) {
    const int i3 = (int)(e % N3);
    const int i2 = (int)((e / N3) % N2);
    const int i1 = (int)(e / ((long)N2 * N3));
    const int n1 = min_image(i1, N1), n2 = min_image(i2, N2), n3 = min_image(i3, N3);
    const bool nyq = ((N1 % 2 == 0) && n1 == -N1 / 2) || ((N2 % 2 == 0) && n2 == -N2 / 2) ||
                     ((N3 % 2 == 0) && n3 == -N3 / 2);
    double re = 0.0, im = 0.0;
    if (!nyq) {
      const double gx = tp * n1 / L1, gy = tp * n2 / L2, gz = tp * n3 / L3;
      const double g2 = gx * gx + gy * gy + gz * gz;
      for (int s = 0; s < nsites; ++s) {
        const double w = width[s];
        const double amp = -(depth[s] / omega) * pow(tp * w * w, 1.5) * exp(-0.5 * w * w * g2);
        const double th = gx * xyz[3 * s] + gy * xyz[3 * s + 1] + gz * xyz[3 * s + 2];
        double sn, cs;
        sincos(th, &sn, &cs);
        re += amp * cs;
        im -= amp * sn;
      }
    }
    out[e] = make_double2(re, im);
  }
}

__global__ void k_coulomb(int N1, int N2, int N3, double L1, double L2, double L3,
                          double* __restrict__ out) {
  const long nr = (long)N1 * N2 * N3;
  const double tp = 6.283185307179586477;
  for (long e = gtid(); e < nr; e += gstride()) {
    const int i3 = (int)(e % N3);
    const int i2 = (int)((e / N3) % N2);
    const int i1 = (int)(e / ((long)N2 * N3));
    const double gx = tp * min_image(i1, N1) / L1, gy = tp * min_image(i2, N2) / L2,
                 gz = tp * min_image(i3, N3) / L3;
    const double g2 = gx * gx + gy * gy + gz * gz;
    out[e] = (e == 0) ? 0.0 : 4.0 * M_PI / g2;
  }
}

__global__ void k_force_density(const double2* __restrict__ a, const double2* __restrict__ phit,
                                const double2* __restrict__ z, const double2* __restrict__ phir,
                                int nvh, long nr, double2* __restrict__ rho) {
  for (long r = gtid(); r < nr; r += gstride()) {
    double s = 0.0;
    for (int p = 0; p < nvh; ++p) {
      const long i = (long)p * nr + r;
      const double2 x = a[i], t = phit[i], q = z[i], f = phir[i];
      s += x.x * x.x + x.y * x.y - (f.x * t.x + f.y * t.y) + 2.0 * (q.x * f.x + q.y * f.y);
    }
    rho[r] = make_double2(s, 0.0);
  }
}

// ---------------------------------------------------------------------------
// self-consistent Kohn-Sham model: local exchange-correlation fields
// ---------------------------------------------------------------------------
// From rho_occ = sum_v phi_v^2 (real part of the grid): rho = occ rho_occ,
//   V_xc  = -(3/pi)^(1/3) [ (rho + f)^(1/3) - f^(1/3) ]
//   f_xc  = dV_xc/drho = -(1/3)(3/pi)^(1/3) (rho + f)^(-2/3)
// (Slater exchange with a density floor f).  rho_out may be null.
__global__ void k_xc_fields(const double2* __restrict__ rho_occ, long nr, double occ, double f,
                            double* __restrict__ vxc, double* __restrict__ fxc,
                            double* __restrict__ rho_out) {
  const double cx = 0.98474502184269654;  // (3/pi)^(1/3)
  const double f3 = cbrt(f);
  for (long r = gtid(); r < nr; r += gstride()) {
    const double rho = occ * rho_occ[r].x;
    const double q = cbrt(rho + f);
    vxc[r] = -cx * (q - f3);
    fxc[r] = -(cx / 3.0) / (q * q);
    if (rho_out) rho_out[r] = rho;
  }
}

// w = scale (w + f_xc t) on both components: f_Hxc * t once w holds v_c * t
__global__ void k_hxc_field(double2* __restrict__ w, const double2* __restrict__ t,
                            const double* __restrict__ fxc, long ngrid, long nr, double scale) {
  const long n = ngrid * nr;
  for (long e = gtid(); e < n; e += gstride()) {
    const double fx = fxc[e % nr];
    const double2 a = w[e], b = t[e];
    w[e] = make_double2(scale * (a.x + fx * b.x), scale * (a.y + fx * b.y));
  }
}

// exchange-like terms: pair grids q = (M_2q x, M_2q+1 x) for one real grid
// function x (component xc of the packed grid x2)
__global__ void k_pair_times(const double2* __restrict__ M, int nvh, const double2* __restrict__ x2,
                             int xc, long nr, double2* __restrict__ out) {
  const long n = (long)nvh * nr;
  for (long e = gtid(); e < n; e += gstride()) {
    const long r = e % nr;
    const double2 xv = x2[r];
    const double x = xc ? xv.y : xv.x;
    const double2 m = M[e];
    out[e] = make_double2(m.x * x, m.y * x);
  }
}

// out (component oc of the packed grid o2) += scale sum_w L_w(r) P_w(r)
__global__ void k_contract_pairs(const double2* __restrict__ L, const double2* __restrict__ P,
                                 int nvh, long nr, double2* __restrict__ o2, int oc,
                                 double scale) {
  for (long r = gtid(); r < nr; r += gstride()) {
    double s = 0.0;
    for (int q = 0; q < nvh; ++q) {
      const double2 l = L[(long)q * nr + r], p = P[(long)q * nr + r];
      s += l.x * p.x + l.y * p.y;
    }
    double2 o = o2[r];
    if (oc)
      o.y += scale * s;
    else
      o.x += scale * s;
    o2[r] = o;
  }
}

// occupied density sum_v phi_v(r)^2 (two orbitals per complex grid)
__global__ void k_occupied_density(const double2* __restrict__ phir, int nvh, long nr,
                                   double2* __restrict__ rho) {
  for (long r = gtid(); r < nr; r += gstride()) {
    double s = 0.0;
    for (int p = 0; p < nvh; ++p) {
      const double2 f = phir[(long)p * nr + r];
      s += f.x * f.x + f.y * f.y;
    }
    rho[r] = make_double2(s, 0.0);
  }
}

// part[site][chunk][3]; G over chunk ranges; fixed-order tree reduction
__global__ __launch_bounds__(256) void k_force_partial(
    const double2* __restrict__ rhoG, const double* __restrict__ xyz,
    const double* __restrict__ depth, const double* __restrict__ width, int N1, int N2, int N3,
    double L1, double L2, double L3, double omega, long chunk, double* __restrict__ part) {
  __shared__ double red[3][256];
  const int site = blockIdx.y;
  const long nr = (long)N1 * N2 * N3;
  const long g0 = (long)blockIdx.x * chunk;
  const long g1 = min(nr, g0 + chunk);
  const double tp = 6.283185307179586477;
  const double w = width[site];
  const double cI = (depth[site] / omega) * pow(tp * w * w, 1.5);
  const double R0 = xyz[3 * site], R1 = xyz[3 * site + 1], R2 = xyz[3 * site + 2];
  double s0 = 0, s1 = 0, s2 = 0;
  for (long e = g0 + threadIdx.x; e < g1; e += 256) {
    const int i3 = (int)(e % N3);
    const int i2 = (int)((e / N3) % N2);
    const int i1 = (int)(e / ((long)N2 * N3));
    const int n1 = min_image(i1, N1), n2 = min_image(i2, N2), n3 = min_image(i3, N3);
    const bool nyq = ((N1 % 2 == 0) && n1 == -N1 / 2) || ((N2 % 2 == 0) && n2 == -N2 / 2) ||
                     ((N3 % 2 == 0) && n3 == -N3 / 2);
    if (nyq) continue;
    const double gx = tp * n1 / L1, gy = tp * n2 / L2, gz = tp * n3 / L3;
    const double g2 = gx * gx + gy * gy + gz * gz;
    double sn, cs;
    sincos(gx * R0 + gy * R1 + gz * R2, &sn, &cs);
    const double2 rg = rhoG[e];
    const double f = cI * exp(-0.5 * w * w * g2) * (sn * rg.x + cs * rg.y);
    s0 += gx * f;
    s1 += gy * f;
    s2 += gz * f;
  }
  red[0][threadIdx.x] = s0;
  red[1][threadIdx.x] = s1;
  red[2][threadIdx.x] = s2;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h)
      for (int c = 0; c < 3; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int c = 0; c < 3; ++c) part[((long)site * gridDim.x + blockIdx.x) * 3 + c] = red[c][0];
}

__global__ void k_force_final(const double* __restrict__ part, int nsites, int nchunk, double scale,
                              double* __restrict__ out) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nsites * 3) return;
  const int site = e / 3, c = e % 3;
  double s = 0.0;
  for (int k = 0; k < nchunk; ++k) s += part[((long)site * nchunk + k) * 3 + c];
  out[e] = scale * s;
}

// ---------------------------------------------------------------------------
// solver vector helpers
// ---------------------------------------------------------------------------
// partial dot products of rows: grid (nsplit, rows); block s of row r sums the
// s-th of nsplit equal chunks
__global__ __launch_bounds__(256) void k_row_dots(const double* __restrict__ A,
                                                  const double* __restrict__ B, long len,
                                                  int nsplit, double* __restrict__ part) {
  __shared__ double red[256];
  const long row = blockIdx.y;
  const long chunk = (len + nsplit - 1) / nsplit;
  const long j0 = blockIdx.x * chunk;
  const long j1 = j0 + chunk < len ? j0 + chunk : len;
  const double* a = A + row * len;
  const double* b = B + row * len;
  double s = 0.0;
  for (long j = j0 + threadIdx.x; j < j1; j += 256) s += a[j] * b[j];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[row * nsplit + blockIdx.x] = red[0];
}

__global__ void k_row_dots_final(const double* __restrict__ part, long rows, int nsplit,
                                 double* __restrict__ out) {
  const long r = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= rows) return;
  double s = 0.0;
  for (int q = 0; q < nsplit; ++q) s += part[r * nsplit + q];
  out[r] = s;
}

__global__ void k_zero(double* __restrict__ p, long n) {
  for (long e = gtid(); e < n; e += gstride()) p[e] = 0.0;
}

__global__ void k_row_axpby(const double* __restrict__ a, const double* __restrict__ X,
                            const double* __restrict__ b, double* __restrict__ Y, long rows,
                            long len) {
  for (long e = gtid(); e < rows * len; e += gstride()) {
    const long r = e / len;
    const double av = a ? a[r] : 1.0;
    const double bv = b ? b[r] : 1.0;
    Y[e] = av * X[e] + bv * Y[e];
  }
}

__global__ void k_row_scale(const double* __restrict__ s, double* __restrict__ Y, long rows,
                            long len) {
  for (long e = gtid(); e < rows * len; e += gstride()) Y[e] *= s[e / len];
}

// Y[b][v][k] += (T_k - eps_v + shift) A[b][v][k]: the diagonal part of D
__global__ void k_diag_axpy(const double* __restrict__ A, const double* __restrict__ Tk,
                            const double* __restrict__ eps, double shift, int nv, long npw, long n,
                            double* __restrict__ Y) {
  for (long e = gtid(); e < n; e += gstride()) {
    const long k = e % npw;
    const int v = (int)((e / npw) % nv);
    Y[e] += (Tk[k] - eps[v] + shift) * A[e];
  }
}

__global__ void k_axpby(double alpha, const double* __restrict__ X, double beta,
                        double* __restrict__ Y, long n) {
  for (long e = gtid(); e < n; e += gstride()) Y[e] = alpha * X[e] + (beta == 0.0 ? 0.0 : beta * Y[e]);
}

__global__ void k_precond_davidson(const double* __restrict__ R, double* __restrict__ T,
                                   const double* __restrict__ Tk, const double* __restrict__ eps,
                                   const double* __restrict__ theta, double shift, int nk, int nv,
                                   int npw, const double* __restrict__ vshift) {
  const long n = (long)nk * nv * npw;
  for (long e = gtid(); e < n; e += gstride()) {
    const int j = (int)(e % npw);
    const int v = (int)((e / npw) % nv);
    const int k = (int)(e / ((long)npw * nv));
    double den = Tk[j] - eps[v] + shift + (vshift ? vshift[v] : 0.0) - theta[k];
    if (fabs(den) < 0.1) den = (den < 0.0) ? -0.1 : 0.1;
    T[e] = R[e] / den;
  }
}

__global__ void k_precond_cg(const double* __restrict__ R, double* __restrict__ T,
                             const double* __restrict__ Tk, const double* __restrict__ eps,
                             double shift, int nv, int npw, const double* __restrict__ vshift) {
  const long n = (long)nv * npw;
  for (long e = gtid(); e < n; e += gstride()) {
    const int j = (int)(e % npw);
    const int v = (int)(e / npw);
    const double den = fmax(Tk[j] - eps[v] + (vshift ? vshift[v] : shift), 0.1);
    T[e] = R[e] / den;
  }
}

__global__ void k_coarse_scale(double* __restrict__ C, int nk, int nv, int nc,
                               const double* __restrict__ eps, const double* __restrict__ theta,
                               double shift, double dmin) {
  const long n = (long)nk * nv * nc;
  for (long e = gtid(); e < n; e += gstride()) {
    const int cc = (int)(e % nc);
    const int v = (int)((e / nc) % nv);
    const int k = (int)(e / ((long)nc * nv));
    double den = eps[nv + cc] - eps[v] + shift - (theta ? theta[k] : 0.0);
    if (fabs(den) < dmin) den = den < 0.0 ? -dmin : dmin;
    C[e] /= den;
  }
}

// one workgroup per band, fixed-order tree reductions
__global__ __launch_bounds__(256) void k_band_features(
    const double* __restrict__ Phi, const double* __restrict__ Tk, const double* __restrict__ eps,
    const double* __restrict__ U, const double2* __restrict__ phir, double shift, int npw, long nr,
    double* __restrict__ out) {
  __shared__ double sh[4][256];
  const int v = blockIdx.x;
  const double* ph = Phi + (long)v * npw;
  const double* u = U ? U + (long)v * npw : nullptr;
  double a = 0, b = 0, c = 0, d = 0;
  for (int j = threadIdx.x; j < npw; j += 256) {
    a += Tk[j] * ph[j] * ph[j];
    if (u) {
      const double uu = u[j] * u[j];
      b += uu;
      c += uu / fmax(Tk[j] - eps[v] + shift, 0.1);
    }
  }
  const double* pr = reinterpret_cast<const double*>(phir + (long)(v >> 1) * nr) + (v & 1);
  for (long r = threadIdx.x; r < nr; r += 256) {
    const double f = pr[2 * r];
    d += f * f * f * f;
  }
  sh[0][threadIdx.x] = a;
  sh[1][threadIdx.x] = b;
  sh[2][threadIdx.x] = c;
  sh[3][threadIdx.x] = d;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h)
      for (int q = 0; q < 4; ++q) sh[q][threadIdx.x] += sh[q][threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x < 4) out[(long)v * 4 + threadIdx.x] = sh[threadIdx.x][0];
}

}  // namespace

// ============================================================================
// launchers
// ============================================================================
#define CHECK_LAUNCH() BSE_HIP(hipGetLastError())

template <typename V2, typename XT>
static int scatter_impl(const SphereMap& m, const XT* X, int nv, int nset, V2* grid,
                        int accumulate, hipStream_t st) {
  const int nvh = (nv + 1) / 2;
  const long ngrid = (long)nset * nvh;
  if (ngrid <= 0) return BSE_OK;
  const int nbx = (m.nhalf + 1 + TPB - 1) / TPB;
  const bool group = xcd_group_on();
  const long nblk = (long)nbx * (group ? round8(ngrid) : ngrid);
  if (nblk > 0x7fffffffL) return fail(BSE_EINVAL, "scatter: %ld workgroups", nblk);
  hipLaunchKernelGGL((k_scatter<V2, XT>), dim3((unsigned)nblk), dim3(TPB), 0, st, m.idx_p, m.idx_m,
                     m.nhalf, m.npw, m.nr, m.zero, X, nv, nvh, ngrid, nbx, (int)group, grid,
                     accumulate, 1.0 / std::sqrt(m.omega), 1.0 / std::sqrt(2.0 * m.omega));
  CHECK_LAUNCH();
  return BSE_OK;
}

int scatter_sets(const SphereMap& m, const double* X, int nv, int nset, double2* grid,
                 int accumulate, hipStream_t st) {
  return scatter_impl(m, X, nv, nset, grid, accumulate, st);
}

int scatter_sets(const SphereMap& m, const double* X, int nv, int nset, float2* grid,
                 int accumulate, hipStream_t st) {
  return scatter_impl(m, X, nv, nset, grid, accumulate, st);
}

int scatter_sets(const SphereMap& m, const float* X, int nv, int nset, float2* grid,
                 int accumulate, hipStream_t st) {
  return scatter_impl(m, X, nv, nset, grid, accumulate, st);
}

template <typename V2, typename YT>
static int gather_impl(const SphereMap& m, const V2* grid, int nv, int nset, double scale,
                       const double* A, const double* T, const double* eps, double shift,
                       double beta, YT* Y, hipStream_t st) {
  const int nvh = (nv + 1) / 2;
  const long ngrid = (long)nset * nvh;
  if (ngrid <= 0) return BSE_OK;
  const int nbx = (m.nhalf + 1 + TPB - 1) / TPB;
  const bool group = xcd_group_on();
  const long nblk = (long)nbx * (group ? round8(ngrid) : ngrid);
  if (nblk > 0x7fffffffL) return fail(BSE_EINVAL, "gather: %ld workgroups", nblk);
  hipLaunchKernelGGL((k_gather<V2, YT>), dim3((unsigned)nblk), dim3(TPB), 0, st, m.idx_p, m.idx_m,
                     m.nhalf, m.npw, m.nr, m.zero, grid, nv, nvh, ngrid, nbx, (int)group,
                     scale * std::sqrt(m.omega), scale * std::sqrt(2.0 * m.omega), A, T, eps,
                     shift, beta, Y);
  CHECK_LAUNCH();
  return BSE_OK;
}

int gather_sets(const SphereMap& m, const double2* grid, int nv, int nset, double scale,
                const double* A, const double* T, const double* eps, double shift, double beta,
                double* Y, hipStream_t st) {
  return gather_impl(m, grid, nv, nset, scale, A, T, eps, shift, beta, Y, st);
}

int gather_sets(const SphereMap& m, const float2* grid, int nv, int nset, double scale,
                const double* A, const double* T, const double* eps, double shift, double beta,
                double* Y, hipStream_t st) {
  return gather_impl(m, grid, nv, nset, scale, A, T, eps, shift, beta, Y, st);
}

int gather_sets(const SphereMap& m, const float2* grid, int nv, int nset, double scale, float* Y,
                hipStream_t st) {
  return gather_impl(m, grid, nv, nset, scale, (const double*)nullptr, (const double*)nullptr,
                     (const double*)nullptr, 0.0, 0.0, Y, st);
}

int mul_real_field(double2* grid, long ngrid, long nr, const double* f, double scale,
                   hipStream_t st) {
  const long n = ngrid * nr;
  if (n <= 0) return BSE_OK;
  hipLaunchKernelGGL((k_mul_real<double2, double>), dim3(nblocks(n)), dim3(TPB), 0, st, grid, n,
                     nr, f, scale);
  CHECK_LAUNCH();
  return BSE_OK;
}

int mul_real_field(float2* grid, long ngrid, long nr, const float* f, float scale,
                   hipStream_t st) {
  const long n = ngrid * nr;
  if (n <= 0) return BSE_OK;
  hipLaunchKernelGGL((k_mul_real<float2, float>), dim3(nblocks(n)), dim3(TPB), 0, st, grid, n, nr,
                     f, scale);
  CHECK_LAUNCH();
  return BSE_OK;
}

int xc_fields(const double2* rho_occ, long nr, double occ, double floor_, double* vxc,
              double* fxc, double* rho_out, hipStream_t st) {
  hipLaunchKernelGGL(k_xc_fields, dim3(nblocks(nr)), dim3(TPB), 0, st, rho_occ, nr, occ, floor_,
                     vxc, fxc, rho_out);
  CHECK_LAUNCH();
  return BSE_OK;
}

int hxc_field(double2* w, const double2* t, const double* fxc, long ngrid, long nr, double scale,
              hipStream_t st) {
  hipLaunchKernelGGL(k_hxc_field, dim3(nblocks(ngrid * nr)), dim3(TPB), 0, st, w, t, fxc, ngrid,
                     nr, scale);
  CHECK_LAUNCH();
  return BSE_OK;
}

int pair_times(const double2* M, int nv, const double2* x2, int xc, long nr, double2* out,
               hipStream_t st) {
  const int nvh = (nv + 1) / 2;
  hipLaunchKernelGGL(k_pair_times, dim3(nblocks((long)nvh * nr)), dim3(TPB), 0, st, M, nvh, x2, xc,
                     nr, out);
  CHECK_LAUNCH();
  return BSE_OK;
}

int contract_pairs(const double2* L, const double2* P, int nv, long nr, double2* o2, int oc,
                   double scale, hipStream_t st) {
  hipLaunchKernelGGL(k_contract_pairs, dim3(nblocks(nr)), dim3(TPB), 0, st, L, P, (nv + 1) / 2,
                     nr, o2, oc, scale);
  CHECK_LAUNCH();
  return BSE_OK;
}

int real_part(const double2* grid, long nr, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_real_part, dim3(nblocks(nr)), dim3(TPB), 0, st, grid, nr, out);
  CHECK_LAUNCH();
  return BSE_OK;
}

int transition_density(const double2* phir, const double2* a, int nv, int nb, long nr,
                       double2* drho, hipStream_t st) {
  const long n = (long)((nb + TD_B - 1) / TD_B) * nr;
  if (n <= 0) return BSE_OK;
  hipLaunchKernelGGL((k_transition_density<double2, double>), dim3(nblocks(n)), dim3(TPB), 0, st,
                     phir, a, (nv + 1) / 2, nb, nr, drho);
  CHECK_LAUNCH();
  return BSE_OK;
}

int transition_density(const float2* phir, const float2* a, int nv, int nb, long nr, float2* drho,
                       hipStream_t st) {
  const long n = (long)((nb + TD_B - 1) / TD_B) * nr;
  if (n <= 0) return BSE_OK;
  hipLaunchKernelGGL((k_transition_density<float2, float>), dim3(nblocks(n)), dim3(TPB), 0, st,
                     phir, a, (nv + 1) / 2, nb, nr, drho);
  CHECK_LAUNCH();
  return BSE_OK;
}

__global__ void k_to_f32(const double* __restrict__ x, float* __restrict__ y, long n) {
  for (long e = gtid(); e < n; e += gstride()) y[e] = (float)x[e];
}

int to_f32(const double* x, float* y, long n, hipStream_t st) {
  if (n <= 0) return BSE_OK;
  hipLaunchKernelGGL(k_to_f32, dim3(nblocks(n)), dim3(TPB), 0, st, x, y, n);
  CHECK_LAUNCH();
  return BSE_OK;
}

// SplitMix64 finaliser (Steele, Lea and Flood, OOPSLA 2014) as a counter-based
// generator: element e of stream seed draws from mix(seed, e) only, so the
// result does not depend on the launch shape.
__device__ __forceinline__ unsigned long long mix64(unsigned long long z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}

// X[i][j] = g_ij / (1 + T_j), g_ij standard normal (Box-Muller on two 32-bit
// uniforms of one 64-bit draw)
__global__ void k_random_smooth(double* __restrict__ X, long rows, long len,
                                const double* __restrict__ T, unsigned long long seed) {
  const long n = rows * len;
  for (long e = gtid(); e < n; e += gstride()) {
    const unsigned long long h = mix64(seed + 0x9e3779b97f4a7c15ULL * (unsigned long long)(e + 1));
    const double u1 = ((double)(h >> 32) + 1.0) * 2.3283064365386963e-10;  // (0, 1]
    const double u2 = (double)(h & 0xffffffffULL) * 2.3283064365386963e-10;  // [0, 1)
    const double g = sqrt(-2.0 * log(u1)) * cos(6.283185307179586477 * u2);
    X[e] = g / (1.0 + T[e % len]);
  }
}

int random_smooth(double* X, long rows, long len, const double* T, unsigned long long seed,
                  hipStream_t st) {
  const long n = rows * len;
  if (n <= 0) return BSE_OK;
  hipLaunchKernelGGL(k_random_smooth, dim3(nblocks(n)), dim3(TPB), 0, st, X, rows, len, T, seed);
  CHECK_LAUNCH();
  return BSE_OK;
}

__global__ void k_to_f64(const float* __restrict__ x, double* __restrict__ y, long n) {
  for (long e = gtid(); e < n; e += gstride()) y[e] = (double)x[e];
}

int to_f64(const float* x, double* y, long n, hipStream_t st) {
  if (n <= 0) return BSE_OK;
  hipLaunchKernelGGL(k_to_f64, dim3(nblocks(n)), dim3(TPB), 0, st, x, y, n);
  CHECK_LAUNCH();
  return BSE_OK;
}

int combine(const double2* a, const double2* phir, const double* V, const double2* vdrho,
            const double2* y, double2* out, int nv, int nb, long nr, double s, int with_v,
            hipStream_t st) {
  const long n = (long)nb * ((nv + 1) / 2) * nr;
  if (n <= 0) return BSE_OK;
  hipLaunchKernelGGL((k_combine<double2, double>), dim3(nblocks(n)), dim3(TPB), 0, st, a, phir, V,
                     vdrho, y, out, (nv + 1) / 2, nb, nr, s, with_v);
  CHECK_LAUNCH();
  return BSE_OK;
}

int combine(const float2* a, const float2* phir, const float* V, const float2* vdrho,
            const float2* y, float2* out, int nv, int nb, long nr, double s, int with_v,
            hipStream_t st) {
  const long n = (long)nb * ((nv + 1) / 2) * nr;
  if (n <= 0) return BSE_OK;
  hipLaunchKernelGGL((k_combine<float2, float>), dim3(nblocks(n)), dim3(TPB), 0, st, a, phir, V,
                     vdrho, y, out, (nv + 1) / 2, nb, nr, (float)s, with_v);
  CHECK_LAUNCH();
  return BSE_OK;
}

template <typename V2>
static int pair_density_impl(const V2* phir, int nv, const int2* blkIJ, long nblk, long nr,
                             V2* grids, hipStream_t st) {
  const long n = nblk * 32 * nr;
  if (n <= 0) return BSE_OK;
  hipLaunchKernelGGL((k_pair_density<V2>), dim3(nblocks(n)), dim3(TPB), 0, st, phir, nv, blkIJ,
                     nblk, nr, grids);
  CHECK_LAUNCH();
  return BSE_OK;
}

int pair_density(const double2* phir, int nv, const int2* blkIJ, long nblk, long nr,
                 double2* grids, hipStream_t st) {
  return pair_density_impl(phir, nv, blkIJ, nblk, nr, grids, st);
}

int pair_density(const float2* phir, int nv, const int2* blkIJ, long nblk, long nr,
                 float2* grids, hipStream_t st) {
  return pair_density_impl(phir, nv, blkIJ, nblk, nr, grids, st);
}

static bool tau_store_lds_on() {
  static const bool on = [] {
    const char* e = getenv("BSEX_TAU_STORE_LDS");
    return !e || atoi(e) != 0;
  }();
  return on;
}

template <typename G2, typename TD>
static int tau_store_impl(const G2* grids, const int2* blkIJ, long nblk, long nr, int R,
                          TD* dst, long dst_nblk, long dst_blk0, hipStream_t st) {
  const long n = (nr / R) * nblk * 64 * R;
  if (n <= 0) return BSE_OK;
  if (tau_store_lds_on() && (R == 1 || R == 2)) {
    const long nrb = nr / R;
    const long npg = (nrb + TS_P / R - 1) / (TS_P / R);
    const long nwg = npg * ((nblk + TS_NB - 1) / TS_NB);
    if (nwg > 0x7fffffffL) return fail(BSE_EINVAL, "tau store: %ld workgroups", nwg);
    if (R == 2)
      hipLaunchKernelGGL((k_tau_store_lds<G2, TD, 2>), dim3((unsigned)nwg), dim3(256), 0, st,
                         grids, blkIJ, nblk, nr, dst, dst_nblk, dst_blk0);
    else
      hipLaunchKernelGGL((k_tau_store_lds<G2, TD, 1>), dim3((unsigned)nwg), dim3(256), 0, st,
                         grids, blkIJ, nblk, nr, dst, dst_nblk, dst_blk0);
    CHECK_LAUNCH();
    return BSE_OK;
  }
  hipLaunchKernelGGL((k_tau_store<G2, TD>), dim3(nblocks(n)), dim3(TPB), 0, st, grids, blkIJ, nblk,
                     nr, R, dst, dst_nblk, dst_blk0);
  CHECK_LAUNCH();
  return BSE_OK;
}

int tau_store(const double2* grids, const int2* blkIJ, long nblk, long nr, int R, double* dst,
              long dst_nblk, long dst_blk0, hipStream_t st) {
  return tau_store_impl(grids, blkIJ, nblk, nr, R, dst, dst_nblk, dst_blk0, st);
}

int tau_store(const double2* grids, const int2* blkIJ, long nblk, long nr, int R, float* dst,
              long dst_nblk, long dst_blk0, hipStream_t st) {
  return tau_store_impl(grids, blkIJ, nblk, nr, R, dst, dst_nblk, dst_blk0, st);
}

int tau_store(const float2* grids, const int2* blkIJ, long nblk, long nr, int R, float* dst,
              long dst_nblk, long dst_blk0, hipStream_t st) {
  return tau_store_impl(grids, blkIJ, nblk, nr, R, dst, dst_nblk, dst_blk0, st);
}

size_t tau_stream_lds(int nv, int R, size_t elem, int bl) {
  (void)bl;  // every variant stages the same LDS rows
  const int nv8 = (nv + 7) / 8 * 8;
  return (elem + sizeof(double)) * (size_t)nv8 * (NBT * R + SPAD);
}

template <int R, bool F, typename T>
static void launch_stream_qs(long nrb, size_t shm, hipStream_t st, const T* tau, long stride,
                             long nblk, const int2* blkIJ, const typename vec2_of<T>::type* a,
                             typename vec2_of<T>::type* y, int nb, int nv, long nr, int row0,
                             int nrows, int accumulate, const T* V,
                             const typename vec2_of<T>::type* vdrho,
                             const typename vec2_of<T>::type* phir, T s, int with_v) {
  hipLaunchKernelGGL((k_tau_stream_qs<R, F, T>), dim3((unsigned)nrb), dim3(NSLOT * R * QS_BL),
                     shm, st, tau, stride, nblk, blkIJ, a, y, nb, nv, (nv + 1) / 2, nr, row0,
                     nrows, accumulate, V, vdrho, phir, s, with_v);
}

template <int R, int BL, bool F, typename T>
static void launch_stream(long nrb, size_t shm, hipStream_t st, const T* tau, long stride,
                          long nblk, const int2* blkIJ, const typename vec2_of<T>::type* a,
                          typename vec2_of<T>::type* y, int nb, int nv, long nr, int row0,
                          int nrows, int accumulate, const T* V,
                          const typename vec2_of<T>::type* vdrho,
                          const typename vec2_of<T>::type* phir, T s, int with_v) {
  hipLaunchKernelGGL((k_tau_stream<R, BL, F, T>), dim3((unsigned)nrb), dim3(NSLOT * R * BL), shm,
                     st, tau, stride, nblk, blkIJ, a, y, nb, nv, (nv + 1) / 2, nr, row0, nrows,
                     accumulate, V, vdrho, phir, s, with_v);
}

template <typename T, typename FA>
static int tau_stream_impl(const T* tau, long buf_nblk, long nblk, const int2* blkIJ, int R,
                           const typename vec2_of<T>::type* a, typename vec2_of<T>::type* y,
                           int nb, int nv, long nr, int accumulate, size_t max_lds,
                           hipStream_t st, const FA* fuse, int bl, int row0, int rows) {
  if (nb > NBT) return fail(BSE_EINVAL, "tau_stream: at most %d vectors per call", NBT);
  if (nr % R) return fail(BSE_EINVAL, "tau_stream: grid size not a multiple of %d", R);
  const int nv8 = (nv + 7) / 8 * 8;
  if (rows <= 0) {
    row0 = 0;
    rows = nv8;
  }
  if (row0 < 0 || row0 % 8 || rows % 8 || row0 + rows > nv8)
    return fail(BSE_EINVAL, "tau_stream: band rows %d..%d outside 0..%d", row0, row0 + rows, nv8);
  if (fuse && rows != nv8) return fail(BSE_EINVAL, "tau_stream: the fused epilogue needs every band");
  const size_t shm = tau_stream_lds(rows, R, sizeof(T), bl);
  if (shm > max_lds) return fail(BSE_EINVAL, "tau_stream: %zu bytes of LDS exceed %zu", shm, max_lds);
  const long nrb = nr / R;
  if (nrb > 0x7fffffffL) return fail(BSE_EINVAL, "tau_stream: grid too large");
  const long stride = buf_nblk * 64 * R;
  const T* V = fuse ? fuse->V : nullptr;
  const typename vec2_of<T>::type* vd = fuse ? fuse->vdrho : nullptr;
  const typename vec2_of<T>::type* ph = fuse ? fuse->phir : nullptr;
  const T sf = fuse ? (T)fuse->s : (T)0;
  const int wv = fuse ? fuse->with_v : 0;
#define GO(R_, BL_)                                                                              \
  do {                                                                                           \
    if (fuse)                                                                                    \
      launch_stream<R_, BL_, true, T>(nrb, shm, st, tau, stride, nblk, blkIJ, a, y, nb, nv, nr,   \
                                      row0, rows, accumulate, V, vd, ph, sf, wv);                \
    else                                                                                         \
      launch_stream<R_, BL_, false, T>(nrb, shm, st, tau, stride, nblk, blkIJ, a, y, nb, nv, nr,  \
                                       row0, rows, accumulate, V, vd, ph, sf, wv);               \
  } while (0)
#define GO_QS(R_)                                                                                \
  do {                                                                                           \
    if (fuse)                                                                                    \
      launch_stream_qs<R_, true, T>(nrb, shm, st, tau, stride, nblk, blkIJ, a, y, nb, nv, nr,     \
                                    row0, rows, accumulate, V, vd, ph, sf, wv);                  \
    else                                                                                         \
      launch_stream_qs<R_, false, T>(nrb, shm, st, tau, stride, nblk, blkIJ, a, y, nb, nv, nr,    \
                                     row0, rows, accumulate, V, vd, ph, sf, wv);                 \
  } while (0)
  if (R == 2 && bl == 1)
    GO_QS(2);
  else if (R == 1 && bl == 1)
    GO_QS(1);
  else if (R == 2 && bl == 4)
    GO(2, 4);
  else if (R == 2 && bl == 2)
    GO(2, 2);
  else if (R == 1 && bl == 4)
    GO(1, 4);
  else if (R == 1 && bl == 2)
    GO(1, 2);
  else
    return fail(BSE_EINVAL, "tau_stream: R = %d, BL = %d unsupported", R, bl);
#undef GO
#undef GO_QS
  CHECK_LAUNCH();
  return BSE_OK;
}

int tau_stream(const double* tau, long buf_nblk, long nblk, const int2* blkIJ, int R,
               const double2* a, double2* y, int nb, int nv, long nr, int accumulate,
               size_t max_lds, hipStream_t st, const FuseArgs* fuse, int bl, int row0, int rows) {
  return tau_stream_impl(tau, buf_nblk, nblk, blkIJ, R, a, y, nb, nv, nr, accumulate, max_lds, st,
                         fuse, bl, row0, rows);
}

int tau_stream(const float* tau, long buf_nblk, long nblk, const int2* blkIJ, int R,
               const float2* a, float2* y, int nb, int nv, long nr, int accumulate,
               size_t max_lds, hipStream_t st, const FuseArgsF* fuse, int bl, int row0, int rows) {
  return tau_stream_impl(tau, buf_nblk, nblk, blkIJ, R, a, y, nb, nv, nr, accumulate, max_lds, st,
                         fuse, bl, row0, rows);
}

int tau_stream_set_lds_limit(size_t bytes) {
  const void* fns[] = {
      (const void*)k_tau_stream<2, 4, false, double>, (const void*)k_tau_stream<2, 2, false, double>,
      (const void*)k_tau_stream<1, 4, false, double>, (const void*)k_tau_stream<1, 2, false, double>,
      (const void*)k_tau_stream<2, 4, true, double>,  (const void*)k_tau_stream<2, 2, true, double>,
      (const void*)k_tau_stream<1, 4, true, double>,  (const void*)k_tau_stream<1, 2, true, double>,
      (const void*)k_tau_stream<2, 4, false, float>,  (const void*)k_tau_stream<2, 2, false, float>,
      (const void*)k_tau_stream<1, 4, false, float>,  (const void*)k_tau_stream<1, 2, false, float>,
      (const void*)k_tau_stream<2, 4, true, float>,   (const void*)k_tau_stream<2, 2, true, float>,
      (const void*)k_tau_stream<1, 4, true, float>,   (const void*)k_tau_stream<1, 2, true, float>,
      (const void*)k_tau_stream_qs<2, false, double>, (const void*)k_tau_stream_qs<2, true, double>,
      (const void*)k_tau_stream_qs<1, false, double>, (const void*)k_tau_stream_qs<1, true, double>,
      (const void*)k_tau_stream_qs<2, false, float>,  (const void*)k_tau_stream_qs<2, true, float>,
      (const void*)k_tau_stream_qs<1, false, float>,  (const void*)k_tau_stream_qs<1, true, float>};
  for (const void* f : fns)
    BSE_HIP(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
  return BSE_OK;
}

int site_potential(const double* xyz, const double* depth, const double* width, int nsites,
                   const int grid[3], const double cell[3], double2* out, hipStream_t st) {
  const long nr = (long)grid[0] * grid[1] * grid[2];
  hipLaunchKernelGGL(k_site_potential, dim3(nblocks(nr)), dim3(TPB), 0, st, xyz, depth, width,
                     nsites, grid[0], grid[1], grid[2], cell[0], cell[1], cell[2],
                     cell[0] * cell[1] * cell[2], out);
  CHECK_LAUNCH();
  return BSE_OK;
}

int coulomb_kernel(const int grid[3], const double cell[3], double* out, hipStream_t st) {
  const long nr = (long)grid[0] * grid[1] * grid[2];
  hipLaunchKernelGGL(k_coulomb, dim3(nblocks(nr)), dim3(TPB), 0, st, grid[0], grid[1], grid[2],
                     cell[0], cell[1], cell[2], out);
  CHECK_LAUNCH();
  return BSE_OK;
}

int force_density(const double2* a, const double2* phit, const double2* z, const double2* phir,
                  int nv, long nr, double2* rho, hipStream_t st) {
  hipLaunchKernelGGL(k_force_density, dim3(nblocks(nr)), dim3(TPB), 0, st, a, phit, z, phir,
                     (nv + 1) / 2, nr, rho);
  CHECK_LAUNCH();
  return BSE_OK;
}

int occupied_density(const double2* phir, int nv, long nr, double2* rho, hipStream_t st) {
  hipLaunchKernelGGL(k_occupied_density, dim3(nblocks(nr)), dim3(TPB), 0, st, phir, (nv + 1) / 2,
                     nr, rho);
  CHECK_LAUNCH();
  return BSE_OK;
}

static long force_chunks(long nr) {
  long c = (nr + 4095) / 4096;
  if (c > 256) c = 256;
  if (c < 1) c = 1;
  return c;
}

long force_reduce_work(int nsites, long nr) { return (long)nsites * force_chunks(nr) * 3; }

int force_reduce(const double2* rhoG, const double* xyz, const double* depth, const double* width,
                 int nsites, const int grid[3], const double cell[3], double* part,
                 long part_len, double* out_dev, hipStream_t st) {
  if (nsites <= 0) return BSE_OK;
  const long nr = (long)grid[0] * grid[1] * grid[2];
  const long nch = force_chunks(nr);
  if (nsites * nch * 3 > part_len) return fail(BSE_EINVAL, "force_reduce: work too small");
  const long chunk = (nr + nch - 1) / nch;
  const double omega = cell[0] * cell[1] * cell[2];
  hipLaunchKernelGGL(k_force_partial, dim3((unsigned)nch, (unsigned)nsites), dim3(256), 0, st,
                     rhoG, xyz, depth, width, grid[0], grid[1], grid[2], cell[0], cell[1],
                     cell[2], omega, chunk, part);
  CHECK_LAUNCH();
  hipLaunchKernelGGL(k_force_final, dim3((unsigned)((nsites * 3 + 255) / 256)), dim3(256), 0, st,
                     part, nsites, (int)nch, omega / (double)nr, out_dev);
  CHECK_LAUNCH();
  return BSE_OK;
}

static int row_dots_split(long rows, long len) {
  // ~64k elements per block, at most 512 blocks per row and 64k blocks in all
  long ns = std::max(1L, std::min(512L, len / 65536));
  while (ns > 1 && rows * ns > 65536) ns /= 2;
  return (int)ns;
}

long row_dots_work(long rows, long len) { return rows * row_dots_split(rows, len); }

int row_dots(const double* A, const double* B, long rows, long len, double* out, double* work,
             long work_len, hipStream_t st) {
  if (rows <= 0) return BSE_OK;
  if (rows > 65535) return fail(BSE_EINVAL, "row_dots: too many rows");
  const int ns = row_dots_split(rows, len);
  if (work_len < rows * ns) return fail(BSE_EINVAL, "row_dots: work buffer too small");
  hipLaunchKernelGGL(k_row_dots, dim3((unsigned)ns, (unsigned)rows), dim3(256), 0, st, A, B, len,
                     ns, work);
  hipLaunchKernelGGL(k_row_dots_final, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, st, work,
                     rows, ns, out);
  CHECK_LAUNCH();
  return BSE_OK;
}

int row_axpby(const double* a, const double* X, const double* b, double* Y, long rows, long len,
              hipStream_t st) {
  const long n = rows * len;
  if (n <= 0) return BSE_OK;
  hipLaunchKernelGGL(k_row_axpby, dim3(nblocks(n)), dim3(TPB), 0, st, a, X, b, Y, rows, len);
  CHECK_LAUNCH();
  return BSE_OK;
}

int row_scale(const double* s, double* Y, long rows, long len, hipStream_t st) {
  const long n = rows * len;
  if (n <= 0) return BSE_OK;
  hipLaunchKernelGGL(k_row_scale, dim3(nblocks(n)), dim3(TPB), 0, st, s, Y, rows, len);
  CHECK_LAUNCH();
  return BSE_OK;
}

int diag_axpy(const double* A, const double* Tk, const double* eps, double shift, int nv,
              long npw, int nb, double* Y, hipStream_t st) {
  const long n = (long)nb * nv * npw;
  if (n <= 0) return BSE_OK;
  hipLaunchKernelGGL(k_diag_axpy, dim3(nblocks(n)), dim3(TPB), 0, st, A, Tk, eps, shift, nv, npw,
                     n, Y);
  CHECK_LAUNCH();
  return BSE_OK;
}

int zero_fill(double* p, long n, hipStream_t st) {
  if (n <= 0) return BSE_OK;
  hipLaunchKernelGGL(k_zero, dim3(nblocks(n)), dim3(TPB), 0, st, p, n);
  CHECK_LAUNCH();
  return BSE_OK;
}

int axpby(double alpha, const double* X, double beta, double* Y, long n, hipStream_t st) {
  if (n <= 0) return BSE_OK;
  hipLaunchKernelGGL(k_axpby, dim3(nblocks(n)), dim3(TPB), 0, st, alpha, X, beta, Y, n);
  CHECK_LAUNCH();
  return BSE_OK;
}

int precond_davidson(const double* R, double* T, const double* Tk, const double* eps,
                     const double* theta, double shift, int nk, int nv, int npw, hipStream_t st,
                     const double* vshift) {
  const long n = (long)nk * nv * npw;
  if (n <= 0) return BSE_OK;
  hipLaunchKernelGGL(k_precond_davidson, dim3(nblocks(n)), dim3(TPB), 0, st, R, T, Tk, eps, theta,
                     shift, nk, nv, npw, vshift);
  CHECK_LAUNCH();
  return BSE_OK;
}

int precond_cg(const double* R, double* T, const double* Tk, const double* eps, double shift,
               int nv, int npw, hipStream_t st, const double* vshift) {
  const long n = (long)nv * npw;
  if (n <= 0) return BSE_OK;
  hipLaunchKernelGGL(k_precond_cg, dim3(nblocks(n)), dim3(TPB), 0, st, R, T, Tk, eps, shift, nv,
                     npw, vshift);
  CHECK_LAUNCH();
  return BSE_OK;
}

int coarse_scale(double* C, int nk, int nv, int nc, const double* eps, const double* theta,
                 double shift, double dmin, hipStream_t st) {
  const long n = (long)nk * nv * nc;
  if (n <= 0) return BSE_OK;
  hipLaunchKernelGGL(k_coarse_scale, dim3(nblocks(n)), dim3(TPB), 0, st, C, nk, nv, nc, eps, theta,
                     shift, dmin);
  CHECK_LAUNCH();
  return BSE_OK;
}

int band_features(const double* Phi, const double* Tk, const double* eps, const double* U,
                  const double2* phir, double shift, int nv, int npw, long nr, double* out,
                  hipStream_t st) {
  if (nv <= 0) return BSE_OK;
  hipLaunchKernelGGL(k_band_features, dim3(nv), dim3(256), 0, st, Phi, Tk, eps, U, phir, shift, npw,
                     nr, out);
  CHECK_LAUNCH();
  return BSE_OK;
}

}  // namespace bsex
