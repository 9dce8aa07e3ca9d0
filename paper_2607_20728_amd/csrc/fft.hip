// Batched in-place 3-D complex FFT (FP64) for gfx950.
//
// One kernel launch per axis.  A workgroup stages L lines of the axis in LDS,
// runs a mixed-radix (2, 3, 4, 5) Stockham transform there (autosort, no
// bit reversal; each pass reads one LDS buffer and writes the other), and
// writes the lines back.  Lines along the two strided axes are taken as L
// neighbours along the contiguous axis, so every global access touches L
// consecutive complex values.  Twiddles come from a per-axis table
// exp(-2 pi i k/n) computed on the host in long double.
#include <cmath>
#include <cstring>

#include "common.h"

namespace bsex {

namespace {

constexpr int kThreads = 256;
constexpr int kMaxN = 512;

struct AxisArgs {
  int n;
  int nrad;
  int rad[8];
  const double2* tw;
};

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) {
  return make_double2(a.x + b.x, a.y + b.y);
}
__device__ __forceinline__ double2 csub(double2 a, double2 b) {
  return make_double2(a.x - b.x, a.y - b.y);
}
// multiply by -i (dir = -1) or +i (dir = +1)
template <int DIR>
__device__ __forceinline__ double2 mul_i(double2 a) {
  return DIR < 0 ? make_double2(a.y, -a.x) : make_double2(-a.y, a.x);
}

// In-register DFT of length R: v[m] <- sum_r v[r] exp(DIR 2 pi i r m / R).
template <int DIR>
__device__ __forceinline__ void dft2(double2* v) {
  const double2 a = v[0], b = v[1];
  v[0] = cadd(a, b);
  v[1] = csub(a, b);
}
template <int DIR>
__device__ __forceinline__ void dft3(double2* v) {
  const double s3 = 0.86602540378443864676;  // sin(2 pi/3)
  const double2 t1 = cadd(v[1], v[2]);
  const double2 t2 = make_double2(v[0].x - 0.5 * t1.x, v[0].y - 0.5 * t1.y);
  const double2 d = csub(v[1], v[2]);
  const double2 t3 = mul_i<DIR>(make_double2(s3 * d.x, s3 * d.y));
  v[0] = cadd(v[0], t1);
  v[1] = cadd(t2, t3);
  v[2] = csub(t2, t3);
}
template <int DIR>
__device__ __forceinline__ void dft4(double2* v) {
  const double2 a = cadd(v[0], v[2]), b = csub(v[0], v[2]);
  const double2 c = cadd(v[1], v[3]), d = mul_i<DIR>(csub(v[1], v[3]));
  v[0] = cadd(a, c);
  v[2] = csub(a, c);
  v[1] = cadd(b, d);
  v[3] = csub(b, d);
}
template <int DIR>
__device__ __forceinline__ void dft5(double2* v) {
  // cos/sin of 2 pi/5 and 4 pi/5 from their closed forms
  const double c1 = 0.30901699437494742410, c2 = -0.80901699437494742410;
  const double s1 = 0.95105651629515357212, s2 = 0.58778525229247312917;
  const double2 t1 = cadd(v[1], v[4]), t2 = cadd(v[2], v[3]);
  const double2 t3 = csub(v[1], v[4]), t4 = csub(v[2], v[3]);
  const double2 a1 = make_double2(v[0].x + c1 * t1.x + c2 * t2.x, v[0].y + c1 * t1.y + c2 * t2.y);
  const double2 a2 = make_double2(v[0].x + c2 * t1.x + c1 * t2.x, v[0].y + c2 * t1.y + c1 * t2.y);
  const double2 b1 = mul_i<DIR>(make_double2(s1 * t3.x + s2 * t4.x, s1 * t3.y + s2 * t4.y));
  const double2 b2 = mul_i<DIR>(make_double2(s2 * t3.x - s1 * t4.x, s2 * t3.y - s1 * t4.y));
  v[0] = cadd(v[0], cadd(t1, t2));
  v[1] = cadd(a1, b1);
  v[4] = csub(a1, b1);
  v[2] = cadd(a2, b2);
  v[3] = csub(a2, b2);
}

// One Stockham pass of radix R over L lines held as buf[k * L + l].
template <int R, int DIR>
__device__ void stockham_pass(const double2* __restrict__ in, double2* __restrict__ out, int n,
                              int L, int ns, const double2* __restrict__ tw) {
  const int nq = n / R;
  const int tstride = n / (ns * R);
  for (int u = threadIdx.x; u < nq * L; u += kThreads) {
    const int l = u % L;
    const int j = u / L;
    const int k = j % ns;
    double2 v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      double2 x = in[(j + r * nq) * L + l];
      if (r > 0 && k > 0) {
        double2 w = tw[k * r * tstride];
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
    for (int r = 0; r < R; ++r) out[(base + r * ns) * L + l] = v[r];
  }
}

// Lines: base = o1 * s_o1 + o2 * s_o2 + inner * s_in, elements at base + k * es.
// A workgroup takes L consecutive inner lines of one (o1, o2).
template <int DIR>
__global__ __launch_bounds__(kThreads) void k_fft_axis(double2* __restrict__ data, AxisArgs ax,
                                                       int es, int n_inner, long s_in, int n_o2,
                                                       long s_o2, long s_o1, int L) {
  extern __shared__ double2 lds[];
  const int n = ax.n;
  double2* b0 = lds;
  double2* b1 = lds + (long)n * L;
  const int tiles = (n_inner + L - 1) / L;
  long w = blockIdx.x;
  const int tile = (int)(w % tiles);
  w /= tiles;
  const int o2 = (int)(w % n_o2);
  const long o1 = w / n_o2;
  const int i0 = tile * L;
  const int nl = min(L, n_inner - i0);
  double2* base = data + o1 * s_o1 + (long)o2 * s_o2 + (long)i0 * s_in;
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
    double2 x = make_double2(0.0, 0.0);
    if (l < nl) x = base[(long)l * s_in + (long)k * es];
    b0[k * L + l] = x;
  }
  __syncthreads();
  int ns = 1;
  double2* src = b0;
  double2* dst = b1;
  for (int p = 0; p < ax.nrad; ++p) {
    const int R = ax.rad[p];
    if (R == 4)
      stockham_pass<4, DIR>(src, dst, n, L, ns, ax.tw);
    else if (R == 2)
      stockham_pass<2, DIR>(src, dst, n, L, ns, ax.tw);
    else if (R == 3)
      stockham_pass<3, DIR>(src, dst, n, L, ns, ax.tw);
    else
      stockham_pass<5, DIR>(src, dst, n, L, ns, ax.tw);
    ns *= R;
    __syncthreads();
    double2* t = src;
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
    if (l < nl) base[(long)l * s_in + (long)k * es] = src[k * L + l];
  }
}

int lines_per_group(int n) {
  // about 16 KB of LDS per buffer; at least 4 lines
  int L = 16384 / (16 * n);
  if (L < 4) L = 4;
  if (L > 32) L = 32;
  return L;
}

}  // namespace

int fft_plan_init(FftPlan* p, const int grid[3]) {
  p->nr = 1;
  for (int a = 0; a < 3; ++a) {
    const int n = grid[a];
    if (n < 2 || n > kMaxN) return fail(BSE_EINVAL, "FFT length %d unsupported", n);
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
    for (int k = 0; k < n; ++k) {
      const long double ang = -2.0L * 3.141592653589793238462643383279502884L * k / n;
      tw[k] = make_double2((double)cosl(ang), (double)sinl(ang));
    }
    BSE_HIP(hipMalloc(&ax.tw, sizeof(double2) * n));
    BSE_HIP(hipMemcpy(ax.tw, tw.data(), sizeof(double2) * n, hipMemcpyHostToDevice));
    p->N[a] = n;
    p->nr *= n;
  }
  return BSE_OK;
}

void fft_plan_free(FftPlan* p) {
  for (int a = 0; a < 3; ++a) {
    if (p->ax[a].tw) (void)hipFree(p->ax[a].tw);
    p->ax[a].tw = nullptr;
  }
}

static int launch_axis(const FftAxis& a, double2* data, int dir, int es, int n_inner, long s_in,
                       int n_o2, long s_o2, long n_o1, long s_o1, hipStream_t st) {
  AxisArgs ax;
  ax.n = a.n;
  ax.nrad = a.nrad;
  for (int i = 0; i < 8; ++i) ax.rad[i] = a.rad[i];
  ax.tw = a.tw;
  const int L = lines_per_group(a.n);
  const long tiles = (n_inner + L - 1) / L;
  const long groups = tiles * n_o2 * n_o1;
  if (groups <= 0) return BSE_OK;
  if (groups > 0x7fffffffL) return fail(BSE_EINVAL, "FFT batch too large");
  const size_t shm = 2 * sizeof(double2) * a.n * L;
  if (dir < 0)
    hipLaunchKernelGGL(k_fft_axis<-1>, dim3((unsigned)groups), dim3(kThreads), shm, st, data, ax,
                       es, n_inner, s_in, n_o2, s_o2, s_o1, L);
  else
    hipLaunchKernelGGL(k_fft_axis<1>, dim3((unsigned)groups), dim3(kThreads), shm, st, data, ax,
                       es, n_inner, s_in, n_o2, s_o2, s_o1, L);
  BSE_HIP(hipGetLastError());
  return BSE_OK;
}

int fft3d(const FftPlan& p, double2* data, long batch, int dir, hipStream_t st) {
  if (batch <= 0) return BSE_OK;
  const int N1 = p.N[0], N2 = p.N[1], N3 = p.N[2];
  const long nr = p.nr;
  // axis 3 (contiguous lines): lines (b, i1, i2); inner = i2 with stride N3
  BSE_TRY(launch_axis(p.ax[2], data, dir, 1, N2, N3, N1, (long)N2 * N3, batch, nr, st));
  // axis 2: lines (b, i1, i3); inner = i3 (stride 1), elements stride N3
  BSE_TRY(launch_axis(p.ax[1], data, dir, N3, N3, 1, N1, (long)N2 * N3, batch, nr, st));
  // axis 1: lines (b, i2, i3); inner = i3, elements stride N2*N3
  BSE_TRY(launch_axis(p.ax[0], data, dir, N2 * N3, N3, 1, N2, N3, batch, nr, st));
  return BSE_OK;
}

}  // namespace bsex
