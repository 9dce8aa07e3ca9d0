// In-register complex arithmetic and DFT butterflies of the FFT.  Included
// inside a namespace that defines `real`, `cplx` (with members x, y) and
// `mk(re, im)`, once per precision (no include guard).  Plain C++ with
// __device__ and __forceinline__ defined away compiles it for the host too.

__device__ __forceinline__ cplx cmul(cplx a, cplx b) {
  return mk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ cplx cadd(cplx a, cplx b) {
  return mk(a.x + b.x, a.y + b.y);
}
__device__ __forceinline__ cplx csub(cplx a, cplx b) {
  return mk(a.x - b.x, a.y - b.y);
}
// multiply by -i (dir = -1) or +i (dir = +1)
template <int DIR>
__device__ __forceinline__ cplx mul_i(cplx a) {
  return DIR < 0 ? mk(a.y, -a.x) : mk(-a.y, a.x);
}

// In-register DFT of length R: v[m] <- sum_r v[r] exp(DIR 2 pi i r m / R).
template <int DIR>
__device__ __forceinline__ void dft2(cplx* v) {
  const cplx a = v[0], b = v[1];
  v[0] = cadd(a, b);
  v[1] = csub(a, b);
}
template <int DIR>
__device__ __forceinline__ void dft3(cplx* v) {
  const real s3 = (real)0.86602540378443864676;  // sin(2 pi/3)
  const cplx t1 = cadd(v[1], v[2]);
  const cplx t2 = mk(v[0].x - (real)0.5 * t1.x, v[0].y - (real)0.5 * t1.y);
  const cplx d = csub(v[1], v[2]);
  const cplx t3 = mul_i<DIR>(mk(s3 * d.x, s3 * d.y));
  v[0] = cadd(v[0], t1);
  v[1] = cadd(t2, t3);
  v[2] = csub(t2, t3);
}
template <int DIR>
__device__ __forceinline__ void dft4(cplx* v) {
  const cplx a = cadd(v[0], v[2]), b = csub(v[0], v[2]);
  const cplx c = cadd(v[1], v[3]), d = mul_i<DIR>(csub(v[1], v[3]));
  v[0] = cadd(a, c);
  v[2] = csub(a, c);
  v[1] = cadd(b, d);
  v[3] = csub(b, d);
}
template <int DIR>
__device__ __forceinline__ void dft5(cplx* v) {
  // cos/sin of 2 pi/5 and 4 pi/5 from their closed forms
  const real c1 = (real)0.30901699437494742410, c2 = (real)-0.80901699437494742410;
  const real s1 = (real)0.95105651629515357212, s2 = (real)0.58778525229247312917;
  const cplx t1 = cadd(v[1], v[4]), t2 = cadd(v[2], v[3]);
  const cplx t3 = csub(v[1], v[4]), t4 = csub(v[2], v[3]);
  const cplx a1 = mk(v[0].x + c1 * t1.x + c2 * t2.x, v[0].y + c1 * t1.y + c2 * t2.y);
  const cplx a2 = mk(v[0].x + c2 * t1.x + c1 * t2.x, v[0].y + c2 * t1.y + c1 * t2.y);
  const cplx b1 = mul_i<DIR>(mk(s1 * t3.x + s2 * t4.x, s1 * t3.y + s2 * t4.y));
  const cplx b2 = mul_i<DIR>(mk(s2 * t3.x - s1 * t4.x, s2 * t3.y - s1 * t4.y));
  v[0] = cadd(v[0], cadd(t1, t2));
  v[1] = cadd(a1, b1);
  v[4] = csub(a1, b1);
  v[2] = cadd(a2, b2);
  v[3] = csub(a2, b2);
}

// v times exp(DIR i theta), given cos(theta) = c and sin(theta) = s
template <int DIR>
__device__ __forceinline__ cplx rot(cplx v, real c, real s) {
  const real ds = DIR > 0 ? s : -s;
  return mk(c * v.x - ds * v.y, c * v.y + ds * v.x);
}
// Length 8 as 2 x 4: with r = 4a + b and m = c + 2d the kernel
// exp(DIR 2 pi i r m / 8) splits into a length-2 DFT over a, the twiddle
// exp(DIR 2 pi i b c / 8), and a length-4 DFT over b.
template <int DIR>
__device__ __forceinline__ void dft8(cplx* v) {
  const real h = (real)0.70710678118654752440;  // cos(pi/4) = sin(pi/4)
  cplx y0[4], y1[4];
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    y0[b] = cadd(v[b], v[b + 4]);
    y1[b] = csub(v[b], v[b + 4]);
  }
  y1[1] = rot<DIR>(y1[1], h, h);
  y1[2] = mul_i<DIR>(y1[2]);
  y1[3] = rot<DIR>(y1[3], -h, h);
  dft4<DIR>(y0);
  dft4<DIR>(y1);
#pragma unroll
  for (int d = 0; d < 4; ++d) {
    v[2 * d] = y0[d];
    v[2 * d + 1] = y1[d];
  }
}
// Length 9 as 3 x 3: with r = 3a + b and m = c + 3d, a length-3 DFT over a,
// the twiddle exp(DIR 2 pi i b c / 9), and a length-3 DFT over b.
template <int DIR>
__device__ __forceinline__ void dft9(cplx* v) {
  const real c1 = (real)0.76604444311897803520, s1 = (real)0.64278760968653932632;   // 2 pi/9
  const real c2 = (real)0.17364817766693034885, s2 = (real)0.98480775301220805937;   // 4 pi/9
  const real c4 = (real)-0.93969262078590838405, s4 = (real)0.34202014332566873304;  // 8 pi/9
  cplx y[3][3];
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    y[b][0] = v[b];
    y[b][1] = v[b + 3];
    y[b][2] = v[b + 6];
    dft3<DIR>(y[b]);
  }
  y[1][1] = rot<DIR>(y[1][1], c1, s1);
  y[1][2] = rot<DIR>(y[1][2], c2, s2);
  y[2][1] = rot<DIR>(y[2][1], c2, s2);
  y[2][2] = rot<DIR>(y[2][2], c4, s4);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    cplx t[3] = {y[0][c], y[1][c], y[2][c]};
    dft3<DIR>(t);
    v[c] = t[0];
    v[c + 3] = t[1];
    v[c + 6] = t[2];
  }
}
