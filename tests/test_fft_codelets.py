"""The in-register DFT butterflies of the HIP FFT, compiled for the host.

The butterflies (lengths 2, 3, 4, 5, 8, 9) are plain arithmetic on a
complex type, so the same header that the gfx950 kernels include builds with
g++ when the HIP qualifiers are defined away.  Each is checked against
numpy's FFT on seeded inputs, in both directions and in FP64 and FP32:
v[m] <- sum_r v[r] exp(DIR 2 pi i r m / R), so DIR = -1 is numpy's forward
transform and DIR = +1 is R times its inverse.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

HDR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "paper_2607_20728_amd", "csrc")
LENGTHS = (2, 3, 4, 5, 8, 9)
NTRIAL = 20

SRC = r"""
#include <cstdio>
#include <cstdlib>
#define __device__
#define __forceinline__ inline
namespace host {
typedef REAL real;
struct cplx { real x, y; };
inline cplx mk(real a, real b) { return cplx{a, b}; }
#include "fft_codelets.h"
}
using namespace host;
template <int DIR, int R> void run(const double* in, int ntrial) {
  for (int t = 0; t < ntrial; ++t) {
    cplx v[R];
    for (int r = 0; r < R; ++r) v[r] = mk((real)in[2 * (t * 9 + r)], (real)in[2 * (t * 9 + r) + 1]);
    if (R == 2) dft2<DIR>(v);
    if (R == 3) dft3<DIR>(v);
    if (R == 4) dft4<DIR>(v);
    if (R == 5) dft5<DIR>(v);
    if (R == 8) dft8<DIR>(v);
    if (R == 9) dft9<DIR>(v);
    for (int m = 0; m < R; ++m) printf("%.17g %.17g\n", (double)v[m].x, (double)v[m].y);
  }
}
template <int DIR> void all(const double* in, int ntrial) {
  run<DIR, 2>(in, ntrial); run<DIR, 3>(in, ntrial); run<DIR, 4>(in, ntrial);
  run<DIR, 5>(in, ntrial); run<DIR, 8>(in, ntrial); run<DIR, 9>(in, ntrial);
}
int main(int argc, char** argv) {
  const int ntrial = atoi(argv[1]);
  const int n = 2 * 9 * ntrial;
  double* in = (double*)malloc(sizeof(double) * n);
  for (int i = 0; i < n; ++i)
    if (scanf("%lf", &in[i]) != 1) return 1;
  all<-1>(in, ntrial);
  all<1>(in, ntrial);
  free(in);
  return 0;
}
"""


@pytest.fixture(scope="module")
def inputs():
    rng = np.random.default_rng(20260728)
    return rng.standard_normal((NTRIAL, 9)) + 1j * rng.standard_normal((NTRIAL, 9))


@pytest.mark.parametrize("real,tol", [("double", 1e-14), ("float", 3e-6)])
def test_butterflies_match_numpy_fft(tmp_path, inputs, real, tol):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not found")
    src = tmp_path / "codelets.cpp"
    src.write_text(SRC)
    exe = tmp_path / "codelets"
    subprocess.run([gxx, "-O1", "-std=c++17", f"-DREAL={real}", f"-I{HDR}", str(src), "-o",
                    str(exe)], check=True, capture_output=True, text=True)
    flat = np.stack([inputs.real, inputs.imag], axis=-1).reshape(-1)
    out = subprocess.run([str(exe), str(NTRIAL)], input="\n".join(f"{x:.17g}" for x in flat),
                         check=True, capture_output=True, text=True).stdout.split()
    vals = np.array(out, dtype=float).reshape(-1, 2)
    got = vals[:, 0] + 1j * vals[:, 1]
    pos = 0
    for d in (-1, 1):
        for R in LENGTHS:
            x = inputs[:, :R]
            ref = np.fft.fft(x, axis=1) if d < 0 else R * np.fft.ifft(x, axis=1)
            g = got[pos:pos + NTRIAL * R].reshape(NTRIAL, R)
            pos += NTRIAL * R
            err = np.abs(g - ref).max() / np.abs(ref).max()
            assert err < tol, (real, d, R, err)
    assert pos == got.size
