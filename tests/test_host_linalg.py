"""The library's host dense linear algebra (csrc/linalg_host.cpp): the
symmetric eigensolver behind every Rayleigh-Ritz and Gram step, and the
Cholesky factor and its inverse behind the ground state's Cholesky QR.

The source is compiled here with g++ into a small driver (no GPU needed) and
checked against numpy.linalg (LAPACK): eigenvalues, the eigen-residual
||A Q - Q diag(w)||, orthonormality, L L^T = A, L^{-1} L = I.  The worker
threads split rows, columns and column bands without changing any sum's
order, so every result must be bitwise the same for 1 and 4 threads.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2607_20728_amd", "csrc")

DRIVER = r"""
#include <cstdio>
#include <cstdlib>
#include <vector>
namespace bsex {
int host_syev(int n, double* A, double* w);
int host_cholesky(int n, double* A);
int host_trinv_lower(int n, double* L);
}
// usage: driver mode n in out ; mode 0 syev, 1 cholesky, 2 trinv
int main(int argc, char** argv) {
  const int mode = atoi(argv[1]), n = atoi(argv[2]);
  std::vector<double> A((size_t)n * n), w(n);
  FILE* f = fopen(argv[3], "rb");
  if (!f || fread(A.data(), sizeof(double), A.size(), f) != A.size()) return 3;
  fclose(f);
  int rc = mode == 0 ? bsex::host_syev(n, A.data(), w.data())
         : mode == 1 ? bsex::host_cholesky(n, A.data()) : bsex::host_trinv_lower(n, A.data());
  FILE* g = fopen(argv[4], "wb");
  fwrite(&rc, sizeof(int), 1, g);
  fwrite(A.data(), sizeof(double), A.size(), g);
  fwrite(w.data(), sizeof(double), w.size(), g);
  fclose(g);
  return 0;
}
"""


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None or not os.path.isdir("/opt/rocm/include"):
        pytest.skip("g++ or the ROCm headers are missing")
    d = tmp_path_factory.mktemp("linalg")
    src = d / "driver.cpp"
    src.write_text(DRIVER)
    exe = d / "driver"
    cmd = [gxx, "-O2", "-std=c++17", "-pthread", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           "-I", CSRC, str(src), os.path.join(CSRC, "linalg_host.cpp"), "-o", str(exe)]
    p = subprocess.run(cmd, capture_output=True, text=True)
    if p.returncode != 0:
        pytest.fail("g++ failed:\n" + p.stderr[-2000:])
    return d, exe


def _run(driver, mode, A, threads):
    d, exe = driver
    n = A.shape[0]
    fin, fout = d / f"in_{mode}_{n}", d / f"out_{mode}_{n}_{threads}"
    np.ascontiguousarray(A, dtype=np.float64).tofile(fin)
    env = dict(os.environ, BSEX_HOST_THREADS=str(threads))
    p = subprocess.run([str(exe), str(mode), str(n), str(fin), str(fout)], env=env,
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 0, p.stderr
    raw = np.fromfile(fout, dtype=np.uint8)
    rc = int(np.frombuffer(raw[:4].tobytes(), dtype=np.int32)[0])
    vals = np.frombuffer(raw[4:].tobytes(), dtype=np.float64)
    return rc, vals[:n * n].reshape(n, n), vals[n * n:]


def _matrices():
    rng = np.random.default_rng(77)
    out = {}
    for n in (1, 2, 7, 64, 300):
        B = rng.standard_normal((n, n))
        out[f"random{n}"] = B + B.T
    out["repeated"] = np.diag(np.repeat(np.arange(6.0), 25))  # 150, six 25-fold values
    v = rng.standard_normal(120)
    out["rank_one"] = np.outer(v, v)
    Q, _ = np.linalg.qr(rng.standard_normal((200, 200)))
    w = np.concatenate([np.full(100, 1.0), 1.0 + 1e-9 * np.arange(50), np.linspace(3, 9, 50)])
    out["clustered"] = (Q * w) @ Q.T
    return out


@pytest.mark.parametrize("name", list(_matrices()))
def test_syev_against_lapack(driver, name):
    A = _matrices()[name]
    n = A.shape[0]
    rc, Q, w = _run(driver, 0, A, 4)
    assert rc == 0
    scale = max(np.abs(A).max(), 1.0)
    wl = np.linalg.eigvalsh(A)
    assert np.all(np.diff(w) >= 0)
    assert np.abs(w - wl).max() <= 1e-12 * scale * max(n, 1) ** 0.5
    assert np.abs(A @ Q - Q * w).max() <= 1e-12 * scale * n
    assert np.abs(Q.T @ Q - np.eye(n)).max() <= 1e-13 * n
    rc1, Q1, w1 = _run(driver, 0, A, 1)
    assert rc1 == 0 and np.array_equal(Q1, Q) and np.array_equal(w1, w)


@pytest.mark.parametrize("n", [1, 5, 64, 257])
def test_cholesky_and_inverse(driver, n):
    rng = np.random.default_rng(n)
    B = rng.standard_normal((n, n))
    A = B @ B.T + n * np.eye(n)
    rc, L, _ = _run(driver, 1, A, 4)
    assert rc == 0
    assert np.array_equal(np.triu(L, 1), np.zeros_like(L))
    assert np.abs(L - np.linalg.cholesky(A)).max() <= 1e-12 * np.abs(L).max()
    assert np.array_equal(_run(driver, 1, A, 1)[1], L)
    rc, M, _ = _run(driver, 2, L, 4)
    assert rc == 0
    assert np.abs(M @ L - np.eye(n)).max() <= 1e-13 * n
    assert np.array_equal(_run(driver, 2, L, 1)[1], M)


def test_cholesky_rejects_indefinite(driver):
    A = np.diag([1.0, 2.0, -1.0, 4.0])
    rc, _, _ = _run(driver, 1, A, 1)
    assert rc != 0
    rc, _, _ = _run(driver, 2, np.diag([1.0, 0.0, 2.0]), 1)
    assert rc != 0
