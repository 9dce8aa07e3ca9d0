"""The batch runner's host side under the sanitizers, on the CPU.

The scheduler of the uneven batch (csrc/batch_sched.h) and the host eigensolver's
worker pool (csrc/linalg_host.cpp) are compiled with g++ into a driver (no GPU
and no HIP calls) and run with ThreadSanitizer and with AddressSanitizer.
The driver schedules 40 jobs of random size on 4 slot threads with a memory
budget; every job calls the threaded host eigensolver at the same time as
the others (the pool's concurrent-caller path) on its own matrix.  Checked:
every job runs exactly once, on a slot's own thread with the stack size the
scheduler asked for; the admission rule holds (the jobs running never exceed
the budget unless one runs alone); every eigen-decomposition is bitwise the
one a single caller gets.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2607_20728_amd", "csrc")

DRIVER = r"""
#include <pthread.h>

#include <atomic>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <random>
#include <vector>

#include "batch_sched.h"
namespace bsex {
int host_syev(int n, double* A, double* w);
}

static std::vector<double> sym(int n, unsigned seed) {
  std::mt19937_64 g(seed);
  std::normal_distribution<double> N(0.0, 1.0);
  std::vector<double> A((size_t)n * n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j <= i; ++j) A[(size_t)i * n + j] = A[(size_t)j * n + i] = N(g);
  return A;
}

int main() {
  const int n = 40, ns = 4, m = 96;
  const size_t stack = (size_t)64 << 20;
  std::mt19937 g(7);
  std::uniform_real_distribution<double> U(1.0, 10.0);
  std::vector<double> est(n);
  for (auto& e : est) e = U(g);
  est[3] = 25.0;  // larger than the budget: must still run, alone
  const double budget = 20.0;
  // single-caller reference decompositions
  std::vector<std::vector<double>> ref(n);
  for (int i = 0; i < n; ++i) {
    std::vector<double> A = sym(m, 100 + i), w(m);
    if (bsex::host_syev(m, A.data(), w.data())) return 10;
    A.insert(A.end(), w.begin(), w.end());
    ref[i] = A;
  }
  std::vector<std::atomic<int>> runs(n);
  for (auto& r : runs) r.store(0);
  std::mutex mu;
  double running_est = 0.0;
  int running = 0, bad_admit = 0, bad_stack = 0, bad_result = 0;
  std::vector<pthread_t> slot_thread(ns);
  bsex::BatchHooks h;
  h.slot_begin = [&](int s) {
    slot_thread[s] = pthread_self();
    pthread_attr_t a;
    size_t sz = 0;
    if (pthread_getattr_np(pthread_self(), &a) == 0) {
      pthread_attr_getstacksize(&a, &sz);
      pthread_attr_destroy(&a);
    }
    if (sz < stack) { std::lock_guard<std::mutex> lk(mu); ++bad_stack; }
  };
  h.run = [&](int s, int i) {
    {
      std::lock_guard<std::mutex> lk(mu);
      running_est += est[i];
      ++running;
      if (running > 1 && running_est > budget + 1e-9) ++bad_admit;
      if (!pthread_equal(slot_thread[s], pthread_self())) ++bad_stack;
    }
    runs[i].fetch_add(1);
    std::vector<double> A = sym(m, 100 + i), w(m);
    if (bsex::host_syev(m, A.data(), w.data())) { std::lock_guard<std::mutex> lk(mu); ++bad_result; }
    A.insert(A.end(), w.begin(), w.end());
    if (std::memcmp(A.data(), ref[i].data(), sizeof(double) * A.size()) != 0) {
      std::lock_guard<std::mutex> lk(mu);
      ++bad_result;
    }
    std::lock_guard<std::mutex> lk(mu);
    running_est -= est[i];
    --running;
  };
  if (bsex::schedule_batch(n, est, budget, ns, stack, h) != 0) return 11;
  int once = 0;
  for (auto& r : runs) once += r.load() == 1;
  std::printf("jobs run once %d/%d, admission violations %d, stack/thread errors %d, "
              "result mismatches %d\n", once, n, bad_admit, bad_stack, bad_result);
  return (once == n && !bad_admit && !bad_stack && !bad_result) ? 0 : 1;
}
"""


@pytest.mark.parametrize("san", ["thread", "address"])
def test_scheduler_and_host_pool_under_sanitizer(san, tmp_path):
    gxx = shutil.which("g++")
    if gxx is None or not os.path.isdir("/opt/rocm/include"):
        pytest.skip("g++ or the ROCm headers are missing")
    src = tmp_path / "driver.cpp"
    src.write_text(DRIVER)
    exe = tmp_path / "driver"
    cmd = [gxx, "-O1", "-g", "-std=c++17", "-pthread", f"-fsanitize={san}",
           "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-I", CSRC, str(src),
           os.path.join(CSRC, "linalg_host.cpp"), "-o", str(exe)]
    p = subprocess.run(cmd, capture_output=True, text=True)
    assert p.returncode == 0, p.stderr[-3000:]
    env = dict(os.environ, BSEX_HOST_THREADS="4",
               TSAN_OPTIONS="halt_on_error=1 second_deadlock_stack=1",
               ASAN_OPTIONS="detect_leaks=0 halt_on_error=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=600)
    print(r.stdout)
    assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
    assert "WARNING: ThreadSanitizer" not in r.stderr, r.stderr[-4000:]
