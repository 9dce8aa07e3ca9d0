// Small dense symmetric eigensolver and Cholesky on the host (FP64).
//
// Eigensolver: Householder reduction to tridiagonal form T = Q^T A Q, then
// implicit symmetric QR steps with the Wilkinson shift, chasing the bulge
// with plane rotations and deflating negligible off-diagonal entries (the
// method of Golub and Van Loan, "Matrix Computations", Sec. 8.3).  Used for
// the Rayleigh-Ritz and Gram problems of the Davidson and ground-state
// subspace solvers (n up to several hundred).
//
// The O(n^3) parts run on a small pool of host threads: the matrix-vector
// product and rank-2 update of each reduction step (split by rows), the
// product of the reflectors that forms Q^T (split by rows of Q^T), and the
// plane rotations, which are recorded while the QR steps run on the
// tridiagonal matrix alone and applied afterwards (split by columns).
#include <sched.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <condition_variable>
#include <cstdint>
#include <cstdlib>
#include <functional>
#include <mutex>
#include <thread>
#include <vector>

#include "common.h"

namespace bsex {

namespace {

// Host worker threads.  The caller takes part as worker 0; idle workers spin
// for a short while, then sleep on a condition variable.  A call made while
// another thread holds the pool runs its parts one after another instead.
class Workers {
 public:
  static Workers& get() {
    static Workers* w = new Workers(count());  // kept until the process ends
    return *w;
  }
  int size() const { return n_; }
  void run(const std::function<void(int, int)>& fn) {
    std::unique_lock<std::mutex> own(run_mx_, std::try_to_lock);
    if (n_ == 1 || !own.owns_lock()) {
      for (int t = 0; t < n_; ++t) fn(t, n_);
      return;
    }
    job_ = &fn;
    left_.store(n_ - 1, std::memory_order_relaxed);
    {
      std::lock_guard<std::mutex> g(mx_);
      gen_.fetch_add(1, std::memory_order_release);
    }
    cv_.notify_all();
    fn(0, n_);
    while (left_.load(std::memory_order_acquire) != 0) relax();
  }

 private:
  explicit Workers(int n) : n_(n) {
    for (int t = 1; t < n_; ++t) std::thread([this, t] { loop(t); }).detach();
  }
  // threads: BSEX_HOST_THREADS, else the CPUs this process may run on, at most 16
  static int count() {
    int n = 1;
    if (const char* s = std::getenv("BSEX_HOST_THREADS")) {
      n = std::atoi(s);
    } else {
      cpu_set_t set;
      CPU_ZERO(&set);
      n = sched_getaffinity(0, sizeof(set), &set) == 0 ? CPU_COUNT(&set)
                                                        : (int)std::thread::hardware_concurrency();
      n = std::min(n, 16);
    }
    return std::max(1, std::min(n, 64));
  }
  static void relax() { __builtin_ia32_pause(); }
  void loop(int t) {
    unsigned seen = 0;
    for (;;) {
      unsigned g;
      int spins = 0;
      while ((g = gen_.load(std::memory_order_acquire)) == seen) {
        if (++spins < (1 << 14)) {
          relax();
          continue;
        }
        std::unique_lock<std::mutex> lk(mx_);
        cv_.wait(lk, [&] { return gen_.load(std::memory_order_acquire) != seen; });
      }
      seen = g;
      (*job_)(t, n_);
      left_.fetch_sub(1, std::memory_order_acq_rel);
    }
  }
  const int n_;
  std::mutex run_mx_, mx_;
  std::condition_variable cv_;
  std::atomic<unsigned> gen_{0};
  std::atomic<int> left_{0};
  const std::function<void(int, int)>* job_ = nullptr;
};

// fn(lo, hi) over [0, m) in contiguous parts; one part when the work is small
template <class F>
void split_range(int m, double flops, F&& fn) {
  Workers& w = Workers::get();
  if (w.size() == 1 || flops < 4.0e4) {
    fn(0, m);
    return;
  }
  w.run([&](int t, int nt) {
    const int lo = (int)((long)m * t / nt), hi = (int)((long)m * (t + 1) / nt);
    if (hi > lo) fn(lo, hi);
  });
}

struct Rot {
  int k;
  double c, s;
};

// A <- Q^T A Q tridiagonal.  Reflector k, I - beta_k v_k v_k^T acting on
// indices k+1..n-1, is kept in row k of V (columns k+1..n-1).
void householder_tridiag(int n, std::vector<double>& A, std::vector<double>& V,
                         std::vector<double>& beta, std::vector<double>& d,
                         std::vector<double>& e) {
  auto a = [&](int i, int j) -> double& { return A[(size_t)i * n + j]; };
  std::vector<double> p(n), w(n);
  for (int k = 0; k + 2 < n; ++k) {
    const int m = n - k - 1;  // length of the column below the diagonal
    double* v = &V[(size_t)k * n + k + 1];
    double nrm2 = 0.0;
    for (int i = 0; i < m; ++i) {
      v[i] = a(k + 1 + i, k);
      nrm2 += v[i] * v[i];
    }
    const double tail = nrm2 - v[0] * v[0];
    beta[k] = 0.0;
    if (tail <= 0.0) continue;  // already tridiagonal in this column
    const double nrm = std::sqrt(nrm2);
    const double alpha = v[0] > 0 ? -nrm : nrm;
    v[0] -= alpha;
    const double bk = 2.0 / (v[0] * v[0] + tail);
    beta[k] = bk;
    // p = beta B v, B the trailing block
    split_range(m, 2.0 * m * m, [&](int lo, int hi) {
      for (int i = lo; i < hi; ++i) {
        const double* row = &a(k + 1 + i, k + 1);
        double s0 = 0.0, s1 = 0.0;
        int j = 0;
        for (; j + 1 < m; j += 2) {
          s0 += row[j] * v[j];
          s1 += row[j + 1] * v[j + 1];
        }
        if (j < m) s0 += row[j] * v[j];
        p[i] = bk * (s0 + s1);
      }
    });
    double pv = 0.0;
    for (int i = 0; i < m; ++i) pv += p[i] * v[i];
    const double K = 0.5 * bk * pv;
    for (int i = 0; i < m; ++i) w[i] = p[i] - K * v[i];
    // B <- B - v w^T - w v^T
    split_range(m, 4.0 * m * m, [&](int lo, int hi) {
      for (int i = lo; i < hi; ++i) {
        double* row = &a(k + 1 + i, k + 1);
        const double vi = v[i], wi = w[i];
        for (int j = 0; j < m; ++j) row[j] -= vi * w[j] + wi * v[j];
      }
    });
    a(k + 1, k) = a(k, k + 1) = alpha;
    for (int i = 1; i < m; ++i) a(k + 1 + i, k) = a(k, k + 1 + i) = 0.0;
  }
  for (int i = 0; i < n; ++i) d[i] = a(i, i);
  for (int i = 0; i + 1 < n; ++i) e[i] = a(i + 1, i);
  e[n - 1] = 0.0;
}

// Q^T with Q = H_0 H_1 ... H_{n-3}: row j of Q^T is Q e_j, the reflectors
// applied to e_j from the last to the first (H_k leaves e_j alone for k >= j).
// Qt rows are ld apart.
void form_qt(int n, const std::vector<double>& V, const std::vector<double>& beta, double* Qt,
             int ld) {
  std::fill(Qt, Qt + (size_t)n * ld, 0.0);
  auto body = [&](int j) {
    double* x = Qt + (size_t)j * ld;
    x[j] = 1.0;
    for (int k = std::min(j - 1, n - 3); k >= 0; --k) {
      if (beta[k] == 0.0) continue;
      const double* v = &V[(size_t)k * n + k + 1];
      double* y = x + k + 1;
      const int m = n - k - 1;
      double s = 0.0;
      for (int i = 0; i < m; ++i) s += v[i] * y[i];
      s *= beta[k];
      for (int i = 0; i < m; ++i) y[i] -= s * v[i];
    }
  };
  Workers& w = Workers::get();
  if (w.size() == 1 || n < 64) {
    for (int j = 0; j < n; ++j) body(j);
    return;
  }
  // row j costs about j (2n - j) flops: deal rows out in turn
  w.run([&](int t, int nt) {
    for (int j = t; j < n; j += nt) body(j);
  });
}

// apply recorded plane rotations to the rows of Qt (rows ld apart).  Each
// worker copies its own band of columns into a private dense block, rotates
// it there and copies it back: with the bands left in place, the prefetchers
// of one core keep pulling lines that another core is writing.
void apply_rotations(int n, const std::vector<Rot>& rots, double* Qt, int ld) {
  if (rots.empty()) return;
  const int lines = (n + 7) / 8;
  split_range(lines, 6.0 * (double)rots.size() * n, [&](int l0, int l1) {
    const int c0 = 8 * l0, bw = std::min(n, 8 * l1) - c0;
    std::vector<double> band((size_t)n * bw);
    for (int r = 0; r < n; ++r)
      std::copy(Qt + (size_t)r * ld + c0, Qt + (size_t)r * ld + c0 + bw, &band[(size_t)r * bw]);
    for (const Rot& r : rots) {
      double* rk = &band[(size_t)r.k * bw];
      double* r1 = rk + bw;
      const double cs = r.c, sn = r.s;
      for (int i = 0; i < bw; ++i) {
        const double qk = rk[i], q1 = r1[i];
        rk[i] = cs * qk + sn * q1;
        r1[i] = -sn * qk + cs * q1;
      }
    }
    for (int r = 0; r < n; ++r)
      std::copy(&band[(size_t)r * bw], &band[(size_t)r * bw] + bw, Qt + (size_t)r * ld + c0);
  });
}

// One implicit Wilkinson-shifted QR step on the unreduced block [lo, hi] of
// the tridiagonal (d, e); the rotations are appended to rots.
void qr_step(int lo, int hi, std::vector<double>& d, std::vector<double>& e,
             std::vector<Rot>& rots) {
  const double a = d[hi - 1], b = e[hi - 1], c = d[hi];
  const double delta = 0.5 * (a - c);
  const double rad = std::hypot(delta, b);
  const double mu = c - b * b / (delta + (delta >= 0 ? rad : -rad));
  double x = d[lo] - mu, z = e[lo];
  for (int k = lo; k < hi; ++k) {
    double r = std::sqrt(x * x + z * z);
    if (!(r > 1e-150 && r < 1e150)) r = std::hypot(x, z);  // squares out of range
    double cs = 1.0, sn = 0.0;
    if (r > 0.0) {
      cs = x / r;
      sn = z / r;
    }
    if (k > lo) e[k - 1] = r;
    const double akk = d[k], ak1 = e[k], a11 = d[k + 1];
    d[k] = cs * cs * akk + 2 * cs * sn * ak1 + sn * sn * a11;
    d[k + 1] = sn * sn * akk - 2 * cs * sn * ak1 + cs * cs * a11;
    e[k] = cs * sn * (a11 - akk) + (cs * cs - sn * sn) * ak1;
    if (k + 1 < hi) {
      z = sn * e[k + 1];
      e[k + 1] = cs * e[k + 1];
      x = e[k];
    }
    rots.push_back(Rot{k, cs, sn});
  }
}

}  // namespace

int host_syev(int n, double* Ain, double* w) {
  if (n <= 0) return 0;
  std::vector<double> A((size_t)n * n), V((size_t)n * n, 0.0), beta(n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j)
      A[(size_t)i * n + j] = 0.5 * (Ain[(size_t)i * n + j] + Ain[(size_t)j * n + i]);
  std::vector<double> d(n), e(n);
  householder_tridiag(n, A, V, beta, d, e);
  const int ld = (n + 7) & ~7;
  std::vector<double> qbuf((size_t)n * ld + 8);
  double* Qt = qbuf.data();
  Qt += (8 - (reinterpret_cast<uintptr_t>(Qt) / sizeof(double)) % 8) % 8;  // 64-byte aligned
  form_qt(n, V, beta, Qt, ld);
  std::vector<Rot> rots;
  const size_t flush_at = (size_t)1 << 20;
  rots.reserve(std::min(flush_at, (size_t)n * n));
  int hi = n - 1, guard = 0;
  const double eps = 2.220446049250313e-16;
  while (hi > 0) {
    if (std::fabs(e[hi - 1]) <= eps * (std::fabs(d[hi - 1]) + std::fabs(d[hi]))) {
      e[hi - 1] = 0.0;
      --hi;
      continue;
    }
    int lo = hi - 1;
    while (lo > 0 && std::fabs(e[lo - 1]) > eps * (std::fabs(d[lo - 1]) + std::fabs(d[lo]))) --lo;
    if (lo > 0) e[lo - 1] = 0.0;
    qr_step(lo, hi, d, e, rots);
    if (rots.size() >= flush_at) {
      apply_rotations(n, rots, Qt, ld);
      rots.clear();
    }
    if (++guard > 60 * n + 100) return 1;
  }
  apply_rotations(n, rots, Qt, ld);
  std::vector<int> idx(n);
  for (int i = 0; i < n; ++i) idx[i] = i;
  std::stable_sort(idx.begin(), idx.end(), [&](int x, int y) { return d[x] < d[y]; });
  for (int j = 0; j < n; ++j) {
    w[j] = d[idx[j]];
    for (int i = 0; i < n; ++i) Ain[(size_t)i * n + j] = Qt[(size_t)idx[j] * ld + i];
  }
  return 0;
}

int host_cholesky(int n, double* A) {
  // column by column; the rows below the pivot are independent
  for (int j = 0; j < n; ++j) {
    const double* lj = A + (size_t)j * n;
    double s = lj[j];
    for (int k = 0; k < j; ++k) s -= lj[k] * lj[k];
    if (!(s > 0.0)) return 1;
    const double r = std::sqrt(s);
    A[(size_t)j * n + j] = r;
    split_range(n - j - 1, 2.0 * (n - j - 1) * (double)j, [&](int lo, int hi) {
      for (int i = j + 1 + lo; i < j + 1 + hi; ++i) {
        const double* li = A + (size_t)i * n;
        double t = li[j];
        for (int k = 0; k < j; ++k) t -= li[k] * lj[k];
        A[(size_t)i * n + j] = t / r;
      }
    });
  }
  for (int j = 0; j < n; ++j)
    for (int k = j + 1; k < n; ++k) A[(size_t)j * n + k] = 0.0;
  return 0;
}

int host_trinv_lower(int n, double* L) {
  for (int i = 0; i < n; ++i) {
    const double d = L[(size_t)i * n + i];
    if (!(d != 0.0) || !std::isfinite(d)) return 1;
  }
  // column j of M = L^{-1} by forward substitution, M_ij = (delta_ij -
  // sum_{j<=k<i} L_ik M_kj) / L_ii; the columns are independent and are
  // dealt out to the workers in turn (column j costs about (n - j)^2)
  std::vector<double> M((size_t)n * n, 0.0);
  auto column = [&](int j, std::vector<double>& x) {
    for (int i = j; i < n; ++i) {
      const double* li = L + (size_t)i * n;
      double s = (i == j) ? 1.0 : 0.0;
      for (int k = j; k < i; ++k) s -= li[k] * x[k];
      x[i] = s / li[i];
    }
    for (int i = j; i < n; ++i) M[(size_t)i * n + j] = x[i];
  };
  Workers& w = Workers::get();
  if (w.size() == 1 || n < 64) {
    std::vector<double> x(n);
    for (int j = 0; j < n; ++j) column(j, x);
  } else {
    w.run([&](int t, int nt) {
      std::vector<double> x(n);
      for (int j = t; j < n; j += nt) column(j, x);
    });
  }
  std::copy(M.begin(), M.end(), L);
  return 0;
}

}  // namespace bsex
