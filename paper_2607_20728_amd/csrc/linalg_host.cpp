// Small dense symmetric eigensolver and Cholesky on the host (FP64).
//
// Eigensolver: Householder reduction to tridiagonal form T = Q^T A Q (Q
// accumulated explicitly), then implicit symmetric QR steps with the
// Wilkinson shift, chasing the bulge with plane rotations and deflating
// negligible off-diagonal entries (the method of Golub and Van Loan,
// "Matrix Computations", Sec. 8.3).  Used for the Rayleigh-Ritz problems of
// the Davidson and ground-state subspace solvers (n up to a few hundred).
#include <algorithm>
#include <cmath>
#include <vector>

#include "common.h"

namespace bsex {

namespace {

struct Mat {
  int n;
  std::vector<double> a;
  double& operator()(int i, int j) { return a[(size_t)i * n + j]; }
};

// A <- Q^T A Q tridiagonal; Q accumulated (Q starts as identity).
void householder_tridiag(Mat& A, Mat& Q, std::vector<double>& d, std::vector<double>& e) {
  const int n = A.n;
  std::vector<double> v(n), p(n), w(n);
  for (int k = 0; k + 2 < n; ++k) {
    const int m = n - k - 1;  // length of the column below the diagonal
    double nrm2 = 0.0;
    for (int i = 0; i < m; ++i) {
      v[i] = A(k + 1 + i, k);
      nrm2 += v[i] * v[i];
    }
    double tail = nrm2 - v[0] * v[0];
    if (tail <= 0.0) continue;  // already tridiagonal in this column
    const double nrm = std::sqrt(nrm2);
    const double alpha = v[0] > 0 ? -nrm : nrm;
    v[0] -= alpha;
    double vv = v[0] * v[0] + tail;
    const double beta = 2.0 / vv;
    // p = beta * B v, B the trailing block
    for (int i = 0; i < m; ++i) {
      double s = 0.0;
      for (int j = 0; j < m; ++j) s += A(k + 1 + i, k + 1 + j) * v[j];
      p[i] = beta * s;
    }
    double pv = 0.0;
    for (int i = 0; i < m; ++i) pv += p[i] * v[i];
    const double K = 0.5 * beta * pv;
    for (int i = 0; i < m; ++i) w[i] = p[i] - K * v[i];
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j) A(k + 1 + i, k + 1 + j) -= v[i] * w[j] + w[i] * v[j];
    A(k + 1, k) = A(k, k + 1) = alpha;
    for (int i = 1; i < m; ++i) A(k + 1 + i, k) = A(k, k + 1 + i) = 0.0;
    // Q <- Q (I - beta v v^T) on columns k+1..n-1
    for (int r = 0; r < n; ++r) {
      double s = 0.0;
      for (int j = 0; j < m; ++j) s += Q(r, k + 1 + j) * v[j];
      s *= beta;
      for (int j = 0; j < m; ++j) Q(r, k + 1 + j) -= s * v[j];
    }
  }
  for (int i = 0; i < n; ++i) d[i] = A(i, i);
  for (int i = 0; i + 1 < n; ++i) e[i] = A(i + 1, i);
  e[n - 1] = 0.0;
}

// One implicit Wilkinson-shifted QR step on the unreduced block [lo, hi].
// Qt holds the eigenvector estimates as rows (Q transposed), so each plane
// rotation combines two contiguous rows.
void qr_step(int lo, int hi, std::vector<double>& d, std::vector<double>& e, Mat& Qt) {
  const int n = Qt.n;
  const double a = d[hi - 1], b = e[hi - 1], c = d[hi];
  const double delta = 0.5 * (a - c);
  const double rad = std::hypot(delta, b);
  const double mu = c - b * b / (delta + (delta >= 0 ? rad : -rad));
  double x = d[lo] - mu, z = e[lo];
  for (int k = lo; k < hi; ++k) {
    const double r = std::hypot(x, z);
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
    double* rk = &Qt(k, 0);
    double* r1 = &Qt(k + 1, 0);
    for (int i = 0; i < n; ++i) {
      const double qk = rk[i], q1 = r1[i];
      rk[i] = cs * qk + sn * q1;
      r1[i] = -sn * qk + cs * q1;
    }
  }
}

}  // namespace

int host_syev(int n, double* Ain, double* w) {
  if (n <= 0) return 0;
  Mat A{n, std::vector<double>((size_t)n * n)};
  Mat Q{n, std::vector<double>((size_t)n * n, 0.0)};
  for (int i = 0; i < n; ++i) {
    Q(i, i) = 1.0;
    for (int j = 0; j < n; ++j) A(i, j) = 0.5 * (Ain[(size_t)i * n + j] + Ain[(size_t)j * n + i]);
  }
  std::vector<double> d(n), e(n);
  householder_tridiag(A, Q, d, e);
  Mat& Qt = A;  // A is no longer needed: it receives Q transposed
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) Qt(j, i) = Q(i, j);
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
    qr_step(lo, hi, d, e, Qt);
    if (++guard > 60 * n + 100) return 1;
  }
  std::vector<int> idx(n);
  for (int i = 0; i < n; ++i) idx[i] = i;
  std::stable_sort(idx.begin(), idx.end(), [&](int x, int y) { return d[x] < d[y]; });
  for (int j = 0; j < n; ++j) {
    w[j] = d[idx[j]];
    for (int i = 0; i < n; ++i) Ain[(size_t)i * n + j] = Qt(idx[j], i);
  }
  return 0;
}

int host_cholesky(int n, double* A) {
  for (int j = 0; j < n; ++j) {
    double s = A[(size_t)j * n + j];
    for (int k = 0; k < j; ++k) s -= A[(size_t)j * n + k] * A[(size_t)j * n + k];
    if (!(s > 0.0)) return 1;
    const double r = std::sqrt(s);
    A[(size_t)j * n + j] = r;
    for (int i = j + 1; i < n; ++i) {
      double t = A[(size_t)i * n + j];
      for (int k = 0; k < j; ++k) t -= A[(size_t)i * n + k] * A[(size_t)j * n + k];
      A[(size_t)i * n + j] = t / r;
    }
    for (int k = j + 1; k < n; ++k) A[(size_t)j * n + k] = 0.0;
  }
  return 0;
}

}  // namespace bsex
