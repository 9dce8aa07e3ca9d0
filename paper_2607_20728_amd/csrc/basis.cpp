// Plane-wave basis of the Gamma-point sphere: enumeration, order and grid maps.
// The basis is the real orthonormal set of cos/sin plane waves of a sphere
// S = {G : |G|^2/2 <= ecut} (Gamma-only orbitals, SM Sec. IV).
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>

#include "common.h"

namespace bsex {

static thread_local std::string g_err;

void set_error(const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
}

int fail(int code, const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

const char* last_error() { return g_err.c_str(); }

static bool first_nonzero_positive(const int* m) {
  for (int a = 0; a < 3; ++a)
    if (m[a] != 0) return m[a] > 0;
  return false;
}

static bool grid_ok(int n) {
  if (n < 4 || n > 512) return false;
  for (int r : {2, 3, 5})
    while (n % r == 0) n /= r;
  return n == 1;
}

int basis_build(const double cell[3], const int grid[3], double ecut, Basis* b) {
  for (int a = 0; a < 3; ++a) {
    if (!(cell[a] > 0) || !std::isfinite(cell[a]))
      return fail(BSE_EINVAL, "cell length %d must be positive and finite", a);
    if (!grid_ok(grid[a]))
      return fail(BSE_EINVAL, "grid[%d] = %d must be 4..512 and a product of 2, 3, 5", a,
                  grid[a]);
  }
  if (!(ecut > 0) || !std::isfinite(ecut)) return fail(BSE_EINVAL, "ecut must be positive");
  for (int a = 0; a < 3; ++a) {
    b->cell[a] = cell[a];
    b->grid[a] = grid[a];
  }
  b->ecut = ecut;
  b->omega = cell[0] * cell[1] * cell[2];
  b->nr = (long)grid[0] * grid[1] * grid[2];
  const double tp = 2.0 * M_PI;
  // largest |n_a| any sphere vector can have
  int nmax[3];
  for (int a = 0; a < 3; ++a) nmax[a] = (int)std::floor(std::sqrt(2.0 * ecut) * cell[a] / tp) + 1;
  std::vector<int> half;
  for (int i = -nmax[0]; i <= nmax[0]; ++i)
    for (int j = -nmax[1]; j <= nmax[1]; ++j)
      for (int k = -nmax[2]; k <= nmax[2]; ++k) {
        const double gx = tp * i / cell[0], gy = tp * j / cell[1], gz = tp * k / cell[2];
        if (0.5 * (gx * gx + gy * gy + gz * gz) > ecut) continue;
        const int m[3] = {i, j, k};
        for (int a = 0; a < 3; ++a)
          if (2 * std::abs(m[a]) >= grid[a])
            return fail(BSE_EINVAL, "sphere does not fit strictly inside the grid (axis %d)", a);
        if (first_nonzero_positive(m)) half.insert(half.end(), m, m + 3);
      }
  const int nh = (int)half.size() / 3;
  std::vector<int> order(nh);
  for (int i = 0; i < nh; ++i) order[i] = i;
  std::sort(order.begin(), order.end(), [&](int x, int y) {
    const int* a = &half[3 * x];
    const int* c = &half[3 * y];
    const long na = (long)a[0] * a[0] + (long)a[1] * a[1] + (long)a[2] * a[2];
    const long nc = (long)c[0] * c[0] + (long)c[1] * c[1] + (long)c[2] * c[2];
    if (na != nc) return na < nc;
    for (int t = 0; t < 3; ++t)
      if (a[t] != c[t]) return a[t] < c[t];
    return false;
  });
  b->nhalf = nh;
  b->npw = 1 + 2 * nh;
  b->mill_half.resize(3 * (size_t)nh);
  b->idx_p.resize(nh);
  b->idx_m.resize(nh);
  b->g2.assign(b->npw, 0.0);
  for (int s = 0; s < nh; ++s) {
    const int* m = &half[3 * order[s]];
    int lp = 0, lm = 0;
    double g2 = 0;
    for (int a = 0; a < 3; ++a) {
      b->mill_half[3 * s + a] = m[a];
      const int ip = ((m[a] % grid[a]) + grid[a]) % grid[a];
      const int im = ((-m[a] % grid[a]) + grid[a]) % grid[a];
      lp = lp * grid[a] + ip;
      lm = lm * grid[a] + im;
      const double g = tp * m[a] / cell[a];
      g2 += g * g;
    }
    b->idx_p[s] = lp;
    b->idx_m[s] = lm;
    b->g2[1 + 2 * s] = g2;
    b->g2[2 + 2 * s] = g2;
  }
  return BSE_OK;
}

}  // namespace bsex
