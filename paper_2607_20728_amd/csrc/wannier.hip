// Wannier localisation of the occupied orbitals and 8x8 block pruning of the
// W integrals over occupied pairs (the paper's Wannier-localised W
// integrals, main text, computational-cost paragraph after Eq. 7).
//
// Localisation: maximally localised Wannier functions at Gamma by
// simultaneous diagonalisation (F. Gygi, J.-L. Fattebert and E. Schwegler,
// Comput. Phys. Commun. 155, 1 (2003)) of the six real symmetric matrices
//   C_k = <phi| cos(2 pi x_k / L_k) |phi>,  S_k = <phi| sin(2 pi x_k / L_k) |phi>,
// each weighted by (L_k / 2 pi)^2: the spread
//   sum_k (L_k / 2 pi)^2 sum_j [1 - C_k[j][j]^2 - S_k[j][j]^2]
// falls as the weighted squared diagonals grow.  A Jacobi sweep is a
// round-robin tournament (circle method, a dummy index for odd n): the
// pairs of a round are disjoint, so the round takes all its angles from the
// same matrices (the 2x2 eigenproblem of Cardoso and Souloumiac, SIAM J.
// Matrix Anal. Appl. 17, 161 (1996)) and then rotates every 2x2 block of
// the six matrices, and the columns of U, at once.  The matrices are grid
// quadratures: GEMMs of the orbital rows with their cos / sin weighted
// copies on the MFMA FP64 path.  Centres come from the final diagonals and
// the localised orbitals are put in Morton order of them (1024 cells per
// axis, ties by index), so the 8 orbitals of a band block lie together.
//
// Pruning: s[j][j'] = ||w_j w_j'|| / (||w_j^2|| ||w_j'^2||)^(1/2), L2 norms
// (one more GEMM, of the squared rows): the norm of the pair density, which
// bounds that of tau_jj' = W(w_j w_j'), made scale free (in [0, 1], 1 on the
// diagonal).  An 8x8 block (I, J), I <= J, keeps its W integrals when its
// largest s is at least the threshold (diagonal blocks always).  The kept list replaces the full block triangle in
// the tau cache, its rebuild tiles and the stream launches.
#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

#include "context.h"
#include "kernels.h"

namespace bsex {
namespace {

constexpr int TPB = 256;

unsigned nblocks_of(long n) { return (unsigned)((n + TPB - 1) / TPB); }

struct Scratch {  // device scratch owned by the context for one call
  bse_ctx* c;
  double* p = nullptr;
  explicit Scratch(bse_ctx* c_) : c(c_) {}
  int alloc(size_t n) { return ctx_alloc_t(c, &p, n); }
  ~Scratch() { ctx_release(c, p); }
  Scratch(const Scratch&) = delete;
  Scratch& operator=(const Scratch&) = delete;
};

int put(bse_ctx* c, void* dst, const void* src, size_t bytes) {
  return stage_h2d(&c->hstage, src, dst, bytes, c->st);
}

int get(bse_ctx* c, const double* src, std::vector<double>& h, size_t n) {
  if (n > h.size()) return fail(BSE_EINVAL, "copy of %zu values into %zu", n, h.size());
  return stage_d2h(&c->hstage, src, h.data(), sizeof(double) * n, c->st);
}

// real rows of packed orbital grids: out[v][r] = component v & 1 of grid
// v >> 1 (its square when squared)
__global__ void k_unpack_rows(const double2* __restrict__ g, int nv, long nr, int squared,
                              double* __restrict__ out) {
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i >= (long)nv * nr) return;
  const int v = (int)(i / nr);
  const long r = i - (long)v * nr;
  const double2 w = g[(long)(v >> 1) * nr + r];
  const double x = (v & 1) ? w.y : w.x;
  out[i] = squared ? x * x : x;
}

// out[v][r] = P[v][r] f(2 pi i_k / N_k), f = cos or sin, i_k the grid index
// of point r along axis k
__global__ void k_axis_weight(const double* __restrict__ P, long n, int n1, int n2, int n3,
                              int axis, int fsin, double* __restrict__ out) {
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const long nr = (long)n1 * n2 * n3;
  const long r = i % nr;
  int ik, nk;
  if (axis == 0) {
    ik = (int)(r / ((long)n2 * n3));
    nk = n1;
  } else if (axis == 1) {
    ik = (int)((r / n3) % n2);
    nk = n2;
  } else {
    ik = (int)(r % n3);
    nk = n3;
  }
  const double a = 2.0 * M_PI * (double)ik / (double)nk;
  out[i] = P[i] * (fsin ? sin(a) : cos(a));
}

struct Weights {
  double w[6];
};

// the plane rotation (c, s) of each pair slot of one round: the dominant
// eigenvector (cos 2t, sin 2t) of G = sum_m w_m g_m g_m^T,
// g_m = (A_m[i][i] - A_m[j][j], 2 A_m[i][j]), with cos 2t >= 0
__global__ void k_jacobi_angles(const double* __restrict__ M, long nn, int n,
                                const int2* __restrict__ slots, int ns, Weights wt,
                                double2* __restrict__ cs) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= ns) return;
  const int2 q = slots[p];
  if (q.y < 0) {
    cs[p] = make_double2(1.0, 0.0);
    return;
  }
  double a = 0.0, b = 0.0, d = 0.0;
  for (int m = 0; m < 6; ++m) {
    const double* A = M + m * nn;
    const double g0 = A[(long)q.x * n + q.x] - A[(long)q.y * n + q.y];
    const double g1 = 2.0 * A[(long)q.x * n + q.y];
    a += wt.w[m] * g0 * g0;
    b += wt.w[m] * g0 * g1;
    d += wt.w[m] * g1 * g1;
  }
  const double h = 0.5 * (a - d), r = sqrt(h * h + b * b);
  if (r == 0.0) {  // every angle is as good
    cs[p] = make_double2(1.0, 0.0);
    return;
  }
  // (G - lambda_max) v = 0, from whichever row is better conditioned
  double x, y;
  if (h >= 0.0) {
    x = h + r;
    y = b;
  } else {
    x = b;
    y = r - h;
  }
  const double nrm = sqrt(x * x + y * y);
  x /= nrm;
  y /= nrm;
  if (x < 0.0) {
    x = -x;
    y = -y;
  }
  const double c = sqrt(0.5 * (1.0 + x));
  cs[p] = make_double2(c, y / (2.0 * c));
}

// A <- R^T A R for the six matrices, one 2x2 block (rows of slot p, columns
// of slot q) per thread; R maps column i to c e_i + s e_j and column j to
// -s e_i + c e_j for every pair (i, j) of the round
__global__ void k_jacobi_rotate(double* __restrict__ M, long nn, int n,
                                const int2* __restrict__ slots, int ns,
                                const double2* __restrict__ cs) {
  const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  const long per = (long)ns * ns;
  if (t >= 6 * per) return;
  const int m = (int)(t / per);
  const long pq = t - m * per;
  const int p = (int)(pq / ns), q = (int)(pq % ns);
  const int2 P = slots[p], Q = slots[q];
  const double2 cp = cs[p], cq = cs[q];
  double* A = M + m * nn;
  const bool py = P.y >= 0, qy = Q.y >= 0;
  const double a00 = A[(long)P.x * n + Q.x];
  const double a01 = qy ? A[(long)P.x * n + Q.y] : 0.0;
  const double a10 = py ? A[(long)P.y * n + Q.x] : 0.0;
  const double a11 = (py && qy) ? A[(long)P.y * n + Q.y] : 0.0;
  // B = A R (columns of slot q)
  const double b00 = cq.x * a00 + cq.y * a01, b01 = -cq.y * a00 + cq.x * a01;
  const double b10 = cq.x * a10 + cq.y * a11, b11 = -cq.y * a10 + cq.x * a11;
  // R^T B (rows of slot p)
  A[(long)P.x * n + Q.x] = cp.x * b00 + cp.y * b10;
  if (qy) A[(long)P.x * n + Q.y] = cp.x * b01 + cp.y * b11;
  if (py) A[(long)P.y * n + Q.x] = -cp.y * b00 + cp.x * b10;
  if (py && qy) A[(long)P.y * n + Q.y] = -cp.y * b01 + cp.x * b11;
}

// U <- U R (columns of every pair), one (row, slot) per thread
__global__ void k_jacobi_rotate_u(double* __restrict__ U, int n, const int2* __restrict__ slots,
                                  int ns, const double2* __restrict__ cs) {
  const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (t >= (long)n * ns) return;
  const int x = (int)(t / ns), p = (int)(t % ns);
  const int2 P = slots[p];
  if (P.y < 0) return;
  const double2 c = cs[p];
  const double u0 = U[(long)x * n + P.x], u1 = U[(long)x * n + P.y];
  U[(long)x * n + P.x] = c.x * u0 + c.y * u1;
  U[(long)x * n + P.y] = -c.y * u0 + c.x * u1;
}

__global__ void k_diag6(const double* __restrict__ M, long nn, int n, double* __restrict__ out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 6 * n) return;
  const int m = t / n, j = t % n;
  out[t] = M[m * nn + (long)j * n + j];
}

__global__ void k_eye(double* U, int n) {
  const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (t >= (long)n * n) return;
  U[t] = (t / n == t % n) ? 1.0 : 0.0;
}

// rounds of the circle method: round r pairs positions k and m-1-k of
// p_r, p_r[0] = 0 and p_r[i] = 1 + ((i - 1 - r) mod (m - 1)); an index
// paired with the dummy m - 1 of odd n (m = n + 1) idles (slot (i, -1))
std::vector<int2> tournament_slots(int n, int* nrounds, int* nslots) {
  const int m = n + (n % 2);
  *nrounds = std::max(1, m - 1);
  *nslots = m / 2;
  std::vector<int2> out;
  for (int r = 0; r < *nrounds; ++r) {
    std::vector<int> p(m);
    p[0] = 0;
    for (int i = 1; i < m; ++i) p[i] = 1 + (((i - 1 - r) % (m - 1)) + (m - 1)) % (m - 1);
    for (int k = 0; k < m / 2; ++k) {
      int a = p[k], b = p[m - 1 - k];
      if (a >= n) std::swap(a, b);
      if (b >= n)
        out.push_back(make_int2(a, -1));
      else
        out.push_back(make_int2(std::min(a, b), std::max(a, b)));
    }
  }
  return out;
}

double spread_of(const std::vector<double>& diag, int n, const double* wt) {
  double tot = 0.0;
  for (int k = 0; k < 3; ++k) {
    double s = 0.0;
    for (int j = 0; j < n; ++j) {
      const double cc = diag[(2 * k) * n + j], ss = diag[(2 * k + 1) * n + j];
      s += cc * cc + ss * ss;
    }
    tot += wt[2 * k] * ((double)n - s);
  }
  return tot;
}

// the six position matrices of the orbital grids g (packed [nvh][nr])
int position_matrices(bse_ctx* c, const double2* g, double* P, double* W, double* M) {
  const int nv = c->nv;
  const long nr = c->basis.nr, n = (long)nv * nr, nn = (long)nv * nv;
  const double dv = c->basis.omega / (double)nr;
  hipLaunchKernelGGL(k_unpack_rows, dim3(nblocks_of(n)), dim3(TPB), 0, c->st, g, nv, nr, 0, P);
  BSE_HIP(hipGetLastError());
  for (int k = 0; k < 3; ++k)
    for (int f = 0; f < 2; ++f) {
      hipLaunchKernelGGL(k_axis_weight, dim3(nblocks_of(n)), dim3(TPB), 0, c->st, P, n,
                         c->basis.grid[0], c->basis.grid[1], c->basis.grid[2], k, f, W);
      BSE_HIP(hipGetLastError());
      BSE_TRY(dgemm(0, 1, nv, nv, nr, dv, W, nr, P, nr, 0.0, M + (2 * k + f) * nn, nv, c->st));
    }
  return BSE_OK;
}

int diagonals(bse_ctx* c, const double* M, double* d6, std::vector<double>& h) {
  const int nv = c->nv;
  hipLaunchKernelGGL(k_diag6, dim3(nblocks_of(6L * nv)), dim3(TPB), 0, c->st, M, (long)nv * nv,
                     nv, d6);
  BSE_HIP(hipGetLastError());
  h.resize(6 * (size_t)nv);
  return get(c, d6, h, h.size());
}

}  // namespace

// Localised frame, rotated orbitals and the kept block list (sets c->Uloc,
// Phi_loc, phir_loc, loc_*, blkIJ_h; the caller uploads the block list)
int localize(bse_ctx* c, const bse_system_desc* d) {
  const int nv = c->nv;
  const long nr = c->basis.nr, npw = c->basis.npw, nn = (long)nv * nv;
  const double dv = c->basis.omega / (double)nr;
  double wt[6];
  for (int k = 0; k < 3; ++k) wt[2 * k] = wt[2 * k + 1] = std::pow(c->basis.cell[k] / (2.0 * M_PI), 2);
  Scratch P(c), W(c), M(c), d6(c);
  BSE_TRY(P.alloc((size_t)nv * nr));
  BSE_TRY(W.alloc((size_t)nv * nr));
  BSE_TRY(M.alloc(6 * (size_t)nn));
  BSE_TRY(d6.alloc(6 * (size_t)nv));
  BSE_TRY(ctx_alloc_t(c, &c->Uloc, (size_t)nn));
  BSE_TRY(ctx_alloc_t(c, &c->Phi_loc, (size_t)nv * npw));
  BSE_TRY(ctx_alloc_t(c, &c->phir_loc, (size_t)c->nvh * nr));
  std::vector<double> dh;
  auto rotate_orbitals = [&]() -> int {
    // Phi_loc = U^T Phi, then its grids
    BSE_TRY(dgemm(1, 0, nv, npw, nv, 1.0, c->Uloc, nv, c->Phi, npw, 0.0, c->Phi_loc, npw,
                  c->st));
    return to_grid(c, c->Phi_loc, nv, 1, c->phir_loc);
  };
  c->loc_U_h.assign((size_t)nn, 0.0);
  if (d->loc_rotation) {
    std::copy(d->loc_rotation, d->loc_rotation + nn, c->loc_U_h.begin());
    BSE_TRY(put(c, c->Uloc, c->loc_U_h.data(), sizeof(double) * nn));
    BSE_TRY(rotate_orbitals());
    BSE_TRY(position_matrices(c, c->phir_loc, P.p, W.p, M.p));
    BSE_TRY(diagonals(c, M.p, d6.p, dh));
    c->loc_sweeps = 0;
  } else {
    BSE_TRY(position_matrices(c, c->phir, P.p, W.p, M.p));
    hipLaunchKernelGGL(k_eye, dim3(nblocks_of(nn)), dim3(TPB), 0, c->st, c->Uloc, nv);
    BSE_HIP(hipGetLastError());
    int nrounds = 0, ns = 0;
    const std::vector<int2> slots = tournament_slots(nv, &nrounds, &ns);
    int2* sl = nullptr;
    double2* cs = nullptr;
    BSE_TRY(ctx_alloc_t(c, &sl, slots.size()));
    BSE_TRY(ctx_alloc_t(c, &cs, (size_t)ns));
    int rc = put(c, sl, slots.data(), sizeof(int2) * slots.size());
    Weights w6;
    for (int m = 0; m < 6; ++m) w6.w[m] = wt[m];
    const int max_sweeps = d->loc_max_sweeps > 0 ? d->loc_max_sweeps : 100;
    const double tol = d->loc_tol > 0 ? d->loc_tol : 1e-9;
    if (rc == BSE_OK) rc = diagonals(c, M.p, d6.p, dh);
    double prev = spread_of(dh, nv, wt);
    int sweeps = 0;
    for (sweeps = 1; rc == BSE_OK && sweeps <= max_sweeps && nv > 1; ++sweeps) {
      for (int r = 0; r < nrounds; ++r) {
        const int2* rs = sl + (long)r * ns;
        hipLaunchKernelGGL(k_jacobi_angles, dim3(nblocks_of(ns)), dim3(TPB), 0, c->st, M.p, nn,
                           nv, rs, ns, w6, cs);
        hipLaunchKernelGGL(k_jacobi_rotate, dim3(nblocks_of(6L * ns * ns)), dim3(TPB), 0, c->st,
                           M.p, nn, nv, rs, ns, cs);
        hipLaunchKernelGGL(k_jacobi_rotate_u, dim3(nblocks_of((long)nv * ns)), dim3(TPB), 0,
                           c->st, c->Uloc, nv, rs, ns, cs);
      }
      if (hipGetLastError() != hipSuccess) {
        rc = fail(BSE_EHIP, "localisation kernels failed");
        break;
      }
      rc = diagonals(c, M.p, d6.p, dh);
      if (rc != BSE_OK) break;
      const double cur = spread_of(dh, nv, wt);
      const bool done = prev - cur < tol * cur;
      prev = cur;
      if (done) break;
    }
    ctx_release(c, sl);
    ctx_release(c, cs);
    BSE_TRY(rc);
    c->loc_sweeps = std::min(sweeps, max_sweeps);
    if (nv <= 1) c->loc_sweeps = 0;
    // Morton order of the centres: permute the columns of U
    std::vector<double> cen(3 * (size_t)nv);
    for (int j = 0; j < nv; ++j)
      for (int k = 0; k < 3; ++k) {
        double f = std::atan2(dh[(2 * k + 1) * nv + j], dh[(2 * k) * nv + j]) / (2.0 * M_PI);
        f -= std::floor(f);
        cen[3 * j + k] = f * c->basis.cell[k];
      }
    std::vector<long long> code(nv, 0);
    for (int j = 0; j < nv; ++j) {
      long long q[3];
      for (int k = 0; k < 3; ++k)
        q[k] = std::min<long long>((long long)(cen[3 * j + k] / c->basis.cell[k] * 1024.0), 1023);
      for (int bit = 0; bit < 10; ++bit)
        for (int k = 0; k < 3; ++k) code[j] |= ((q[k] >> bit) & 1LL) << (3 * bit + k);
    }
    std::vector<int> perm(nv);
    std::iota(perm.begin(), perm.end(), 0);
    std::stable_sort(perm.begin(), perm.end(), [&](int a, int b) { return code[a] < code[b]; });
    std::vector<double> Uh((size_t)nn);
    BSE_TRY(get(c, c->Uloc, Uh, Uh.size()));
    std::vector<double> dp(dh.size());
    for (int v = 0; v < nv; ++v)
      for (int j = 0; j < nv; ++j) c->loc_U_h[(size_t)v * nv + j] = Uh[(size_t)v * nv + perm[j]];
    for (int m = 0; m < 6; ++m)
      for (int j = 0; j < nv; ++j) dp[(size_t)m * nv + j] = dh[(size_t)m * nv + perm[j]];
    dh.swap(dp);
    BSE_TRY(put(c, c->Uloc, c->loc_U_h.data(), sizeof(double) * nn));
    BSE_TRY(rotate_orbitals());
  }
  c->loc_spread = spread_of(dh, nv, wt);
  c->loc_cen_h.assign(3 * (size_t)nv, 0.0);
  for (int j = 0; j < nv; ++j)
    for (int k = 0; k < 3; ++k) {
      double f = std::atan2(dh[(2 * k + 1) * nv + j], dh[(2 * k) * nv + j]) / (2.0 * M_PI);
      f -= std::floor(f);
      c->loc_cen_h[3 * j + k] = f * c->basis.cell[k];
    }
  // pair measure and the kept blocks
  hipLaunchKernelGGL(k_unpack_rows, dim3(nblocks_of((long)nv * nr)), dim3(TPB), 0, c->st,
                     c->phir_loc, nv, nr, 1, P.p);
  BSE_HIP(hipGetLastError());
  BSE_TRY(dgemm(0, 1, nv, nv, nr, dv, P.p, nr, P.p, nr, 0.0, M.p, nv, c->st));
  std::vector<double> s((size_t)nn);
  BSE_TRY(get(c, M.p, s, s.size()));
  {
    std::vector<double> dg(nv);
    for (int j = 0; j < nv; ++j) dg[j] = std::sqrt(s[(size_t)j * nv + j]);
    for (int j = 0; j < nv; ++j)
      for (int jp = 0; jp < nv; ++jp)
        s[(size_t)j * nv + jp] = std::sqrt(s[(size_t)j * nv + jp] / (dg[j] * dg[jp]));
  }
  const long nB = (nv + 7) / 8;
  std::vector<int2> keep;
  for (long I = 0; I < nB; ++I)
    for (long J = I; J < nB; ++J) {
      double mx = 0.0;
      for (long j = 8 * I; j < std::min<long>(8 * I + 8, nv); ++j)
        for (long jp = 8 * J; jp < std::min<long>(8 * J + 8, nv); ++jp)
          mx = std::max(mx, s[(size_t)j * nv + jp]);
      if (I == J || mx >= c->prune_thr) keep.push_back(make_int2((int)I, (int)J));
    }
  c->blkIJ_h = keep;
  c->nblk_all = nB * (nB + 1) / 2;
  return BSE_OK;
}

}  // namespace bsex
