"""Wannier localisation of the occupied orbitals and block pruning of the
occupied-pair W integrals -- oracle, test infrastructure.

The paper makes the integrals that involve W and KS orbitals affordable by
Wannier localisation (main text, the paragraph on computational cost after
Eq. 7, citing Gygi et al. 2003 and Yu et al. 2024); it gives no details.  The
reading taken here:

Localisation.  Maximally localised Wannier functions at Gamma by simultaneous
diagonalisation (F. Gygi, J.-L. Fattebert and E. Schwegler, Comput. Phys.
Commun. 155, 1 (2003)).  In an orthorhombic cell with edges L_k the position
operator enters through the real symmetric matrices

    C_k[v][v'] = <phi_v| cos(2 pi x_k / L_k) |phi_v'>,
    S_k[v][v'] = <phi_v| sin(2 pi x_k / L_k) |phi_v'>       (k = 1, 2, 3),

grid quadratures, exact because the integrand's zero frequency cannot alias
while 2 m_k + 1 < N_k.  The spread

    spread = sum_k (L_k / 2 pi)^2 sum_j [1 - C_k[j][j]^2 - S_k[j][j]^2]

is minimised over orthogonal U (localised orbitals w_j = sum_v U[v][j] phi_v)
by Jacobi sweeps.  A sweep visits every pair once in the rounds of a
round-robin tournament (circle method: n - 1 rounds of n/2 disjoint pairs
for even n, a dummy index added for odd n); rotations in disjoint planes
commute and do not change each other's 2x2 data, so a round takes all its
angles from the same matrices and then applies all its rotations.  A plane
rotation by theta in the (i, j) plane leaves A[i][i] + A[j][j] of every
matrix unchanged and turns A[i][i] - A[j][j] into g . (cos 2 theta,
sin 2 theta) with g = (A[i][i] - A[j][j], 2 A[i][j]); so the weighted sum of
squared diagonals of the six matrices is largest when (cos 2 theta,
sin 2 theta) is the dominant eigenvector of G = sum_m a_m g_m g_m^T
(a_m = (L_k/2 pi)^2), taken with cos 2 theta >= 0 (J.-F. Cardoso and
A. Souloumiac, SIAM J. Matrix Anal. Appl. 17, 161 (1996)).  Sweeps stop when
a sweep lowers the spread by less than tol times the spread, or after
max_sweeps.

Centres and order.  x_k(j) = L_k/(2 pi) arg(C_k[j][j] + i S_k[j][j]) in
[0, L_k).  The localised orbitals are put in the Morton (Z) order of their
centres on a 1024^3 grid of fractional coordinates (ties by index), so that
the 8 orbitals of a band block lie close together.

Pruning.  Pair measure s[j][j'] = ||w_j w_j'|| / (||w_j^2|| ||w_j'^2||)^(1/2)
with the L2 norm on the grid: the norm of the pair density, which bounds the
norm of tau_jj' = W(w_j w_j') by that of W, made scale free (Cauchy-Schwarz
puts it in [0, 1], with 1 on the diagonal).  The bands form blocks of 8 (the
unit of the tau cache);
block (I, J), I <= J, is kept when the largest s over its pairs is at least
the threshold, and then all of its pairs are kept (both orders); diagonal
blocks, which hold the self pairs (s = 1), are always kept.

The pruned model.  Every W integral over a pair of occupied indices in the
localised frame is restricted to the kept pairs, with a~ = U^T a:

    (K1d A)_v = P_c sum_j U[v][j] sum_{j' kept with j} W(w_j' w_j) a~_j'
    sigma_v   = sum_j U[v][j] sum_{j' kept with j} W(a~_j' a~_j) w_j'   (U's W term)

With every block kept both equal the canonical ones (the operator is
covariant under orthogonal rotations of the occupied orbitals when A rotates
with them).  The rest of the method is unchanged, and the pruned operator
stays symmetric.  For forces, the frame and the kept list are those of the
reference geometry; at a displaced geometry the frame is the symmetric
(Loewdin) alignment of the reference localised orbitals to the new occupied
space, which to first order moves the frame only along P_c, so the Z-vector
Lagrangian of Eqs. 4-7 applies unchanged.

Pins: tests/test_oracle_wannier.py (Jacobi angle against a brute-force
search; monotone spread; recovery of mixed, well separated localised
functions and their centres; every block kept reproduces the canonical apply
and U; the pruned apply against the dropped pairs added back one by one;
symmetry; d omega/d R of the pruned model against central differences with
the frame and list frozen).
"""
from __future__ import annotations

import numpy as np

from . import solvers
from .model import System, K_1E, K_1D_BARE, K_1D_PDEP

BLOCK = 8


# ---------------------------------------------------------------------------
# localisation
# ---------------------------------------------------------------------------
def position_matrices(b, phir):
    """The six matrices [C_1, S_1, C_2, S_2, C_3, S_3] of phir[n][grid] and
    their weights (L_k / 2 pi)^2."""
    n = phir.shape[0]
    flat = phir.reshape(n, -1)
    dv = b.omega / b.n_r
    mats, wts = [], []
    for k in range(3):
        ang = 2.0 * np.pi * np.arange(b.grid[k]) / b.grid[k]     # 2 pi x_k / L_k on the grid
        shape = [1, 1, 1]
        shape[k] = b.grid[k]
        for f in (np.cos, np.sin):
            w = f(ang).reshape(shape)
            mats.append(((phir * w).reshape(n, -1) @ flat.T) * dv)
            wts.append((b.cell[k] / (2.0 * np.pi)) ** 2)
    return mats, np.array(wts)


def spread(mats, wts):
    n = mats[0].shape[0]
    tot = 0.0
    for k in range(3):
        c, s = np.diag(mats[2 * k]), np.diag(mats[2 * k + 1])
        tot += wts[2 * k] * (n - (c * c + s * s).sum())
    return tot


def jacobi_angle(mats, wts, i, j):
    """(cos theta, sin theta) of the plane rotation of pair (i, j) that
    maximises the weighted squared diagonals (module docstring)."""
    G = np.zeros((2, 2))
    for A, a in zip(mats, wts):
        g = np.array([A[i, i] - A[j, j], 2.0 * A[i, j]])
        G += a * np.outer(g, g)
    w, V = np.linalg.eigh(G)
    x, y = V[:, 1]
    if w[1] - w[0] <= 1e-300:                       # every angle is as good
        return 1.0, 0.0
    if x < 0:
        x, y = -x, -y
    c = np.sqrt(0.5 * (1.0 + x))
    return c, y / (2.0 * c)


def tournament(n):
    """Rounds of disjoint pairs covering every pair (i < j) of range(n) once
    (circle method; index n stands for the dummy of odd n and is dropped)."""
    m = n + (n % 2)
    p = list(range(m))
    rounds = []
    for _ in range(m - 1):
        pairs = []
        for k in range(m // 2):
            a, b = p[k], p[m - 1 - k]
            if a < n and b < n:
                pairs.append((min(a, b), max(a, b)))
        rounds.append(pairs)
        p = [p[0]] + [p[-1]] + p[1:-1]
    return rounds


def rotate(mats, U, i, j, c, s):
    """Apply the plane rotation (columns i -> c e_i + s e_j, j -> -s e_i +
    c e_j) to every matrix (A <- R^T A R) and to U (U <- U R), in place."""
    for A in mats:
        ai, aj = A[:, i].copy(), A[:, j].copy()
        A[:, i], A[:, j] = c * ai + s * aj, -s * ai + c * aj
        ai, aj = A[i, :].copy(), A[j, :].copy()
        A[i, :], A[j, :] = c * ai + s * aj, -s * ai + c * aj
    ui, uj = U[:, i].copy(), U[:, j].copy()
    U[:, i], U[:, j] = c * ui + s * uj, -s * ui + c * uj


def localize(b, phir, tol=1e-9, max_sweeps=100):
    """Jacobi sweeps from U = 1.  Returns (U, info) with info['spread'] per
    sweep (index 0: before any rotation), info['sweeps'] and the rotated
    matrices."""
    mats, wts = position_matrices(b, phir)
    mats = [A.copy() for A in mats]
    n = phir.shape[0]
    U = np.eye(n)
    hist = [spread(mats, wts)]
    rounds = tournament(n)
    sweeps = 0
    for sweeps in range(1, max_sweeps + 1):
        for pairs in rounds:
            rot = [(i, j) + jacobi_angle(mats, wts, i, j) for i, j in pairs]
            for i, j, c, s in rot:
                rotate(mats, U, i, j, c, s)
        hist.append(spread(mats, wts))
        if hist[-2] - hist[-1] < tol * hist[-1]:
            break
    return U, dict(spread=hist, sweeps=sweeps, mats=mats, wts=wts)


def centres(b, mats):
    """Centre of every localised orbital from the rotated matrices."""
    out = np.zeros((mats[0].shape[0], 3))
    for k in range(3):
        z = np.diag(mats[2 * k]) + 1j * np.diag(mats[2 * k + 1])
        out[:, k] = np.mod(np.angle(z) / (2.0 * np.pi), 1.0) * b.cell[k]
    return out


def morton_order(b, cen):
    """Permutation putting the centres in Morton order (1024 cells per axis,
    ties by index)."""
    q = np.minimum((cen / b.cell[None, :] * 1024.0).astype(np.int64), 1023)
    code = np.zeros(len(cen), dtype=np.int64)
    for bit in range(10):
        for k in range(3):
            code |= ((q[:, k] >> bit) & 1) << (3 * bit + k)
    return np.lexsort((np.arange(len(cen)), code))


def localized_frame(b, phir, tol=1e-9, max_sweeps=100):
    """U whose columns are the localised orbitals in Morton order of their
    centres; also returns the centres (same order) and the localisation
    info."""
    U, info = localize(b, phir, tol=tol, max_sweeps=max_sweeps)
    cen = centres(b, info["mats"])
    perm = morton_order(b, cen)
    return U[:, perm], cen[perm], info


# ---------------------------------------------------------------------------
# pruning
# ---------------------------------------------------------------------------
def pair_measure(b, wr):
    """s[j][j'] = ||w_j w_j'|| / (||w_j^2|| ||w_j'^2||)^(1/2) (L2 norms, grid
    quadrature)."""
    q = wr.reshape(wr.shape[0], -1) ** 2
    G = (q @ q.T) * (b.omega / b.n_r)                # integral w_j^2 w_j'^2
    d = np.sqrt(np.diag(G))
    return np.sqrt(G / np.outer(d, d))


def kept_blocks(s, threshold):
    """[(I, J)] of the blocks kept (I <= J), in row order."""
    n = s.shape[0]
    nb = (n + BLOCK - 1) // BLOCK
    out = []
    for I in range(nb):
        for J in range(I, nb):
            blk = s[I * BLOCK:(I + 1) * BLOCK, J * BLOCK:(J + 1) * BLOCK]
            if I == J or blk.max() >= threshold:
                out.append((I, J))
    return out


def pair_mask(n, blocks):
    """Boolean [n][n]: pair (j, j') kept."""
    m = np.zeros((n, n), dtype=bool)
    for I, J in blocks:
        m[I * BLOCK:(I + 1) * BLOCK, J * BLOCK:(J + 1) * BLOCK] = True
        m[J * BLOCK:(J + 1) * BLOCK, I * BLOCK:(I + 1) * BLOCK] = True
    return m


def loewdin_frame(phi, L0):
    """Orthogonal U (columns: coefficients over the rows of phi) whose
    localised orbitals U^T phi are the symmetric alignment of the reference
    localised orbitals L0[n][N_pw] to the span of phi."""
    O = phi @ L0.T                                    # O[v][j] = <phi_v|l_j>
    w, V = np.linalg.eigh(O.T @ O)
    return O @ (V * (1.0 / np.sqrt(w))) @ V.T


class WannierSystem(System):
    """System whose occupied-pair W integrals are pruned in a localised frame
    (module docstring).  set_frame(U, blocks) fixes the frame and the kept
    blocks; with no frame the model is the canonical one."""

    def set_frame(self, U, blocks):
        self.U = np.asarray(U, dtype=np.float64)
        self.blocks = list(blocks)
        self.mask = pair_mask(self.n_val, self.blocks)
        self.wr = np.einsum("vj,vxyz->jxyz", self.U, self.phir)
        self._taul = None

    def set_orbitals(self, phi, eps, psi_c=None, eps_c=None):
        super().set_orbitals(phi, eps, psi_c, eps_c)
        if getattr(self, "U", None) is not None:
            self.wr = np.einsum("vj,vxyz->jxyz", self.U, self.phir)
            self._taul = None

    def tau_local(self):
        """W(w_j' w_j) for the kept pairs (zero elsewhere), [n][n][grid]."""
        if self._taul is None:
            n = self.n_val
            t = np.zeros((n, n) + self.b.grid)
            for j in range(n):
                for jp in range(j, n):
                    if self.mask[j, jp]:
                        t[j, jp] = t[jp, j] = self.apply_W(self.wr[j] * self.wr[jp])
            self._taul = t
        return self._taul

    def kernel_grid(self, ar, mask=None):
        mask = self.kmask if mask is None else mask
        if getattr(self, "U", None) is None:
            return super().kernel_grid(ar, mask)
        z = np.zeros_like(ar)
        if mask & K_1E:
            drho = (self.phir * ar).sum(0)
            z += self.spin * self.poisson(drho) * self.phir
        if mask & (K_1D_BARE | K_1D_PDEP):
            at = np.einsum("vj,vxyz->jxyz", self.U, ar)
            yt = np.einsum("ujxyz,uxyz->jxyz", self.tau_local(), at)
            z -= np.einsum("vj,jxyz->vxyz", self.U, yt)
        return z

    def sigma_grid(self, ar):
        if getattr(self, "U", None) is None:
            return super().sigma_grid(ar)
        at = np.einsum("vj,vxyz->jxyz", self.U, ar)
        gt = np.zeros_like(at)
        for j in range(self.n_val):
            ks = np.nonzero(self.mask[j])[0]
            if len(ks):
                sig = self.apply_W(at[ks] * at[j])
                gt[j] = (sig * self.wr[ks]).sum(0)
        return np.einsum("vj,jxyz->vxyz", self.U, gt)


def displaced(sys: WannierSystem, site, axis, delta, L0):
    """The pruned model at a displaced geometry: ground state re-solved, the
    frame Loewdin-aligned to the reference localised orbitals L0[n][N_pw],
    the kept blocks and W frozen."""
    xyz = sys.site_xyz.copy()
    xyz[site, axis] += delta
    d = WannierSystem(sys.b, xyz, sys.site_depth, sys.site_width, sys.pdep, sys.lam,
                      sys.n_val, scissor=sys.scissor, spin=sys.spin, kmask=sys.kmask)
    d.ground_state()
    d.set_frame(loewdin_frame(d.phi, L0), sys.blocks)
    return d


def fd_force(sys: WannierSystem, site, axis, delta, n_states=1):
    """Central difference of the lowest omega of the pruned model along one
    site coordinate (frame and kept blocks as in displaced())."""
    L0 = sys.U.T @ sys.phi
    w = []
    for sgn in (+1, -1):
        d = displaced(sys, site, axis, sgn * delta, L0)
        ww, _, info = solvers.davidson(d, n_states, tol=1e-11, max_iter=500)
        if not info["converged"]:
            raise RuntimeError("Davidson did not converge in the FD check")
        w.append(ww[0])
    return (w[0] - w[1]) / (2.0 * delta)
