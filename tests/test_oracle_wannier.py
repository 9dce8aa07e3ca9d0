"""Pins of the Wannier localisation and of the pruned model (oracle/wannier.py;
the paper's Wannier-localised W integrals, main text after Eq. 7).

* the pair measure is symmetric, 1 on the diagonal, at most 1, and equals
  its definition;
* the Jacobi angle maximises the pair objective, checked against a
  brute-force search over rotations built as explicit matrices;
* the tournament visits every pair once per sweep in rounds of disjoint
  pairs;
* the spread never increases over the sweeps, U stays orthogonal, and the
  spread recomputed from scratch for the rotated orbitals equals the one the
  sweeps carried;
* closed forms: the centre of one symmetric function is its centre; mixing
  eight well separated functions by a random rotation and localising
  recovers them (up to sign and order) and their centres;
* every block kept: the operator and U equal the canonical ones (covariance);
* the pruned apply differs from the canonical one by exactly the dropped
  pairs' terms, each recomputed alone from its definition;
* the pruned operator is symmetric;
* d omega/d R of the pruned model (its U from the pruned W terms) against
  central differences with the frame and the kept blocks frozen (SM Sec. II
  protocol); the canonical U misses.
"""
import numpy as np
import pytest

import synth
from oracle import basis, solvers, wannier
from oracle.model import System


def _c1(cls=wannier.WannierSystem, **kw):
    cfg = synth.get_config("c1")
    b = basis.Basis(cfg.cell, cfg.grid, cfg.ecut)
    d = synth.make_system(cfg, b.n_pw)
    S = cls(b, d["site_xyz"], d["site_depth"], d["site_width"], d["pdep"], d["lam"],
            cfg.n_val, **kw)
    S.ground_state(n_extra=4)
    return S


@pytest.fixture(scope="module")
def c1():
    S = _c1()
    U, cen, info = wannier.localized_frame(S.b, S.phir, max_sweeps=30)
    return S, U, cen, info


# --------------------------------------------------------------------------
# localisation
# --------------------------------------------------------------------------
def test_jacobi_angle_maximises_the_pair_objective():
    rng = np.random.default_rng(5)
    n = 6
    mats = []
    for _ in range(6):
        a = rng.standard_normal((n, n))
        mats.append(a + a.T)
    wts = rng.uniform(0.5, 2.0, 6)

    def objective(i, j, th):
        R = np.eye(n)
        R[i, i] = R[j, j] = np.cos(th)
        R[j, i], R[i, j] = np.sin(th), -np.sin(th)   # column i -> c e_i + s e_j
        return sum(w * (np.diag(R.T @ A @ R)[[i, j]] ** 2).sum() for A, w in zip(mats, wts))

    grid = np.linspace(-np.pi / 2, np.pi / 2, 20001)
    for i, j in ((0, 1), (2, 5), (1, 4)):
        c, s = wannier.jacobi_angle(mats, wts, i, j)
        assert abs(c * c + s * s - 1) < 1e-14
        best = max(objective(i, j, t) for t in grid)
        got = objective(i, j, np.arctan2(s, c))
        assert got >= best - 1e-9 * abs(best)
        # the rotation routine applies the same plane rotation
        B = [A.copy() for A in mats]
        U = np.eye(n)
        wannier.rotate(B, U, i, j, c, s)
        R = U
        for A, A2 in zip(mats, B):
            assert np.abs(R.T @ A @ R - A2).max() < 1e-13


@pytest.mark.parametrize("n", [2, 7, 8, 13])
def test_tournament_covers_every_pair_once(n):
    rounds = wannier.tournament(n)
    seen = [p for r in rounds for p in r]
    assert sorted(seen) == [(i, j) for i in range(n) for j in range(i + 1, n)]
    for r in rounds:
        idx = [x for p in r for x in p]
        assert len(idx) == len(set(idx))


def test_spread_monotone_and_recomputed(c1):
    S, U, cen, info = c1
    h = np.array(info["spread"])
    assert np.all(np.diff(h) <= 1e-12 * h[0])
    assert h[-1] < 0.7 * h[0]
    assert np.abs(U.T @ U - np.eye(len(U))).max() < 1e-13
    wr = np.einsum("vj,vxyz->jxyz", U, S.phir)
    mats, wts = wannier.position_matrices(S.b, wr)
    assert abs(wannier.spread(mats, wts) - h[-1]) < 1e-10 * h[-1]
    # centres in Morton order, each inside the cell
    assert np.all((cen >= 0) & (cen < S.b.cell[None, :]))


def _gaussian_set(b, centres, width):
    out = []
    for c in centres:
        d2 = 0
        for k in range(3):
            x = np.arange(b.grid[k]) * b.cell[k] / b.grid[k] - c[k]
            x = x - b.cell[k] * np.round(x / b.cell[k])          # minimum image
            shape = [1, 1, 1]
            shape[k] = b.grid[k]
            d2 = d2 + (x * x).reshape(shape)
        out.append(b.from_grid(np.exp(-0.5 * d2 / width ** 2)))
    return np.array(out)


def test_centre_of_a_symmetric_function():
    b = basis.Basis((12.0, 14.0, 16.0), (24, 28, 32), 8.0)
    c0 = np.array([3.1, 9.7, 12.4])
    f = _gaussian_set(b, [c0], 1.1)
    f /= np.linalg.norm(f)
    mats, _ = wannier.position_matrices(b, b.to_grid(f))
    assert np.abs(wannier.centres(b, mats)[0] - c0).max() < 1e-9


def test_recovers_mixed_separated_functions():
    L = 16.0
    b = basis.Basis((L, L, L), (32, 32, 32), 6.0)
    cs = np.array([[x, y, z] for x in (L / 4, 3 * L / 4) for y in (L / 4, 3 * L / 4)
                   for z in (L / 4, 3 * L / 4)])
    F = _gaussian_set(b, cs, 1.0)
    w, V = np.linalg.eigh(F @ F.T)
    F = (V * (1 / np.sqrt(w))) @ V.T @ F                     # Loewdin orthonormal
    mats0, wts = wannier.position_matrices(b, b.to_grid(F))
    s0 = wannier.spread(mats0, wts)
    Q, _ = np.linalg.qr(np.random.default_rng(2).standard_normal((8, 8)))
    mixed = Q.T @ F
    U, cen, info = wannier.localized_frame(b, b.to_grid(mixed), max_sweeps=50)
    got = U.T @ mixed
    ov = np.abs(got @ F.T)
    assert np.all(ov.max(1) > 0.999999)
    assert sorted(ov.argmax(1)) == list(range(8))
    assert info["spread"][-1] <= s0 * (1 + 1e-9)
    for j in range(8):
        assert np.abs(cen[j] - cs[ov[j].argmax()]).max() < 1e-6
    assert info["spread"][0] > 1.5 * s0


def test_pair_measure_bounds(c1):
    """The pair measure is symmetric, 1 on the diagonal and at most 1
    (Cauchy-Schwarz), and equals its definition for one pair computed
    directly on the grid."""
    S, U, cen, info = c1
    wr = np.einsum("vj,vxyz->jxyz", U, S.phir)
    s = wannier.pair_measure(S.b, wr)
    assert np.abs(s - s.T).max() < 1e-15
    assert np.abs(np.diag(s) - 1).max() < 1e-14 and s.max() <= 1 + 1e-14
    j, jp = 2, 11
    num = np.sqrt(((wr[j] * wr[jp]) ** 2).sum())
    den = np.sqrt(np.sqrt((wr[j] ** 4).sum()) * np.sqrt((wr[jp] ** 4).sum()))
    assert abs(s[j, jp] - num / den) < 1e-14


# --------------------------------------------------------------------------
# pruned model
# --------------------------------------------------------------------------
def _trial(S, nb=2, seed=11):
    return S.proj_c(np.random.default_rng(seed).standard_normal((nb,) + S.phi.shape))


def test_every_block_kept_is_the_canonical_model(c1):
    S, U, cen, info = c1
    n = S.n_val
    nb = (n + 7) // 8
    C = System(S.b, S.site_xyz, S.site_depth, S.site_width, S.pdep, S.lam, n)
    C.set_orbitals(S.phi, S.eps)
    S.set_frame(U, [(I, J) for I in range(nb) for J in range(I, nb)])
    X = _trial(S)
    Yc, Yw = C.apply(X), S.apply(X)
    assert np.abs(Yw - Yc).max() < 1e-12 * np.abs(Yc).max()
    A = X[0] / np.linalg.norm(X[0])
    uc, uw = solvers.u_vector(C, A), solvers.u_vector(S, A)
    assert np.abs(uw - uc).max() < 1e-12 * np.abs(uc).max()


def test_pruned_apply_is_canonical_minus_the_dropped_pairs(c1):
    S, U, cen, info = c1
    n = S.n_val
    C = System(S.b, S.site_xyz, S.site_depth, S.site_width, S.pdep, S.lam, n)
    C.set_orbitals(S.phi, S.eps)
    S.set_frame(U, [(0, 0), (1, 1)])                      # block (0, 1) dropped
    X = _trial(S, nb=1)[0]
    A = S.proj_c(X)
    ar = S.b.to_grid(A)
    at = np.einsum("vj,vxyz->jxyz", U, ar)
    wr = np.einsum("vj,vxyz->jxyz", U, S.phir)
    add = np.zeros_like(at)
    for j in range(8):
        for jp in range(8, 16):
            # pair (j, j') and (j', j), each term alone from Eq. 2c
            add[j] += S.apply_W(wr[jp] * wr[j]) * at[jp]
            add[jp] += S.apply_W(wr[j] * wr[jp]) * at[j]
    back = np.einsum("vj,jxyz->vxyz", U, add)
    want = C.apply(X) + S.proj_c(S.b.from_grid(back))
    got = S.apply(X)
    assert np.abs(got - want).max() < 1e-12 * np.abs(want).max()
    assert np.abs(got - C.apply(X)).max() > 1e-6 * np.abs(want).max()


def test_pruned_operator_symmetric(c1):
    S, U, cen, info = c1
    S.set_frame(U, [(0, 0), (1, 1)])
    X, Y = _trial(S, nb=2, seed=3)
    a = (Y * S.apply(X)).sum()
    b_ = (X * S.apply(Y)).sum()
    assert abs(a - b_) < 1e-12 * max(1.0, abs(a))


def test_pruned_forces_match_central_differences(c1):
    """Analytic d omega/d R of the pruned model (Eqs. 4-7 with the pruned
    K1d in the operator and the pruned W term in U) against Richardson-
    extrapolated central differences of its omega, the frame Loewdin-aligned
    at each displaced geometry and the kept blocks frozen."""
    S0, U, cen, info = c1
    S = _c1()
    S.set_frame(U, [(0, 0), (1, 1)])
    w, X, dinfo = solvers.davidson(S, 1, tol=1e-11, max_iter=400)
    assert dinfo["converged"]
    A = X[0]
    Z, zi = solvers.zvector_cg(S, solvers.u_vector(S, A), tol=1e-12)
    assert zi["converged"]
    F = solvers.dwdR(S, A, Z)
    # the canonical U (unpruned W term) misses
    C = System(S.b, S.site_xyz, S.site_depth, S.site_width, S.pdep, S.lam, S.n_val)
    C.set_orbitals(S.phi, S.eps)
    Zc, _ = solvers.zvector_cg(S, solvers.u_vector(C, A), tol=1e-12)
    Fc = solvers.dwdR(S, A, Zc)
    d = 0.006742
    worst, worst_c = 0.0, 0.0
    for site, ax in ((0, 0), (3, 2)):
        f1 = wannier.fd_force(S, site, ax, d)
        f2 = wannier.fd_force(S, site, ax, d / 2)
        fd = (4 * f2 - f1) / 3
        worst = max(worst, abs(fd - F[site, ax]))
        worst_c = max(worst_c, abs(fd - Fc[site, ax]))
    print(f"pruned: max |F - FD| {worst:.2e}; canonical U {worst_c:.2e}; max |F| "
          f"{np.abs(F).max():.2e}")
    assert worst < 1e-6
    assert worst_c > 20 * worst
