"""Pins of the FP64 oracle against results the paper and the mathematics fix.

* free-electron closed form (V = 0, one occupied orbital): the operator is
  diagonal in plane waves with eigenvalue |G|^2/2 + s 4 pi/(Omega |G|^2)
  (Eq. 2b with a constant occupied orbital; K1d vanishes because the pair
  density is constant and v_c(0) = 0, PDEP has no G = 0 row);
* the semilocal-TDDFT-like special case of Table S-I with f = 0 (W = 0,
  no K1e): eigenvalues are exactly eps_c - eps_v + Delta;
* PDEP vectors chosen as plane-wave pairs with equal lambda: W is diagonal
  in G with W(G) = v_c(G)/(1 - lambda) (Eq. 3 closed form);
* the DMPT apply equals the conventional electron-hole matrix with every
  conduction state (the exact equivalence the formulation rests on), for
  every kernel combination;
* symmetry of the operator; Davidson eigenvalues against dense eigh;
* U against a directional finite difference of A^T M(phi) A (SM Sec. I);
* Z-vector CG against the dense sum over states (Eq. 7 with the KS kernels
  zero for the synthetic Hamiltonian);
* analytic d omega/d R against central finite differences with W frozen
  (SM Sec. II protocol), translational invariance, zero-trace densities;
* the ground-state Hellmann-Feynman derivative of the occupied eigenvalue
  sum against central finite differences.
"""
import numpy as np
import pytest

import synth
from oracle import basis, dense, model, solvers
from oracle.model import K_1D_BARE, K_1D_PDEP, K_1E, K_ALL, K_D, System

from .conftest import _oracle_system


def _m0_basis():
    cfg = synth.get_config("m0")
    return cfg, basis.Basis(cfg.cell, cfg.grid, cfg.ecut)


# --------------------------------------------------------------------------
# closed forms
# --------------------------------------------------------------------------
def test_free_electron_closed_form():
    cfg, b = _m0_basis()
    d = synth.make_system(cfg, b.n_pw)
    S = System(b, np.zeros((0, 3)), np.zeros(0), np.zeros(0), d["pdep"], d["lam"], 1)
    w = S.ground_state(n_extra=4)
    assert abs(w[0]) < 1e-14
    X = np.eye(b.n_pw)[1:, None, :]                    # every plane wave but G = 0
    Y = S.apply(X)[:, 0, :]
    lam = 0.5 * b.g2[1:] + 2 * 4 * np.pi / (b.omega * b.g2[1:])
    assert np.abs(Y - np.diag(lam) @ np.eye(b.n_pw)[1:]).max() < 1e-12
    om, _, info = solvers.davidson(S, n_states=2, tol=1e-11)
    assert np.allclose(om, np.sort(lam)[:2], atol=1e-10)


def test_no_kernel_gives_bare_transitions():
    S, _ = _oracle_system("m0", kmask=K_D, scissor=0.3)
    nv = S.n_val
    de = np.sort((S.eps_all[nv:][None, :] - S.eps_all[:nv][:, None]).reshape(-1)) + 0.3
    om, _, info = solvers.davidson(S, n_states=3, tol=1e-11)
    assert info["converged"]
    assert np.abs(om - de[:3]).max() < 1e-10


def test_diagonal_pdep_closed_form():
    cfg, b = _m0_basis()
    npair = 4
    P = np.zeros((b.n_pw, 2 * npair))
    lam = np.zeros(2 * npair)
    for k in range(npair):
        P[1 + 2 * k, 2 * k] = 1.0
        P[2 + 2 * k, 2 * k + 1] = 1.0
        lam[2 * k] = lam[2 * k + 1] = -0.3 * (k + 1)
    d = synth.make_system(cfg, b.n_pw)
    S = System(b, d["site_xyz"], d["site_depth"], d["site_width"], P, lam, 4)
    rho = np.random.default_rng(5).standard_normal(b.grid)
    got = S.apply_W(rho)
    G = np.fft.fftn(rho) / b.n_r
    fac = np.ones(b.grid)
    for k in range(npair):
        fac[tuple(b.mill_half[k] % np.array(b.grid))] = 1.0 / (1.0 - lam[2 * k])
        fac[tuple((-b.mill_half[k]) % np.array(b.grid))] = 1.0 / (1.0 - lam[2 * k])
    want = (np.fft.ifftn(G * S.vc * fac) * b.n_r).real
    assert np.abs(got - want).max() < 1e-12 * np.abs(want).max()


# --------------------------------------------------------------------------
# DMPT apply == electron-hole matrix
# --------------------------------------------------------------------------
@pytest.mark.parametrize("kmask", [K_D | K_1E, K_D | K_1D_BARE, K_D | K_1D_PDEP, K_ALL])
def test_apply_equals_electron_hole_matrix(kmask):
    S, _ = _oracle_system("m0", kmask=kmask, scissor=0.1)
    A, ev, ec, psi, phi = dense.eh_matrix(S)
    S.set_orbitals(phi, ev)
    nv, nc = S.n_val, len(ec)
    C = np.random.default_rng(1).standard_normal((2, nv, nc))
    Y = S.apply(C @ psi)
    Y2 = (C.reshape(2, -1) @ A.T).reshape(2, nv, nc) @ psi
    assert np.abs(Y - Y2).max() < 1e-12 * np.abs(Y2).max()


def test_davidson_matches_dense_eigh(m0_solved):
    S = m0_solved["S"]
    A, *_ = dense.eh_matrix(S)
    w = np.linalg.eigvalsh(A)
    assert np.abs(m0_solved["omega"] - w[:3]).max() < 1e-10


def test_operator_symmetric(c1_solved):
    S = c1_solved["S"]
    rng = np.random.default_rng(7)
    X = rng.standard_normal((2, S.n_val, S.b.n_pw))
    MX = S.apply(X)
    a, b_ = (X[1] * MX[0]).sum(), (X[0] * MX[1]).sum()
    assert abs(a - b_) < 1e-13 * np.abs(MX).sum() / np.sqrt(MX.size)
    assert np.abs(S.apply(S.proj_c(X) - X)).max() < 1e-12 * np.abs(MX).max()


def test_normalisation_and_orthogonality(m0_solved):
    S, X = m0_solved["S"], m0_solved["X"]
    assert abs((X[0] ** 2).sum() - 1) < 1e-12
    assert np.abs(X[0] @ S.phi.T).max() < 1e-12


# --------------------------------------------------------------------------
# U, Z, forces
# --------------------------------------------------------------------------
def test_u_directional_derivative(m0_solved):
    """dE/d eta along phi -> phi + eta dphi (dphi in P_c, eps fixed) equals
    2 sum_v <dphi_v|u_v> with E = A^T P_c M(phi) P_c A."""
    S, A, U = m0_solved["S"], m0_solved["X"][0], m0_solved["U"]
    dphi = S.proj_c(np.random.default_rng(9).standard_normal(S.phi.shape))
    phi0, eps0 = S.phi.copy(), S.eps.copy()

    def energy(eta):
        S.set_orbitals(phi0 + eta * dphi, eps0)
        return (A * S.apply(A)).sum()

    h = 1e-4
    fd = (energy(h) - energy(-h)) / (2 * h)
    fd2 = (energy(h / 2) - energy(-h / 2)) / h
    S.set_orbitals(phi0, eps0)
    rich = (4 * fd2 - fd) / 3
    want = 2 * (dphi * U).sum()
    assert abs(rich - want) < 1e-9 * max(1.0, abs(want))


def test_zvector_cg_matches_sum_over_states(m0_solved, c1_solved):
    for sol, tol in ((m0_solved, 1e-10), (c1_solved, 1e-6)):
        S = sol["S"]
        Zs = solvers.zvector_sos(S, sol["U"])
        assert np.abs(sol["Z"] - Zs).max() < tol * np.abs(Zs).max()
        R = solvers.apply_DKS(S, sol["Z"]) + sol["U"]
        assert np.linalg.norm(R) / np.linalg.norm(sol["U"]) < (1e-12 if sol is m0_solved else 1e-8)
        assert np.abs(sol["Z"] @ S.phi.T).max() < 1e-12


def test_densities_trace_zero(m0_solved):
    S = m0_solved["S"]
    rx, rz = solvers.densities(S, m0_solved["X"][0], m0_solved["Z"])
    q = S.b.omega / S.b.n_r
    assert abs(q * rx.sum()) < 1e-12 and abs(q * rz.sum()) < 1e-12


def test_forces_match_finite_difference_m0(m0_solved):
    S = m0_solved["S"]
    F = solvers.dwdR(S, m0_solved["X"][0], m0_solved["Z"])
    h = 0.006742                                   # 0.003568 Angstrom (SM Sec. II)
    for site in range(S.n_sites):
        for ax in range(3):
            f1 = solvers.fd_force(S, site, ax, h)
            f2 = solvers.fd_force(S, site, ax, h / 2)
            rich = (4 * f2 - f1) / 3
            assert abs(F[site, ax] - f1) < 1e-5
            assert abs(F[site, ax] - rich) < 1e-7


def test_forces_match_finite_difference_c1(c1_solved):
    S = c1_solved["S"]
    F = solvers.dwdR(S, c1_solved["X"][0], c1_solved["Z"])
    h = 0.006742
    for site, ax in ((0, 0), (3, 2)):
        fd = solvers.fd_force(S, site, ax, h, method="davidson")
        assert abs(F[site, ax] - fd) < 1e-5


def test_hellmann_feynman_ground_forces_m0(m0_solved):
    """d(sum_v eps_v)/dR = sum_v <phi_v|dV/dR|phi_v> (Hellmann-Feynman for the
    occupied eigenvalues of H(R)) against central differences of the
    occupied eigenvalue sum, Richardson-extrapolated."""
    S = m0_solved["S"]
    F = solvers.hf_ground_forces(S)

    def eps_sum(site, ax, d):
        T = solvers.displaced(S, site, ax, d)
        T.ground_state()
        return T.eps.sum()

    h = 0.006742
    for site, ax in ((0, 0), (2, 1), (S.n_sites - 1, 2)):
        f1 = (eps_sum(site, ax, h) - eps_sum(site, ax, -h)) / (2 * h)
        f2 = (eps_sum(site, ax, h / 2) - eps_sum(site, ax, -h / 2)) / h
        rich = (4 * f2 - f1) / 3
        assert abs(F[site, ax]) > 1e-3
        assert abs(F[site, ax] - rich) < 1e-7, (site, ax, F[site, ax], rich)


@pytest.mark.parametrize("diag_pdep", [False, True])
def test_translational_invariance(diag_pdep):
    """With an alias-free grid (N >= 4 n_max + 1) and a translation-invariant W
    the sum of d omega/d R over all sites vanishes.  A random PDEP basis is not
    translation invariant, so it is replaced by plane-wave pairs or dropped."""
    cfg = synth.get_config("m0")
    b = basis.Basis(cfg.cell, (16, 16, 16), cfg.ecut)
    d = synth.make_system(cfg, b.n_pw)
    if diag_pdep:
        P = np.zeros((b.n_pw, 6))
        for k in range(3):
            P[1 + 2 * k, 2 * k] = P[2 + 2 * k, 2 * k + 1] = 1.0
        lam = np.repeat([-0.5, -0.4, -0.3], 2)
        mask = K_ALL
    else:
        P, lam, mask = d["pdep"], d["lam"], K_D | K_1E | K_1D_BARE
    S = System(b, d["site_xyz"], d["site_depth"], d["site_width"], P, lam, cfg.n_val,
               kmask=mask)
    S.ground_state(n_extra=8)
    om, X, info = solvers.davidson(S, n_states=1, tol=1e-11)
    U = solvers.u_vector(S, X[0])
    Z, _ = solvers.zvector_cg(S, U, tol=1e-12)
    F = solvers.dwdR(S, X[0], Z)
    assert np.abs(F).max() > 1e-3
    assert np.abs(F.sum(0)).max() < 1e-9


# --------------------------------------------------------------------------
# the band-subset apply used for parity at full size
# --------------------------------------------------------------------------
@pytest.mark.parametrize("kmask", [K_D, K_D | K_1E, K_D | K_1D_BARE | K_1D_PDEP, K_ALL])
def test_band_subset_apply_equals_rows_of_full_apply(kmask):
    """apply_bands builds tau only for the requested output bands; its rows
    equal the full apply's, with ground-state and with made-up orbitals."""
    for name in ("m0", "c1"):
        S, d = _oracle_system(name, kmask=kmask, scissor=0.05)
        rng = np.random.default_rng(5)
        X = rng.standard_normal((3, S.n_val, S.b.n_pw))
        bands = [0, S.n_val // 2, S.n_val - 1]
        Yf = S.apply(X)[:, bands]
        Yb = S.apply_bands(X, bands)
        assert np.abs(Yb - Yf).max() < 1e-13 * np.abs(Yf).max(), name
    phi, eps = synth.random_orbitals(S.b.n_pw, S.n_val, 4, seed=9)
    S.set_orbitals(phi[:S.n_val], eps[:S.n_val])
    assert np.abs(phi @ phi.T - np.eye(len(phi))).max() < 1e-13
    Yf = S.apply(X)[:, bands]
    assert np.abs(S.apply_bands(X, bands) - Yf).max() < 1e-13 * np.abs(Yf).max()
