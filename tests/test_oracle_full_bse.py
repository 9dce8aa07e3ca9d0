"""Pins of the BSE beyond the Tamm-Dancoff approximation (oracle/full_bse.py;
the coupled form and the coupling operators K^2e, K^2d of SM Sec. I).

* the DMPT coupling apply B = s K2e - K2d equals the conventional
  electron-hole coupling matrix built from every conduction state with
  explicit basis, DFT and W matrices, for every kernel combination;
* free-electron closed form: one constant occupied orbital and plane-wave
  PDEP pairs make A and B diagonal in plane waves, with
  A_G - B_G = T_G + W_G/Omega and A_G + B_G = T_G + 2 s v_c(G)/Omega - W_G/Omega
  (W_G = v_c(G)/(1 - lambda) on the PDEP pairs), so
  omega_G^2 = (A_G - B_G)(A_G + B_G);
* with no kernel the coupling vanishes and the roots are the TDA ones;
* the full matrix [[A, B], [-B, -A]] has its eigenvalues in +-omega pairs
  and the lowest omega lies below the lowest TDA root;
* the subspace solver reaches the dense roots, and its (X, Y) satisfy both
  block equations with X.X - Y.Y = 1.
"""
import numpy as np
import pytest

import synth
from oracle import basis, dense, full_bse, solvers
from oracle.model import K_1D_BARE, K_1D_PDEP, K_1E, K_ALL, K_D, System

from .conftest import _oracle_system


@pytest.mark.parametrize("kmask", [K_D | K_1E, K_D | K_1D_BARE, K_D | K_1D_PDEP, K_ALL])
def test_coupling_apply_equals_electron_hole_matrix(kmask):
    S, _ = _oracle_system("m0", kmask=kmask, scissor=0.1)
    A, ev, ec, psi, phi = dense.eh_matrix(S)
    S.set_orbitals(phi, ev)
    B = full_bse.dense_b(S)
    nv, nc = S.n_val, len(ec)
    C = np.random.default_rng(4).standard_normal((2, nv, nc))
    Y = full_bse.apply_b(S, C @ psi)
    Y2 = (C.reshape(2, -1) @ B.T).reshape(2, nv, nc) @ psi
    assert np.abs(Y - Y2).max() < 1e-12 * np.abs(Y2).max()


def test_free_electron_closed_form():
    cfg = synth.get_config("m0")
    b = basis.Basis(cfg.cell, cfg.grid, cfg.ecut)
    npair = 4
    P = np.zeros((b.n_pw, 2 * npair))
    lam = np.zeros(2 * npair)
    for k in range(npair):
        P[1 + 2 * k, 2 * k] = 1.0
        P[2 + 2 * k, 2 * k + 1] = 1.0
        lam[2 * k] = lam[2 * k + 1] = -0.3 * (k + 1)
    S = System(b, np.zeros((0, 3)), np.zeros(0), np.zeros(0), P, lam, 1)
    w = S.ground_state(n_extra=4)
    assert abs(w[0]) < 1e-14
    g2 = b.g2[1:]
    vc = 4 * np.pi / g2
    W = vc.copy()
    for k in range(npair):                      # basis functions 1 + 2k, 2 + 2k
        W[2 * k] = W[2 * k + 1] = vc[2 * k] / (1.0 - lam[2 * k])
    T = 0.5 * g2
    X = np.eye(b.n_pw)[1:, None, :]
    Bd = full_bse.apply_b(S, X)[:, 0, :]
    want_b = (S.spin * vc - W) / b.omega
    assert np.abs(Bd - np.diag(want_b) @ np.eye(b.n_pw)[1:]).max() < 1e-12
    om_g = np.sqrt((T + W / b.omega) * (T + 2 * S.spin * vc / b.omega - W / b.omega))
    om, Xs, Ys, info = full_bse.davidson_full(S, 2, tol=1e-10)
    assert info["converged"]
    assert np.abs(om - np.sort(om_g)[:2]).max() < 1e-10


def test_no_coupling_without_kernels():
    S, _ = _oracle_system("m0", kmask=K_D, scissor=0.2)
    om, X, Y, info = full_bse.davidson_full(S, 2, tol=1e-10)
    assert info["converged"]
    w, _, _ = solvers.davidson(S, 2, tol=1e-11)
    assert np.abs(om - w).max() < 1e-10
    assert np.abs(Y).max() < 1e-12


@pytest.fixture(scope="module")
def m0_full():
    S, _ = _oracle_system("m0", scissor=0.1)
    A, ev, ec, psi, phi = dense.eh_matrix(S)
    S.set_orbitals(phi, ev)
    B = full_bse.dense_b(S)
    return S, A, B


def test_pairing_and_below_tda(m0_full):
    S, A, B = m0_full
    om = full_bse.omega_dense(A, B)
    full = np.linalg.eigvals(np.block([[A, B], [-B, -A]])).real
    assert np.abs(np.sort(full[full > 0]) - om).max() < 1e-9
    assert np.abs(np.sort(-full[full < 0]) - om).max() < 1e-9
    assert om[0] < np.linalg.eigvalsh(A)[0]


def test_solver_reaches_the_dense_roots(m0_full):
    S, A, B = m0_full
    om_d = full_bse.omega_dense(A, B, 3)
    om, X, Y, info = full_bse.davidson_full(S, 3, tol=1e-9)
    assert info["converged"]
    assert np.abs(om - om_d).max() < 1e-10
    r1 = S.apply(X) + full_bse.apply_b(S, Y) - om[:, None, None] * X
    r2 = full_bse.apply_b(S, X) + S.apply(Y) + om[:, None, None] * Y
    assert max(np.abs(r1).max(), np.abs(r2).max()) < 1e-9
    norm = (X ** 2).sum((1, 2)) - (Y ** 2).sum((1, 2))
    assert np.abs(norm - 1).max() < 1e-12
