"""Host logic of the relaxation driver: BFGS on closed-form functions, and a
ground-state relaxation of the tiny system with the oracle as the evaluator
(every number the driver sees is the oracle's)."""
import numpy as np
import pytest

import synth
from oracle import basis, model, solvers
from paper_2607_20728_amd import relax


def test_bfgs_quadratic_and_rosenbrock():
    rng = np.random.default_rng(3)
    M = rng.standard_normal((6, 6))
    A = M @ M.T + 6 * np.eye(6)
    b = rng.standard_normal(6)
    x, f, g, hist = relax.bfgs(lambda x: (0.5 * x @ A @ x - b @ x, A @ x - b), np.zeros(6),
                               gtol=1e-10, max_steps=100, max_step=10.0)
    assert np.abs(x - np.linalg.solve(A, b)).max() < 1e-8
    assert all(h1[0] <= h0[0] + 1e-15 for h0, h1 in zip(hist, hist[1:]))

    def rosen(x):
        f = 100 * (x[1] - x[0] ** 2) ** 2 + (1 - x[0]) ** 2
        g = np.array([-400 * x[0] * (x[1] - x[0] ** 2) - 2 * (1 - x[0]), 200 * (x[1] - x[0] ** 2)])
        return f, g

    x, f, g, hist = relax.bfgs(rosen, np.array([-1.2, 1.0]), gtol=1e-8, max_steps=500,
                               max_step=0.5)
    assert np.abs(x - 1.0).max() < 1e-6


def test_delta_q():
    a = np.zeros((3, 3))
    b = np.array([[1.0, 0, 0], [0, 2.0, 0], [0, 0, 0]])
    assert relax.delta_q(a, b) == pytest.approx(np.sqrt(5.0))
    assert relax.delta_q(a, b, masses=[4.0, 1.0, 7.0]) == pytest.approx(np.sqrt(8.0))


def _oracle_evaluator(cfg, b):
    def ev(sysd, xyz, *, surface="gs", spring=5.0, f_occ=2.0):
        S = model.System(b, np.asarray(xyz), sysd["site_depth"], sysd["site_width"],
                         sysd["pdep"], sysd["lam"], cfg.n_val)
        S.ground_state(n_extra=8)
        x0 = np.asarray(sysd["site_xyz"])
        E = f_occ * S.eps.sum() + 0.5 * spring * np.sum((xyz - x0) ** 2)
        G = f_occ * solvers.hf_ground_forces(S) + spring * (xyz - x0)
        if surface == "es":
            w, X, _ = solvers.davidson(S, 1, tol=1e-10)
            Z, _ = solvers.zvector_cg(S, solvers.u_vector(S, X[0]), tol=1e-10)
            E += w[0]
            G = G + solvers.dwdR(S, X[0], Z)
        return E, G
    return ev


def test_ground_state_relaxation_with_the_oracle():
    """Relaxed on E_GS, the sites sit where the spring balances the
    Hellmann-Feynman force: the gradient vanishes, the energy fell, and the
    minimum is a minimum along a random direction."""
    cfg = synth.get_config("m0")
    b = basis.Basis(cfg.cell, cfg.grid, cfg.ecut)
    d = synth.make_system(cfg, b.n_pw, n_trial=1)
    ev = _oracle_evaluator(cfg, b)
    xyz, E, hist = relax.relax(d, surface="gs", evaluator=ev, gtol=1e-6, max_steps=60)
    assert hist[-1][1] < 1e-6
    assert E < hist[0][0] - 1e-4
    assert all(h1[0] <= h0[0] + 1e-12 for h0, h1 in zip(hist, hist[1:]))
    u = np.random.default_rng(5).standard_normal(xyz.shape)
    u /= np.linalg.norm(u)
    for h in (0.02, -0.02):
        assert ev(d, xyz + h * u)[0] > E
    assert relax.delta_q(xyz, d["site_xyz"]) > 1e-3


def test_excited_state_relaxation_with_the_oracle():
    """Both minima of the tiny system with the oracle as the evaluator: the
    excited-state minimum differs from the ground-state one (Delta Q > 0)
    and each is a stationary point of its own surface only."""
    cfg = synth.get_config("m0")
    b = basis.Basis(cfg.cell, cfg.grid, cfg.ecut)
    d = synth.make_system(cfg, b.n_pw, n_trial=1)
    ev = _oracle_evaluator(cfg, b)
    xg, _, hg = relax.relax(d, surface="gs", evaluator=ev, gtol=1e-6, max_steps=60)
    xe, _, he = relax.relax(d, surface="es", evaluator=ev, gtol=1e-6, max_steps=60)
    assert hg[-1][1] < 1e-6 and he[-1][1] < 1e-6
    assert all(h1[0] <= h0[0] + 1e-12 for h0, h1 in zip(he, he[1:]))
    assert relax.delta_q(xg, xe) > 1e-3
    assert np.abs(ev(d, xg, surface="es")[1]).max() > 1e-4   # not a minimum of E_ES
