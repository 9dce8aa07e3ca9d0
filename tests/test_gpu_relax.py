"""Excited-state relaxation through the library (GPU): the composed energy
and gradient against the oracle at a displaced geometry, the gradient
against a central difference of the library's own energies, and a BFGS run
on both surfaces of the tiny system; warm-started solves along a path."""
import numpy as np
import pytest

import synth
from oracle import basis, model, solvers

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2607_20728_amd import relax  # noqa: E402


def _system(name="m0"):
    cfg = synth.get_config(name)
    b = basis.Basis(cfg.cell, cfg.grid, cfg.ecut)
    return cfg, b, synth.make_system(cfg, b.n_pw, n_trial=1)


def test_excited_state_energy_and_gradient_vs_oracle():
    print("[gpu] relax: E_ES and gradient vs oracle (m0)", flush=True)
    cfg, b, d = _system()
    rng = np.random.default_rng(11)
    xyz = np.asarray(d["site_xyz"]) + 0.05 * rng.standard_normal(np.shape(d["site_xyz"]))
    E, G = relax.evaluate(d, xyz, surface="es", tol=1e-11)
    S = model.System(b, xyz, d["site_depth"], d["site_width"], d["pdep"], d["lam"], cfg.n_val)
    S.ground_state(n_extra=8)
    w, X, _ = solvers.davidson(S, 1, tol=1e-11)
    Z, _ = solvers.zvector_cg(S, solvers.u_vector(S, X[0]), tol=1e-12)
    dx = xyz - np.asarray(d["site_xyz"])
    Eo = 2.0 * S.eps.sum() + 2.5 * np.sum(dx ** 2) + w[0]
    Go = 2.0 * solvers.hf_ground_forces(S) + 5.0 * dx + solvers.dwdR(S, X[0], Z)
    assert abs(E - Eo) < 1e-9
    assert np.abs(G - Go).max() < 1e-7


def test_gradient_matches_central_difference_of_library_energies():
    print("[gpu] relax: gradient vs central difference (m0)", flush=True)
    cfg, b, d = _system()
    xyz = np.asarray(d["site_xyz"], dtype=float)
    _, G = relax.evaluate(d, xyz, surface="es", tol=1e-11)
    u = np.random.default_rng(2).standard_normal(xyz.shape)
    u /= np.linalg.norm(u)
    def cd(h):
        Ep, _ = relax.evaluate(d, xyz + h * u, surface="es", tol=1e-11)
        Em, _ = relax.evaluate(d, xyz - h * u, surface="es", tol=1e-11)
        return (Ep - Em) / (2 * h)

    h = 2e-3
    fd = (4 * cd(h / 2) - cd(h)) / 3  # Richardson: O(h^4)
    assert abs(fd - np.sum(G * u)) < 1e-6 * max(1.0, abs(fd))


def test_relaxation_on_both_surfaces():
    print("[gpu] relax: BFGS on the ground- and excited-state surfaces (m0)", flush=True)
    cfg, b, d = _system()
    out = {}
    for surface in ("gs", "es"):
        xyz, E, hist = relax.relax(d, surface=surface, gtol=1e-5, max_steps=40)
        assert hist[-1][1] < 1e-5, (surface, hist[-1])
        assert all(h1[0] <= h0[0] + 1e-10 for h0, h1 in zip(hist, hist[1:])), surface
        out[surface] = (xyz, E, len(hist))
    dq = relax.delta_q(out["gs"][0], out["es"][0])
    print(f"  steps gs {out['gs'][2]} es {out['es'][2]}; Delta Q (unit masses) {dq:.4f} bohr")
    assert dq > 1e-4


def test_warm_start_reaches_the_cold_result_in_fewer_iterations():
    """Along a relaxation path (C1), each geometry's solves started from the
    previous geometry's exciton and Z give the energy and gradient of a cold
    solve, in fewer Davidson and Z-vector iterations."""
    print("[gpu] relax: warm-started solves along a path (c1)", flush=True)
    cfg, b, d = _system("c1")
    x0 = np.asarray(d["site_xyz"], dtype=float)
    u = np.random.default_rng(5).standard_normal(x0.shape)
    u *= 0.02 / np.abs(u).max()
    warm, cold = dict(warm=True), dict(warm=False)
    worst_e, worst_g = 0.0, 0.0
    for k in range(4):
        xyz = x0 + k * u
        Ew, Gw = relax.evaluate(d, xyz, surface="es", tol=1e-10, state=warm)
        Ec, Gc = relax.evaluate(d, xyz, surface="es", tol=1e-10, state=cold)
        worst_e = max(worst_e, abs(Ew - Ec))
        worst_g = max(worst_g, np.abs(Gw - Gc).max())
    print(f"  |dE| {worst_e:.1e}  |dG| {worst_g:.1e}  Davidson {warm['davidson_iters']} vs "
          f"{cold['davidson_iters']}, Z {warm['zvector_iters']} vs {cold['zvector_iters']}",
          flush=True)
    assert worst_e < 1e-9 and worst_g < 1e-7
    assert warm["davidson_iters"] < cold["davidson_iters"]
    assert warm["zvector_iters"] < cold["zvector_iters"]
