"""Pins of the self-consistent synthetic KS model and of the KS response
kernels of the Z-vector equation (oracle/ks.py; Eq. 7 and SM Sec. I).

* f_xc against a central difference quotient of V_xc;
* closed form: a uniform system (no sites) with one occupied constant orbital
  has rho = 2/Omega, V_H = 0, V_xc constant, and (K_x e_G) = v_c(G)/Omega e_G,
  so every plane wave is an eigenvector of H_KS with |G|^2/2 + V_xc(2/Omega)
  - alpha 4 pi/(Omega |G|^2) (G != 0) or V_xc(2/Omega) (G = 0);
* the SCF solution solves H[rho(phi)] phi_v = eps_v phi_v;
* U (with its D part) against a directional derivative of A^T M(phi) A with
  H_KS, eps_vv' = <phi_v|H_KS|phi_v'>, P_c and the kernels all rebuilt from the
  displaced orbitals;
* the Z-vector operator is symmetric, and CG reaches the dense solution;
* d omega/d R against central differences of omega with the ground state
  re-converged at each displaced geometry (W frozen, SM Sec. II protocol),
  for alpha = 0 (Hartree + local xc) and alpha = 0.3 (a hybrid starting point);
  the same derivative with the kernels left out of U and Z misses.
"""
import numpy as np
import pytest

import synth
from oracle import basis, ks, solvers
from oracle.model import K_ALL


def _m0_ks(alpha=0.0, seed=None):
    cfg = synth.get_config("m0")
    b = basis.Basis(cfg.cell, cfg.grid, cfg.ecut)
    d = synth.make_system(cfg, b.n_pw, seed=seed)
    S = ks.KSSystem(b, d["site_xyz"], d["site_depth"], d["site_width"], d["pdep"], d["lam"],
                    cfg.n_val, alpha=alpha, kmask=K_ALL)
    S.ground_state(n_extra=8)
    return S, d


def test_fxc_is_the_derivative_of_vxc():
    cfg = synth.get_config("m0")
    b = basis.Basis(cfg.cell, cfg.grid, cfg.ecut)
    S = ks.KSSystem(b, np.zeros((0, 3)), np.zeros(0), np.zeros(0), np.zeros((b.n_pw, 1)),
                    np.zeros(1), 1)
    rho = np.linspace(0.0, 0.5, 101)
    h = 1e-5

    def cd(hh):
        return (S.v_xc(rho + hh) - S.v_xc(rho - hh)) / (2 * hh)
    fd = (4 * cd(h / 2) - cd(h)) / 3
    assert np.abs(fd / S.f_xc(rho) - 1).max() < 1e-8


@pytest.mark.parametrize("alpha", [0.0, 0.4])
def test_uniform_closed_form(alpha):
    cfg = synth.get_config("m0")
    b = basis.Basis(cfg.cell, cfg.grid, cfg.ecut)
    d = synth.make_system(cfg, b.n_pw)
    S = ks.KSSystem(b, np.zeros((0, 3)), np.zeros(0), np.zeros(0), d["pdep"], d["lam"], 1,
                    alpha=alpha)
    w = S.ground_state(n_extra=4)
    vxc = S.v_xc(np.array(2.0 / b.omega))
    g2 = b.g2
    want = np.where(g2 > 0, 0.5 * g2 + vxc - alpha * 4 * np.pi / (b.omega * np.where(g2 > 0, g2, 1)),
                    vxc)
    assert np.abs(np.sort(w) - np.sort(want)).max() < 1e-11
    assert abs(S.eps[0] - vxc) < 1e-12


@pytest.mark.parametrize("alpha", [0.0, 0.3])
def test_scf_solves_the_ks_equations(alpha):
    S, _ = _m0_ks(alpha)
    assert S.scf_residual() < 1e-10
    # the ground-state potential is the Hartree-xc potential of its own density
    rho = S.density(S.b.to_grid(S.phi))
    assert np.abs(S.Vr - S.Vext - S.v_hxc(rho)).max() < 1e-10
    assert S.eps_all[S.n_val] - S.eps_all[S.n_val - 1] > 1e-2


def _solved(alpha):
    S, d = _m0_ks(alpha)
    w, X, info = solvers.davidson(S, 1, tol=1e-11, max_iter=400)
    assert info["converged"]
    A = X[0]
    U = ks.u_vector(S, A)
    Z, zi = ks.zvector_cg(S, U, tol=1e-12)
    assert zi["converged"]
    return S, A, U, Z, w[0]


@pytest.fixture(scope="module", params=[0.0, 0.3])
def ks_solved(request):
    return (request.param,) + _solved(request.param)


def test_u_directional_derivative_with_hamiltonian_rebuilt(ks_solved):
    alpha, S, A, U, Z, _ = ks_solved
    dphi = S.proj_c(np.random.default_rng(13).standard_normal(S.phi.shape))
    phi0, eps0, V0, gs0 = S.phi.copy(), S.eps.copy(), S.Vr.copy(), S.phir_gs

    def energy(eta):
        phi = phi0 + eta * dphi
        phir = S.b.to_grid(phi)
        S.Vr = S.Vext + S.v_hxc(S.density(phir))
        S.set_orbitals(phi, eps0)
        S.phir_gs = S.phir
        PA = S.proj_c(A)
        E = (A * S.apply(A)).sum()
        H = S.apply_H(phi)
        epm = phi @ H.T                                  # eps_vv' = <phi_v|H|phi_v'>
        G = PA @ PA.T
        return E + (eps0 * np.diag(G)).sum() - (epm * G).sum()

    h = 1e-4
    fd = (energy(h) - energy(-h)) / (2 * h)
    fd2 = (energy(h / 2) - energy(-h / 2)) / h
    S.Vr = V0
    S.set_orbitals(phi0, eps0)
    S.phir_gs = gs0
    rich = (4 * fd2 - fd) / 3
    want = 2 * (dphi * U).sum()
    assert abs(rich - want) < 1e-8 * max(1.0, abs(want)), (rich, want)
    # the D part is not small: leaving it out misses
    bare = 2 * (dphi * solvers.u_vector(S, A)).sum()
    assert abs(bare - want) > 1e-4 * abs(want)


def test_zvector_operator_symmetric_and_dense_solve(ks_solved):
    alpha, S, A, U, Z, _ = ks_solved
    rng = np.random.default_rng(3)
    X = S.proj_c(rng.standard_normal(S.phi.shape))
    Y = S.proj_c(rng.standard_normal(S.phi.shape))
    a = (Y * ks.apply_zop(S, X)).sum()
    b_ = (X * ks.apply_zop(S, Y)).sum()
    assert abs(a - b_) < 1e-12 * max(abs(a), 1.0)
    # dense operator on the P_c space: Q^T op Q z = -Q^T u
    n = S.phi.size
    basisP = []
    for k in range(n):
        e = np.zeros(n)
        e[k] = 1.0
        basisP.append(S.proj_c(e.reshape(S.phi.shape)).reshape(-1))
    Bm = np.array(basisP).T                              # columns P_c e_k
    Q, r = np.linalg.qr(Bm)
    keep = np.abs(np.diag(r)) > 1e-8
    Q = Q[:, keep]
    M = np.array([ks.apply_zop(S, q.reshape(S.phi.shape)).reshape(-1) for q in Q.T]).T
    Ms = Q.T @ M
    assert np.abs(Ms - Ms.T).max() < 1e-10
    assert np.linalg.eigvalsh(0.5 * (Ms + Ms.T)).min() > 0
    zd = Q @ np.linalg.solve(Ms, -Q.T @ U.reshape(-1))
    assert np.abs(Z.reshape(-1) - zd).max() < 1e-9 * np.abs(zd).max()


def test_forces_match_central_differences_of_the_scf_energy(ks_solved):
    """d omega/d R (Eqs. 4-6 with the Z of Eq. 7 and its KS kernels) against
    Richardson-extrapolated central differences of omega_1(R), each geometry's
    ground state re-converged, W frozen."""
    alpha, S, A, U, Z, w = ks_solved
    F = solvers.dwdR(S, A, Z)
    # without the KS kernels in U and Z the derivative is wrong
    Zb, _ = solvers.zvector_cg(S, solvers.u_vector(S, A), tol=1e-12)
    Fb = solvers.dwdR(S, A, Zb)
    d = 0.006742
    worst, worst_bare = 0.0, 0.0
    # one component per site, each along a different axis
    for site, ax in ((0, 0), (1, 1), (2, 2)):
        f1 = ks.fd_force(S, site, ax, d)
        f2 = ks.fd_force(S, site, ax, d / 2)
        fd = (4 * f2 - f1) / 3
        worst = max(worst, abs(fd - F[site, ax]))
        worst_bare = max(worst_bare, abs(fd - Fb[site, ax]))
    print(f"alpha {alpha}: max |F - FD| {worst:.2e}; without the kernels {worst_bare:.2e}; "
          f"max |F| {np.abs(F).max():.2e}")
    assert worst < 1e-6
    assert worst_bare > 100 * worst
