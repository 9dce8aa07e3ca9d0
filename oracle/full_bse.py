"""BSE beyond the Tamm-Dancoff approximation -- oracle, test infrastructure.

The coupled form of SM Sec. I (the first equation there, with the A_s and
B_s blocks and the coupling operators K^2e and K^2d).  For the real orbitals
of a Gamma-point calculation every conjugate drops:

    (K2e A)_v = P_c [v_c * sum_v' a_v' phi_v'] phi_v        (equal to (K1e A)_v)
    (K2d A)_v = P_c sum_v' [W (a_v' phi_v)] phi_v'
    A = D + s K1e - K1d,    B = s K2e - K2d,
    [[A, B], [B, A]] (X; Y) = omega (X; -Y).

With A + B and A - B symmetric positive definite on the P_c space (a stable
ground state), omega^2 are the eigenvalues of (A - B)(A + B) acting on X + Y,
and X - Y = (A + B)(X + Y) / omega.

Dense form (conventional electron-hole basis, every conduction state, the
same index layout as dense.eh_matrix):

    B_eh[(v,c),(v',c')] = s <rho_vc | v_c | rho_v'c'> - <rho_cv' | W | rho_c'v>

from projecting (B A)_v on psi_c with a_v' = sum_c' X[v'][c'] psi_c'.

Iterative solver: the subspace method of Stratmann, Scuseria and Frisch
(J. Chem. Phys. 109, 8218 (1998)) for the lowest roots of (A - B)(A + B):
with an orthonormal basis b of the P_c space, P = b^T (A + B) b and
Q = b^T (A - B) b, Q = L L^T, the symmetric eigenproblem L^T P L u = omega^2 u
gives c+ = L u (X + Y = b c+) and c- = P c+ / omega (X - Y = b c-),
normalised so that c+ . c- = 1 (X.X - Y.Y = 1).  Residuals
r+ = (A + B) b c+ - omega b c-, r- = (A - B) b c- - omega b c+; new
directions are both residuals divided by the kinetic diagonal model of D
shifted by -omega, orthonormalised against b (kept when more than 1e-3 of
their norm survives).  Converged when
||r+||^2 + ||r-||^2 <= tol^2 for every requested root.

Pins: tests/test_oracle_full_bse.py (the DMPT B apply against B_eh; the
free-electron closed form omega_G^2 = (T_G - eps + W_G/Omega)(T_G - eps +
2 s v_c(G)/Omega - W_G/Omega) with plane-wave PDEP pairs; B = 0 recovers the
TDA; the lowest omega lies below the TDA one; the +-omega pairing of the
full matrix; the iterative solver against the dense eigenvalues).
"""
from __future__ import annotations

import numpy as np

from . import dense
from .model import K_1D_BARE, K_1D_PDEP, K_1E, PRECOND_SHIFT, System


def apply_b(sys: System, X):
    """Y = P_c B P_c X for X[n_b][N_v][N_pw] (or one [N_v][N_pw])."""
    X = np.asarray(X, dtype=np.float64)
    one = X.ndim == 2
    X = X[None] if one else X
    Y = np.empty_like(X)
    for i in range(X.shape[0]):
        A = sys.proj_c(X[i])
        ar = sys.b.to_grid(A)
        z = np.zeros_like(ar)
        if sys.kmask & K_1E:                                    # s K2e
            drho = (sys.phir * ar).sum(0)
            z += sys.spin * sys.poisson(drho) * sys.phir
        if sys.kmask & (K_1D_BARE | K_1D_PDEP):                 # - K2d
            for v in range(sys.n_val):
                w = sys.apply_W(ar * sys.phir[v])               # W(a_v' phi_v), [v'][grid]
                z[v] -= (w * sys.phir).sum(0)
        Y[i] = sys.proj_c(sys.b.from_grid(z))
    return Y[0] if one else Y


def dense_b(sys: System, E=None):
    """B_eh in the layout of dense.eh_matrix (index v * N_c + c)."""
    b = sys.b
    E = dense.basis_matrix(b) if E is None else E
    H = sys.dense_H(E)
    w, U = np.linalg.eigh(H)
    nv = sys.n_val
    phir = E @ U[:, :nv]
    psir = E @ U[:, nv:]
    nc = psir.shape[1]
    q = b.omega / b.n_r
    B = np.zeros((nv * nc, nv * nc))
    if sys.kmask & K_1E:
        Vc = dense.dft_coulomb(sys)
        R = (phir[:, :, None] * psir[:, None, :]).reshape(b.n_r, nv * nc)
        B += sys.spin * q * R.T @ (Vc @ R)
    if sys.kmask & (K_1D_BARE | K_1D_PDEP):
        Wg = dense.dense_W(sys, E)
        for v in range(nv):
            for vp in range(nv):
                left = psir * phir[:, vp][:, None]              # rho_{c v'}
                right = psir * phir[:, v][:, None]              # rho_{c' v}
                B[v * nc:(v + 1) * nc, vp * nc:(vp + 1) * nc] -= q * left.T @ (Wg @ right)
    return 0.5 * (B + B.T)


def omega_dense(A, B, n=None):
    """Positive roots of [[A, B], [B, A]] (X; Y) = omega (X; -Y), ascending:
    omega^2 = eig((A - B)^(1/2) (A + B) (A - B)^(1/2))."""
    w, V = np.linalg.eigh(A - B)
    if w.min() <= 0:
        raise ValueError("A - B is not positive definite")
    S = (V * np.sqrt(w)) @ V.T
    om2 = np.linalg.eigvalsh(S @ (A + B) @ S)
    if om2.min() <= 0:
        raise ValueError("A + B is not positive definite")
    om = np.sqrt(np.sort(om2))
    return om if n is None else om[:n]


def davidson_full(sys: System, n_states=1, tol=1e-8, max_iter=300, n_start=None):
    """Lowest n_states roots by the Stratmann-Scuseria-Frisch subspace method
    (module docstring).  Returns (omega, X, Y, info) with X, Y [n][N_v][N_pw]."""
    shape = sys.phi.shape
    diag = sys.diag_precond() - PRECOND_SHIFT                  # T_G - eps_v + Delta
    nb = n_start or n_states + 4
    # start: the lowest bare transitions T_G - eps_v (one plane-wave direction each)
    order = np.argsort(diag, axis=None)
    basis = []
    for k in order:
        e = np.zeros(shape)
        e.flat[k] = 1.0
        e = sys.proj_c(e)
        for q in basis:
            e -= (q * e).sum() * q
        n = np.linalg.norm(e)
        if n > 1e-8:
            basis.append(e / n)
        if len(basis) == nb:
            break
    ApB, AmB = [], []
    done = 0
    info = dict(converged=False, iters=0)
    for it in range(1, max_iter + 1):
        for k in range(done, len(basis)):
            Av = sys.apply(basis[k])
            Bv = apply_b(sys, basis[k])
            ApB.append(Av + Bv)
            AmB.append(Av - Bv)
        done = len(basis)
        V = np.array(basis)
        Pp = np.tensordot(V, np.array(ApB), axes=([1, 2], [1, 2]))
        Qm = np.tensordot(V, np.array(AmB), axes=([1, 2], [1, 2]))
        Pp, Qm = 0.5 * (Pp + Pp.T), 0.5 * (Qm + Qm.T)
        L = np.linalg.cholesky(Qm)
        om2, U = np.linalg.eigh(L.T @ Pp @ L)
        om = np.sqrt(om2[:n_states])
        cp = L @ U[:, :n_states]                                 # X + Y coefficients
        cm = (Pp @ cp) / om                                      # X - Y coefficients
        s = np.sqrt(np.einsum("ik,ik->k", cp, cm))
        cp, cm = cp / s, cm / s
        Xp = np.tensordot(cp.T, V, axes=(1, 0))
        Xm = np.tensordot(cm.T, V, axes=(1, 0))
        Rp = np.tensordot(cp.T, np.array(ApB), axes=(1, 0)) - om[:, None, None] * Xm
        Rm = np.tensordot(cm.T, np.array(AmB), axes=(1, 0)) - om[:, None, None] * Xp
        res = np.sqrt((Rp ** 2).sum((1, 2)) + (Rm ** 2).sum((1, 2)))
        info.update(iters=it, resid=res)
        if np.all(res <= tol):
            info["converged"] = True
            break
        for k in range(n_states):
            if res[k] <= tol:
                continue
            den = diag - om[k]
            den = np.where(np.abs(den) < 1e-3, np.copysign(1e-3, den), den)
            for r in (Rp[k], Rm[k]):
                t = sys.proj_c(r / den)
                n0 = np.linalg.norm(t)
                for _ in range(2):                               # Gram-Schmidt, twice
                    for q in basis:
                        t = t - (q * t).sum() * q
                n = np.linalg.norm(t)
                if n > 1e-3 * n0 and n > 1e-300:
                    basis.append(t / n)
        if len(basis) == done:
            break
    X = 0.5 * (Xp + Xm)
    Y = 0.5 * (Xp - Xm)
    return om, X, Y, info
