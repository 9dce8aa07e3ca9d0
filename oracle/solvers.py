"""Exciton eigensolver, U vector, Z-vector solve and forces (oracle).

Plain numpy FP64, test infrastructure only.

Reduction used for the synthetic Hamiltonian (no Hartree, xc or exact
exchange in H_KS): the KS kernels of Eq. 7 vanish (f_Hxc = 0, alpha_EXX = 0),
and the D part of U lies in the occupied space and is removed by P_c
(SM Sec. I, scissor derivation).  Hence

    Z-vector:  P_c (H - eps_v) P_c Z_v = -u_v          for every band v
    u_v = P_c[ s (v_c*Drho) a_v - sum_v' sigma_{v'v} phi_v' ] - sum_v' S_{vv'} a_v'
    sigma_{v'v} = W(a_v' a_v),  S_{vv'} = <phi_v | [(s K1e - K1d) A]_v'> before P_c
    (the K1e and K1d derivatives of SM Sec. I, with dW/dphi = 0)

    dw/dR = int dV/dR (Drho_x + Drho_z)                                  (Eq. 4)
    Drho_x = sum_v a_v^2 - sum_vv' phi_v phi_v' <a_v'|a_v>                (Eq. 5)
    Drho_z = 2 sum_v Z_v phi_v                                           (Eq. 6)
"""
from __future__ import annotations

import numpy as np

from . import fft as _fft
from .model import K_1D_BARE, K_1D_PDEP, K_1E, PRECOND_SHIFT, System


# ---------------------------------------------------------------------------
# Davidson (the paper names no eigensolver; the plain definition is the
# lowest eigenvalues of the operator on the P_c space)
# ---------------------------------------------------------------------------
def _orth_against(V, W, drop=1e-8):
    """Two passes of block Gram-Schmidt of the rows of W against the rows of V,
    then among themselves; rows are normalised first and dropped when less
    than `drop` of their norm survives."""
    out = []
    for w in W:
        w = w / np.linalg.norm(w)
        for _ in range(2):
            if len(V):
                w = w - (V @ w) @ V
            for u in out:
                w = w - (u @ w) * u
        n = np.linalg.norm(w)
        if n > drop:
            out.append(w / n)
    return np.array(out) if out else np.zeros((0, W.shape[1]))


def initial_guess(sys: System, nb):
    """Lowest bare transitions a_v = delta_{v v0} psi_c0 when conduction
    states are known; otherwise P_c-projected plane waves of lowest diagonal."""
    nv, npw = sys.n_val, sys.b.n_pw
    guesses = []
    if getattr(sys, "psi_c", None) is not None and len(sys.psi_c) > 0:
        de = sys.eps_c[None, :] - sys.eps[:, None]
        order = np.argsort(de, axis=None, kind="stable")[:nb]
        for k in order:
            v, c = np.unravel_index(k, de.shape)
            x = np.zeros((nv, npw))
            x[v] = sys.psi_c[c]
            guesses.append(x.reshape(-1))
    else:
        d = sys.diag_precond()
        order = np.argsort(d, axis=None, kind="stable")
        for k in order:
            v, j = np.unravel_index(k, d.shape)
            x = np.zeros((nv, npw))
            x[v, j] = 1.0
            x = sys.proj_c(x)
            if np.linalg.norm(x) > 0.3:
                guesses.append(x.reshape(-1))
            if len(guesses) == nb:
                break
    return np.array(guesses)


def davidson(sys: System, n_states=1, tol=1e-8, max_iter=300, block=None,
             max_sub=None, x0=None, verbose=False):
    """Block Davidson for the lowest n_states eigenpairs of P_c M P_c.

    Returns (omega[n_states], X[n_states][N_v][N_pw], info)."""
    nv, npw = sys.n_val, sys.b.n_pw
    nb = block or n_states + 4
    max_sub = max_sub or 8 * nb
    shape = (nv, npw)
    if x0 is not None:
        W0 = np.asarray(x0).reshape(len(x0), -1)
        extra = initial_guess(sys, nb)
        W0 = np.vstack([W0, extra])[:nb]
    else:
        W0 = initial_guess(sys, nb)
    W0 = sys.proj_c(W0.reshape(-1, *shape)).reshape(len(W0), -1)
    V = _orth_against(np.zeros((0, nv * npw)), W0)
    AV = sys.apply(V.reshape(-1, *shape)).reshape(len(V), -1)
    dpre = sys.diag_precond().reshape(-1)
    hist = []
    theta = None
    for it in range(max_iter):
        Hs = V @ AV.T
        Hs = 0.5 * (Hs + Hs.T)
        th, c = np.linalg.eigh(Hs)
        k = min(nb, len(th))
        X = c[:, :k].T @ V
        AX = c[:, :k].T @ AV
        R = AX - th[:k, None] * X
        rn = np.linalg.norm(R, axis=1)
        hist.append(rn[:n_states].copy())
        theta = th[:n_states]
        if verbose:
            print(it, len(V), th[:n_states], rn[:n_states])
        if (rn[:n_states] <= tol).all():
            return theta.copy(), X[:n_states].reshape(-1, *shape), \
                dict(iters=it, resid=rn[:n_states], hist=hist, converged=True)
        T = []
        for i in range(k):
            if rn[i] <= tol:
                continue
            den = dpre - th[i]
            den = np.where(np.abs(den) < 0.1, np.where(den < 0, -0.1, 0.1), den)
            T.append(R[i] / den)
        T = sys.proj_c(np.array(T).reshape(-1, *shape)).reshape(len(T), -1)
        if len(V) + len(T) > max_sub:
            keep = min(2 * nb, len(th))
            V = c[:, :keep].T @ V
            AV = c[:, :keep].T @ AV
        Tn = _orth_against(V, T)
        if len(Tn) == 0:
            break
        ATn = sys.apply(Tn.reshape(-1, *shape)).reshape(len(Tn), -1)
        V = np.vstack([V, Tn])
        AV = np.vstack([AV, ATn])
    return theta.copy(), X[:n_states].reshape(-1, *shape), \
        dict(iters=max_iter, resid=rn[:n_states], hist=hist, converged=False)


# ---------------------------------------------------------------------------
# U vector (SM Sec. I: derivative of A^T M A with respect to <phi_v|)
# ---------------------------------------------------------------------------
def u_vector(sys: System, A):
    """u_v for one converged exciton A[N_v][N_pw] (A orthogonal to phi,
    sum_v <a_v|a_v> = 1)."""
    b = sys.b
    A = sys.proj_c(np.asarray(A, dtype=np.float64))
    ar = b.to_grid(A)
    g = np.zeros_like(ar)
    if sys.kmask & K_1E:
        drho = (sys.phir * ar).sum(0)
        g += sys.spin * sys.poisson(drho) * ar
    if sys.kmask & (K_1D_BARE | K_1D_PDEP):
        g -= sys.sigma_grid(ar)
    Ktil = b.from_grid(sys.kernel_grid(ar))            # kernel part before P_c
    S = sys.phi @ Ktil.T                               # S[w][v] = <phi_w|K~_v>
    u = sys.proj_c(b.from_grid(g)) - S @ A
    return u


# ---------------------------------------------------------------------------
# Z-vector: P_c (H - eps_v) P_c Z_v = -u_v (Eq. 7 with the KS kernels zero)
# ---------------------------------------------------------------------------
def apply_DKS(sys: System, Z):
    Z = sys.proj_c(Z)
    return sys.proj_c(sys.apply_H(Z) - sys.eps[:, None] * Z)


def zvector_cg(sys: System, U, tol=1e-8, max_iter=5000, z0=None):
    """Block PCG with per-band step sizes; diagonal preconditioner
    1/max(|G|^2/2 - eps_v + PRECOND_SHIFT, 0.1).  Returns (Z, info)."""
    U = sys.proj_c(np.asarray(U, dtype=np.float64))
    nu = np.linalg.norm(U)
    pre = 1.0 / np.maximum(sys.T[None, :] - sys.eps[:, None] + PRECOND_SHIFT, 0.1)
    Z = np.zeros_like(U) if z0 is None else sys.proj_c(np.array(z0, dtype=np.float64))
    R = -U - apply_DKS(sys, Z)
    P = sys.proj_c(pre * R)
    rz = (R * P).sum(1)
    hist = []
    for it in range(max_iter):
        rel = np.linalg.norm(R) / nu if nu > 0 else 0.0
        hist.append(rel)
        if rel <= tol:
            return Z, dict(iters=it, resid=rel, hist=hist, converged=True)
        AP = apply_DKS(sys, P)
        pap = (P * AP).sum(1)
        alpha = np.where(pap != 0, rz / np.where(pap != 0, pap, 1), 0.0)
        Z = Z + alpha[:, None] * P
        R = R - alpha[:, None] * AP
        Zr = sys.proj_c(pre * R)
        rz_new = (R * Zr).sum(1)
        beta = np.where(rz != 0, rz_new / np.where(rz != 0, rz, 1), 0.0)
        P = Zr + beta[:, None] * P
        rz = rz_new
    return Z, dict(iters=max_iter, resid=rel, hist=hist, converged=False)


def zvector_sos(sys: System, U):
    """Dense sum over states Z_v = -sum_c psi_c <psi_c|u_v>/(eps_c - eps_v),
    every conduction state of the dense Hamiltonian (ground_state() first)."""
    nv = sys.n_val
    psi = sys.psi_all[nv:]
    ec = sys.eps_all[nv:]
    proj = U @ psi.T                                   # [v][c]
    return -(proj / (ec[None, :] - sys.eps[:, None])) @ psi


# ---------------------------------------------------------------------------
# forces (Eqs. 4-6)
# ---------------------------------------------------------------------------
def densities(sys: System, A, Z):
    b = sys.b
    A = np.asarray(A, dtype=np.float64)
    ar = b.to_grid(A)
    zr = b.to_grid(np.asarray(Z, dtype=np.float64))
    O = A @ A.T                                        # <a_v|a_v'>
    rho_x = (ar * ar).sum(0) - np.einsum("vw,vxyz,wxyz->xyz", O, sys.phir, sys.phir)
    rho_z = 2.0 * (zr * sys.phir).sum(0)
    return rho_x, rho_z


def dwdR(sys: System, A, Z):
    """d omega / d R_{I alpha} = Omega sum_G Re[conj(-i G_alpha V_I(G)) rho_t(G)]
    over the full grid, rho_t = Drho_x + Drho_z.  Returns [n_sites][3]."""
    b = sys.b
    rx, rz = densities(sys, A, Z)
    rg = _fft.fftn(rx + rz) / b.n_r
    out = np.zeros((sys.n_sites, 3))
    for i in range(sys.n_sites):
        vi = sys.site_potential_G(i)
        for a in range(3):
            dv = -1j * b.grid_g[a] * vi
            out[i, a] = b.omega * (np.conj(dv) * rg).real.sum()
    return out


def hf_ground_forces(sys: System):
    """d(sum of occupied eps)/dR = sum_v <phi_v|dV/dR|phi_v> (Hellmann-Feynman;
    a convenience beside the method's output d omega/d R, pinned against
    central differences of the occupied eigenvalue sum)."""
    b = sys.b
    rho = (sys.phir ** 2).sum(0)
    rg = _fft.fftn(rho) / b.n_r
    out = np.zeros((sys.n_sites, 3))
    for i in range(sys.n_sites):
        vi = sys.site_potential_G(i)
        for a in range(3):
            out[i, a] = b.omega * (np.conj(-1j * b.grid_g[a] * vi) * rg).real.sum()
    return out


# ---------------------------------------------------------------------------
# central finite differences with W frozen (SM Sec. II protocol)
# ---------------------------------------------------------------------------
def displaced(sys: System, site, axis, delta):
    xyz = sys.site_xyz.copy()
    xyz[site, axis] += delta
    return System(sys.b, xyz, sys.site_depth, sys.site_width, sys.pdep, sys.lam,
                  sys.n_val, scissor=sys.scissor, spin=sys.spin, kmask=sys.kmask)


def omega_dense(sys: System, state=0):
    from .dense import eh_matrix
    A, *_ = eh_matrix(sys)
    return np.linalg.eigvalsh(A)[state]


def omega_davidson(sys: System, state=0, tol=1e-11, n_extra=8):
    sys.ground_state(n_extra=n_extra)
    w, _, info = davidson(sys, n_states=state + 1, tol=tol, max_iter=500)
    if not info["converged"]:
        raise RuntimeError("Davidson did not converge in the FD check")
    return w[state]


def fd_force(sys: System, site, axis, delta, method="dense", state=0):
    f = omega_dense if method == "dense" else omega_davidson
    wp = f(displaced(sys, site, axis, +delta), state)
    wm = f(displaced(sys, site, axis, -delta), state)
    return (wp - wm) / (2 * delta)
