"""Conventional electron-hole BSE matrix on the same discrete model (oracle).

This is the plain definition the DMPT operator reproduces exactly when every
conduction state of the discrete Hamiltonian is kept (the paper contrasts the
two formulations after Eq. 3):

    A_eh[(v,c),(v',c')] = (eps_c - eps_v + Delta) d_vv' d_cc'
                          + s <rho_vc | v_c | rho_v'c'>  -  <rho_cc' | W | rho_vv'>

with rho_xy(r) = x(r) y(r).  Everything here is built from explicit matrices
instead of the FFT routines of ``model``: the cos/sin basis matrix E, a dense
DFT matrix for v_c and the dense W kernel on the grid,

    (W rho)(r) = sum_r' Wg[r, r'] rho(r'),  Wg = Vc + (Omega/N_r) E Vs P C P^T Vs E^T,
    Vc[r, r'] = (1/N_r) sum_G v_c(G) exp(i G.(r - r')),

and bilinear forms <f|K|g> = (Omega/N_r) f^T Kg g.  Only tiny systems fit.
"""
from __future__ import annotations

import numpy as np

from .model import K_1D_BARE, K_1D_PDEP, K_1E, K_D


_CACHE = {}


def _key(b):
    return (tuple(b.cell), b.grid, b.ecut)


def basis_matrix(b):
    k = ("E",) + _key(b)
    if k not in _CACHE:
        _CACHE[k] = b.basis_matrix()
    return _CACHE[k]


def dft_coulomb(sys):
    """Dense Vc[r, r'] = (1/N_r) sum_G v_c(G) exp(i G.(r - r'))."""
    b = sys.b
    k = ("Vc",) + _key(b)
    if k in _CACHE:
        return _CACHE[k]
    N = np.array(b.grid)
    j = np.array(np.meshgrid(*[np.arange(n) for n in N], indexing="ij")).reshape(3, -1).T
    nvec = b.grid_n.reshape(3, -1).T                    # minimum-image n for each G
    F = np.exp(-2j * np.pi * (j / N) @ nvec.T)          # F[r, G] = exp(-i G.r)
    vc = sys.vc.reshape(-1)
    Vc = (np.conj(F) * vc) @ F.T / b.n_r                # sum_G e^{iGr} v e^{-iGr'}
    _CACHE[k] = Vc.real.copy()
    return _CACHE[k]


def dense_W(sys, E, mask=None):
    mask = sys.kmask if mask is None else mask
    b = sys.b
    Wg = np.zeros((b.n_r, b.n_r))
    if mask & K_1D_BARE:
        Wg += dft_coulomb(sys)
    if mask & K_1D_PDEP:
        Q = (E * sys.vsqrt) @ sys.pdep                  # [N_r][n_pdep]
        Wg += (b.omega / b.n_r) * (Q * sys.c) @ Q.T
    return Wg


def eh_matrix(sys, E=None):
    """Return (A_eh, eps_v, eps_c, Psi_c) with Psi_c[c][N_pw] every conduction
    state of the dense Hamiltonian.  Index (v, c) -> v * N_c + c."""
    b = sys.b
    E = basis_matrix(b) if E is None else E
    H = sys.dense_H(E)
    w, U = np.linalg.eigh(H)
    nv = sys.n_val
    eps_v, eps_c = w[:nv], w[nv:]
    phi, psi = U[:, :nv], U[:, nv:]                      # columns in the sphere basis
    phir = E @ phi                                       # [N_r][N_v]
    psir = E @ psi                                       # [N_r][N_c]
    nc = psi.shape[1]
    q = b.omega / b.n_r
    A = np.zeros((nv * nc, nv * nc))
    if sys.kmask & K_D:
        A[np.diag_indices_from(A)] = (eps_c[None, :] - eps_v[:, None] + sys.scissor).reshape(-1)
    if sys.kmask & K_1E:
        Vc = dft_coulomb(sys)
        R = (phir[:, :, None] * psir[:, None, :]).reshape(b.n_r, nv * nc)
        A += sys.spin * q * R.T @ (Vc @ R)
    if sys.kmask & (K_1D_BARE | K_1D_PDEP):
        Wg = dense_W(sys, E)
        for v in range(nv):
            for vp in range(nv):
                tau = Wg @ (phir[:, v] * phir[:, vp])   # W(phi_v phi_v')
                blk = q * (psir * tau[:, None]).T @ psir  # <psi_c psi_c'|tau>
                A[v * nc:(v + 1) * nc, vp * nc:(vp + 1) * nc] -= blk
    A = 0.5 * (A + A.T)
    return A, eps_v, eps_c, psi.T.copy(), phi.T.copy()
