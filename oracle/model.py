"""Synthetic Kohn-Sham system, screened interaction and the DMPT BSE operator.

Oracle (test infrastructure).  Plain numpy, FP64, written step by step in the
paper's notation.

Hamiltonian (stands in for the DFT ground state of SM Sec. IV):
    H = T + V(r),  T = |G|^2/2 on the sphere, V a sum of Gaussian wells
    V_I(r) = -D_I exp(-|r - R_I|^2 / (2 w_I^2)), periodised through G space:
    V(G) = -sum_I (D_I/Omega) (2 pi w_I^2)^(3/2) exp(-w_I^2 |G|^2/2) exp(-i G.R_I)
    on every grid frequency, zero on the Nyquist planes so V(r) is real.
    H acts as T x + <e|V(r) (grid of x)>.

Screened interaction (Eq. 3):  W = v_c + v_c^(1/2) [sum_a phi_a c_a phi_a^T] v_c^(1/2),
c_a = lambda_a/(1 - lambda_a), PDEP vectors phi_a orthonormal in the real
basis of the wavefunction sphere with no G = 0 component; v_c(G) = 4 pi/|G|^2
on every grid frequency (minimum image), v_c(0) = 0.

DMPT operator (Eqs. 1-2, scissor form of Table S-I):
    (D A)_v   = P_c (H - eps_v + Delta) a_v
    (K1e A)_v = P_c (v_c * Drho) phi_v,        Drho = sum_v phi_v a_v
    (K1d A)_v = P_c sum_v' tau_{v'v} a_v',     tau_{v'v} = W (phi_v' phi_v)
    M = D + s K1e - K1d  (s = 2: spin-restricted singlet).
The apply returns Y = P_c M P_c X so the operator is symmetric on the whole
N_v x N_pw space (its occupied directions map to zero).
"""
from __future__ import annotations

import numpy as np

from . import fft as _fft

from .basis import Basis

# kernel mask bits (same meaning on both sides; a test hook)
K_D, K_1E, K_1D_BARE, K_1D_PDEP = 1, 2, 4, 8
K_ALL = 0xF

# Ha; shift of the kinetic preconditioner model (Davidson and Z-vector CG)
PRECOND_SHIFT = 0.25


class System:
    def __init__(self, basis: Basis, site_xyz, site_depth, site_width, pdep,
                 lam, n_val, *, scissor=0.0, spin=2, kmask=K_ALL):
        self.b = basis
        self.site_xyz = np.asarray(site_xyz, dtype=np.float64).reshape(-1, 3)
        self.site_depth = np.asarray(site_depth, dtype=np.float64)
        self.site_width = np.asarray(site_width, dtype=np.float64)
        self.n_sites = len(self.site_depth)
        self.pdep = np.asarray(pdep, dtype=np.float64)
        self.lam = np.asarray(lam, dtype=np.float64)
        self.c = self.lam / (1.0 - self.lam)
        self.n_val = int(n_val)
        self.scissor = float(scissor)
        self.spin = float(spin)
        self.kmask = int(kmask)
        b = basis
        self.T = 0.5 * b.g2
        self.VG = self.potential_G()
        self.Vr = (_fft.ifftn(self.VG) * b.n_r).real
        self.V0 = self.VG[0, 0, 0].real
        g2 = b.grid_g2
        vc = np.zeros_like(g2)
        nz = g2 > 0
        vc[nz] = 4 * np.pi / g2[nz]
        self.vc = vc
        vs = np.zeros(b.n_pw)
        vs[1:] = np.sqrt(4 * np.pi / b.g2[1:])
        self.vsqrt = vs
        self.phi = None

    # ---- potential ----------------------------------------------------
    def site_potential_G(self, i):
        """V_I(G) of site i on the full grid (Nyquist planes zero)."""
        b = self.b
        d, w = self.site_depth[i], self.site_width[i]
        R = self.site_xyz[i]
        gr = np.tensordot(R, b.grid_g, axes=(0, 0))
        v = -(d / b.omega) * (2 * np.pi * w * w) ** 1.5 \
            * np.exp(-0.5 * w * w * b.grid_g2) * np.exp(-1j * gr)
        v[b.nyquist] = 0.0
        return v

    def potential_G(self):
        v = np.zeros(self.b.grid, dtype=np.complex128)
        for i in range(self.n_sites):
            v += self.site_potential_G(i)
        return v

    # ---- Hamiltonian ----------------------------------------------------
    def apply_H(self, x):
        """H x for x[..., n_pw]."""
        return self.T * x + self.b.from_grid(self.Vr * self.b.to_grid(x))

    def dense_H(self, E=None):
        """Dense H_jk = T_j delta_jk + <e_j|V|e_k> from the explicit basis matrix."""
        b = self.b
        E = b.basis_matrix() if E is None else E
        Vr = self.Vr.reshape(-1)
        H = (b.omega / b.n_r) * (E.T * Vr) @ E
        H[np.diag_indices_from(H)] += self.T
        return 0.5 * (H + H.T)

    def ground_state(self, n_extra=0, E=None):
        """Lowest n_val + n_extra eigenpairs by dense eigh (small systems)."""
        H = self.dense_H(E)
        w, U = np.linalg.eigh(H)
        self.set_orbitals(U[:, :self.n_val].T.copy(), w[:self.n_val].copy())
        self.eps_all, self.psi_all = w, U.T.copy()
        n = self.n_val
        self.eps_c = w[n:n + n_extra].copy()
        self.psi_c = U[:, n:n + n_extra].T.copy()
        return w

    def set_orbitals(self, phi, eps, psi_c=None, eps_c=None):
        self.phi = np.ascontiguousarray(phi, dtype=np.float64)     # [N_v][N_pw]
        self.eps = np.asarray(eps, dtype=np.float64)
        self.phir = self.b.to_grid(self.phi)                       # [N_v][grid]
        if psi_c is not None:
            self.psi_c = np.asarray(psi_c, dtype=np.float64)
            self.eps_c = np.asarray(eps_c, dtype=np.float64)
        self._tau = None

    # ---- Coulomb and W ----------------------------------------------------
    def poisson(self, rho):
        """v_c * rho on the grid (v_c(G) = 4 pi/|G|^2, v_c(0) = 0)."""
        G = _fft.fftn(rho, axes=(-3, -2, -1))
        return _fft.ifftn(G * self.vc, axes=(-3, -2, -1)).real

    def pdep_term(self, rho):
        """Low-rank part of Eq. 3 acting on a grid density:
        sum_k e_k [V^1/2 P C P^T V^1/2 rho_S]_k with rho_S = <e|rho>."""
        rs = self.b.from_grid(rho)                       # [..., n_pw]
        t = (rs * self.vsqrt) @ self.pdep                # [..., n_pdep]
        f = ((t * self.c) @ self.pdep.T) * self.vsqrt    # [..., n_pw]
        return self.b.to_grid(f)

    def apply_W(self, rho, mask=None):
        mask = self.kmask if mask is None else mask
        out = np.zeros_like(rho)
        if mask & K_1D_BARE:
            out += self.poisson(rho)
        if mask & K_1D_PDEP:
            out += self.pdep_term(rho)
        return out

    def tau(self):
        """tau_{v'v}(r) = W(phi_v' phi_v) for all pairs, [N_v][N_v][grid]."""
        if self._tau is None:
            n = self.n_val
            t = np.zeros((n, n) + self.b.grid)
            for v in range(n):
                rho = self.phir[v:n] * self.phir[v]
                w = self.apply_W(rho)
                t[v, v:n] = w
                t[v:n, v] = w
            self._tau = t
        return self._tau

    # ---- projector and operator ------------------------------------------
    def proj_c(self, X):
        """P_c acting on every orbital of X[..., N_v, N_pw]."""
        S = X @ self.phi.T                       # <phi_w|x_v>  [..., N_v, N_v]
        return X - S @ self.phi

    def kernel_grid(self, ar, mask=None):
        """s v_c*Drho phi_v - sum_v' tau_{v'v} a_v' on the grid, before P_c
        (the kernel part of the operator, K-tilde)."""
        mask = self.kmask if mask is None else mask
        z = np.zeros_like(ar)
        if mask & K_1E:
            drho = (self.phir * ar).sum(0)
            z += self.spin * self.poisson(drho) * self.phir
        if mask & (K_1D_BARE | K_1D_PDEP):
            tau = self.tau()
            z -= np.einsum("uvxyz,uxyz->vxyz", tau, ar)
        return z

    def sigma_grid(self, ar):
        """sigma_v = sum_v' W(a_v' a_v) phi_v' on the grid (the W term of U)."""
        g = np.zeros_like(ar)
        for v in range(self.n_val):
            sig = self.apply_W(ar * ar[v])               # [v'][grid]
            g[v] = (sig * self.phir).sum(0)
        return g

    def apply(self, X):
        """Y = P_c M P_c X for X[n_b][N_v][N_pw] (or one [N_v][N_pw])."""
        X = np.asarray(X, dtype=np.float64)
        one = X.ndim == 2
        X = X[None] if one else X
        Y = np.empty_like(X)
        for i in range(X.shape[0]):
            A = self.proj_c(X[i])
            ar = self.b.to_grid(A)
            z = self.kernel_grid(ar)
            if self.kmask & K_D:
                z += self.Vr * ar
                Z = self.b.from_grid(z) + (self.T[None, :] - self.eps[:, None]
                                           + self.scissor) * A
            else:
                Z = self.b.from_grid(z)
            Y[i] = self.proj_c(Z)
        return Y[0] if one else Y

    def apply_bands(self, X, bands):
        """Rows `bands` of Y = P_c M P_c X for X[n_b][N_v][N_pw], without the
        whole tau: tau_{v'v} = W(phi_v' phi_v) is built for every v' and the
        requested output bands v only (Eq. 2c).  Each output row needs every
        input row (P_c on the input, Drho of Eq. 2b and the sum over v'), but
        the output projector acts on each row alone, so the rows returned are
        those of the full apply.  Returns [n_b][len(bands)][N_pw]."""
        X = np.asarray(X, dtype=np.float64)
        bands = np.asarray(bands, dtype=np.int64)
        mask = self.kmask
        taus = None
        if mask & (K_1D_BARE | K_1D_PDEP):
            taus = [self.apply_W(self.phir * self.phir[v]) for v in bands]
        Y = np.empty((X.shape[0], len(bands), X.shape[2]))
        for i in range(X.shape[0]):
            A = self.proj_c(X[i])
            ar = self.b.to_grid(A)
            z = np.zeros((len(bands),) + self.b.grid)
            if mask & K_1E:
                drho = (self.phir * ar).sum(0)
                z += self.spin * self.poisson(drho) * self.phir[bands]
            if taus is not None:
                for k in range(len(bands)):
                    z[k] -= np.einsum("uxyz,uxyz->xyz", taus[k], ar)
            Ab = A[bands]
            if mask & K_D:
                z += self.Vr * ar[bands]
                Z = self.b.from_grid(z) + (self.T[None, :] - self.eps[bands][:, None]
                                           + self.scissor) * Ab
            else:
                Z = self.b.from_grid(z)
            Y[i] = Z - (Z @ self.phi.T) @ self.phi
        return Y

    def diag_precond(self):
        """Kinetic diagonal model of D used to precondition Davidson:
        |G|^2/2 - eps_v + Delta + PRECOND_SHIFT (the paper names no
        preconditioner; the shift keeps the model positive for low G)."""
        return self.T[None, :] - self.eps[:, None] + self.scissor + PRECOND_SHIFT
