"""Self-consistent synthetic Kohn-Sham model and the KS response kernels of
the Z-vector equation (Eq. 7 and SM Sec. I) -- oracle, test infrastructure.

The paper's ground state is a DFT calculation (semi-local or hybrid); its
Z-vector equation then carries the KS response kernels f_Hxc^loc and
alpha_EXX.  The synthetic stand-in used here (a reading: the paper fixes no
functional for this purpose) is a closed-shell model

    rho(r)    = 2 sum_v phi_v(r)^2                 (spin-restricted, N_v doubly occupied)
    H_KS[phi] = T + V_ext + V_H[rho] + V_xc[rho] - alpha K_x[phi]
    V_H       = v_c * rho                          (the oracle's Poisson solve, v_c(0) = 0)
    V_xc(r)   = -(3/pi)^(1/3) [ (rho(r) + rho_f)^(1/3) - rho_f^(1/3) ]
                (Slater exchange with a density floor rho_f, so the kernel stays
                 finite in empty regions)
    f_xc(r)   = dV_xc/drho = -(1/3)(3/pi)^(1/3) (rho(r) + rho_f)^(-2/3)
    (K_x psi)(r) = sum_w phi_w(r) [v_c * (phi_w psi)](r)   (same-spin exact exchange)

solved to self-consistency.  The BSE operator of Eqs. 1-2 keeps its form with
D = P_c (H_KS - eps_v + Delta), H_KS frozen at the ground state.

What changes for the forces (SM Sec. I, with the real orbitals of a Gamma-point
calculation and the derivative taken with respect to <phi_v|):

* U gains its D part (the scissor derivation of SM Sec. I):
    u^D_v = P_c { 2 [f_Hxc * Drho_x] phi_v
                  - alpha sum_v' [v_c * (a_v' phi_v)] a_v'
                  + alpha sum_v' [v_c * (phi_v' phi_v)] sum_v'' <a_v''|a_v'> phi_v'' }
  with f_Hxc * g = v_c * g + f_xc g.  The factor 2 is dV/d<phi_v| through the
  closed-shell density rho = 2 sum phi^2 (the paper writes the term per spin).
* The Z-vector operator (Eq. 7) is the orbital Hessian of the KS constraint:
    (D^KS Z)_v + 4 P_c [f_Hxc * (sum_v' phi_v' Z_v')] phi_v           (2 K^1e,KS + 2 K^2e,KS)
              - alpha P_c sum_v' [v_c * (phi_v' phi_v)] Z_v'           (K^1d,KS)
              - alpha P_c sum_v' [v_c * (Z_v' phi_v)] phi_v'           (K^2d,KS)
  symmetric and, at a stable ground state, positive definite on the P_c space.
* The force contraction of Eqs. 4-6 is unchanged (V_H, V_xc and K_x depend
  on the sites only through the orbitals, which Z accounts for).

Pins: tests/test_oracle_ks.py (self-consistency residual, f_xc against a
difference quotient of V_xc, U against a directional derivative of A^T M A
with H rebuilt from the displaced orbitals, the Z operator's symmetry and its
dense solve, and d omega/d R against central differences of omega with the
ground state re-converged at each displaced geometry and W frozen).
"""
from __future__ import annotations

import numpy as np

from . import solvers
from .model import System

CX = (3.0 / np.pi) ** (1.0 / 3.0)


class KSSystem(System):
    """System whose H_KS is the self-consistent Hartree + local-xc (+ alpha
    exact exchange) Hamiltonian of the module docstring."""

    def __init__(self, basis, site_xyz, site_depth, site_width, pdep, lam, n_val, *,
                 alpha=0.0, rho_floor=1e-3, **kw):
        super().__init__(basis, site_xyz, site_depth, site_width, pdep, lam, n_val, **kw)
        self.alpha = float(alpha)
        self.rho_floor = float(rho_floor)
        self.Vext = self.Vr.copy()
        self.phir_gs = None       # occupied orbitals on the grid that build H_KS

    # ---- functional ----------------------------------------------------
    def density(self, phir):
        return 2.0 * (phir * phir).sum(0)

    def v_xc(self, rho):
        f = self.rho_floor
        return -CX * (np.cbrt(rho + f) - np.cbrt(f))

    def f_xc(self, rho):
        return -(CX / 3.0) * (rho + self.rho_floor) ** (-2.0 / 3.0)

    def v_hxc(self, rho):
        return self.poisson(rho) + self.v_xc(rho)

    def f_hxc_apply(self, g, rho):
        """f_Hxc * g for a grid function g (f_xc at the density rho)."""
        return self.poisson(g) + self.f_xc(rho) * g

    def exchange_grid(self, occ_r, xr):
        """(K_x x)(r) = sum_w phi_w(r) [v_c * (phi_w x)](r) for grid functions
        xr[..., grid], with the occupied orbitals occ_r[w][grid]."""
        out = np.zeros_like(xr)
        for w in range(occ_r.shape[0]):
            out += occ_r[w] * self.poisson(occ_r[w] * xr)
        return out

    # ---- Hamiltonian of the current ground state -----------------------
    def apply_H(self, x):
        y = super().apply_H(x)
        if self.alpha != 0.0 and self.phir_gs is not None:
            xr = self.b.to_grid(x)
            y = y - self.alpha * self.b.from_grid(self.exchange_grid(self.phir_gs, xr))
        return y

    def dense_exchange(self, occ_r, E):
        """<e_j|K_x|e_k> from the explicit basis matrix E[N_r][N_pw]."""
        b = self.b
        cols = E.T.reshape((b.n_pw,) + b.grid)           # e_k on the grid
        K = self.exchange_grid(occ_r, cols).reshape(b.n_pw, -1)
        M = (b.omega / b.n_r) * (K @ E)                   # M[k][j] = <K_x e_k|e_j>
        return 0.5 * (M + M.T)

    def dense_H(self, E=None):
        E = self.b.basis_matrix() if E is None else E
        H = super().dense_H(E)
        if self.alpha != 0.0 and self.phir_gs is not None:
            H = H - self.alpha * self.dense_exchange(self.phir_gs, E)
        return H

    def ground_state(self, n_extra=0, E=None, tol=1e-12, max_iter=400, verbose=False):
        """Self-consistent ground state by Anderson (Pulay) mixing of the
        Hartree-xc potential (and, with alpha, of the exchange matrix),
        each step a dense eigh.  Returns all eigenvalues."""
        b = self.b
        E = b.basis_matrix() if E is None else E
        nv = self.n_val
        T = self.T
        Vx = b.omega / b.n_r

        def build(vhxc, kx):
            H = (Vx * (E.T * (self.Vext + vhxc).reshape(-1)) @ E)
            H[np.diag_indices_from(H)] += T
            H = 0.5 * (H + H.T)
            if self.alpha != 0.0:
                H = H - self.alpha * kx
            return H

        def outputs(phi):
            phir = b.to_grid(phi)
            rho = self.density(phir)
            kx = self.dense_exchange(phir, E) if self.alpha != 0.0 else None
            return self.v_hxc(rho), kx, phir

        npot = b.n_r
        x = np.zeros(npot + (b.n_pw * b.n_pw if self.alpha != 0.0 else 0))
        hist_x, hist_f = [], []
        beta, m = 0.3, 8
        for it in range(max_iter):
            vin = x[:npot].reshape(b.grid)
            kin = x[npot:].reshape(b.n_pw, b.n_pw) if self.alpha != 0.0 else None
            w, U = np.linalg.eigh(build(vin, kin))
            vout, kout, _ = outputs(U[:, :nv].T)
            xo = np.concatenate([vout.reshape(-1)] +
                                ([kout.reshape(-1)] if self.alpha != 0.0 else []))
            f = xo - x
            res = np.abs(f).max()
            if verbose:
                print(f"scf {it}: {res:.3e}")
            if res <= tol:
                break
            hist_x.append(x.copy())
            hist_f.append(f.copy())
            hist_x, hist_f = hist_x[-m:], hist_f[-m:]
            if len(hist_f) > 1:
                dF = np.array([hist_f[i + 1] - hist_f[i] for i in range(len(hist_f) - 1)])
                dX = np.array([hist_x[i + 1] - hist_x[i] for i in range(len(hist_x) - 1)])
                g, *_ = np.linalg.lstsq(dF.T, f, rcond=None)
                x = x + beta * f - (dX.T + beta * dF.T) @ g
            else:
                x = x + beta * f
        else:
            raise RuntimeError(f"SCF did not converge ({res:.2e})")
        # final Hamiltonian from the converged orbitals, and its eigenpairs
        phi = U[:, :nv].T
        vhxc, kx, phir = outputs(phi)
        self.Vr = self.Vext + vhxc
        self.V0 = None
        self.phir_gs = phir
        self.scf_iters = it
        self.rho_gs = self.density(phir)
        w, U = np.linalg.eigh(build(vhxc, kx))
        self.set_orbitals(U[:, :nv].T.copy(), w[:nv].copy())
        self.phir_gs = self.phir
        self.eps_all, self.psi_all = w, U.T.copy()
        self.eps_c = w[nv:nv + n_extra].copy()
        self.psi_c = U[:, nv:nv + n_extra].T.copy()
        return w

    def scf_residual(self):
        """max_v |H[phi] phi_v - eps_v phi_v| with H rebuilt from phi."""
        R = self.apply_H(self.phi) - self.eps[:, None] * self.phi
        return np.abs(R).max()

    # ---- the BSE operator: D carries the exact-exchange part of H_KS ----
    def apply(self, X):
        Y = super().apply(X)
        if self.alpha != 0.0:
            X = np.asarray(X, dtype=np.float64)
            A = self.proj_c(X)
            xr = self.b.to_grid(A)
            K = self.b.from_grid(self.exchange_grid(self.phir, xr))
            Y = Y - self.alpha * self.proj_c(K)
        return Y

    def apply_bands(self, X, bands):
        Y = super().apply_bands(X, bands)
        if self.alpha != 0.0:
            bands = np.asarray(bands, dtype=np.int64)
            X = np.asarray(X, dtype=np.float64)
            for i in range(X.shape[0]):
                A = self.proj_c(X[i])
                xr = self.b.to_grid(A)[bands]
                K = self.b.from_grid(self.exchange_grid(self.phir, xr))
                Y[i] -= self.alpha * (K - (K @ self.phi.T) @ self.phi)
        return Y


def displaced(sys: KSSystem, site, axis, delta):
    xyz = sys.site_xyz.copy()
    xyz[site, axis] += delta
    return KSSystem(sys.b, xyz, sys.site_depth, sys.site_width, sys.pdep, sys.lam, sys.n_val,
                    alpha=sys.alpha, rho_floor=sys.rho_floor, scissor=sys.scissor,
                    spin=sys.spin, kmask=sys.kmask)


# ---------------------------------------------------------------------------
# U vector: the K part of solvers.u_vector plus the D part (SM Sec. I)
# ---------------------------------------------------------------------------
def u_d_part(sys: KSSystem, A):
    b = sys.b
    A = sys.proj_c(np.asarray(A, dtype=np.float64))
    ar = b.to_grid(A)
    phir = sys.phir
    O = A @ A.T                                              # <a_v|a_v'>
    rho_x = (ar * ar).sum(0) - np.einsum("vw,vxyz,wxyz->xyz", O, phir, phir)
    g = 2.0 * sys.f_hxc_apply(rho_x, sys.rho_gs) * phir      # [v][grid]
    if sys.alpha != 0.0:
        nv = sys.n_val
        P = np.einsum("uv,uxyz->vxyz", O, phir)             # sum_v'' <a_v''|a_v'> phi_v''
        for v in range(nv):
            g[v] -= sys.alpha * (sys.poisson(ar * phir[v]) * ar).sum(0)
            g[v] += sys.alpha * (sys.poisson(phir * phir[v]) * P).sum(0)
    return sys.proj_c(b.from_grid(g))


def u_vector(sys: KSSystem, A):
    return solvers.u_vector(sys, A) + u_d_part(sys, A)


# ---------------------------------------------------------------------------
# Z-vector operator with the KS response kernels (Eq. 7)
# ---------------------------------------------------------------------------
def apply_zop(sys: KSSystem, Z):
    b = sys.b
    Z = sys.proj_c(np.asarray(Z, dtype=np.float64))
    out = sys.apply_H(Z) - sys.eps[:, None] * Z
    zr = b.to_grid(Z)
    phir = sys.phir
    g = 4.0 * sys.f_hxc_apply((phir * zr).sum(0), sys.rho_gs) * phir
    if sys.alpha != 0.0:
        for v in range(sys.n_val):
            g[v] -= sys.alpha * (sys.poisson(phir * phir[v]) * zr).sum(0)
            g[v] -= sys.alpha * (sys.poisson(zr * phir[v]) * phir).sum(0)
    return sys.proj_c(out + b.from_grid(g))


def zvector_cg(sys: KSSystem, U, tol=1e-8, max_iter=5000, z0=None):
    """Preconditioned CG on the whole block (the kernels couple the bands),
    preconditioner 1/max(|G|^2/2 - eps_v + shift, 0.1).  Returns (Z, info)."""
    from .model import PRECOND_SHIFT
    U = sys.proj_c(np.asarray(U, dtype=np.float64))
    nu = np.linalg.norm(U)
    pre = 1.0 / np.maximum(sys.T[None, :] - sys.eps[:, None] + PRECOND_SHIFT, 0.1)
    Z = np.zeros_like(U) if z0 is None else sys.proj_c(np.array(z0, dtype=np.float64))
    R = -U - apply_zop(sys, Z)
    P = sys.proj_c(pre * R)
    rz = (R * P).sum()
    hist = []
    for it in range(max_iter):
        rel = np.linalg.norm(R) / nu if nu > 0 else 0.0
        hist.append(rel)
        if rel <= tol:
            return Z, dict(iters=it, resid=rel, hist=hist, converged=True)
        AP = apply_zop(sys, P)
        a = rz / (P * AP).sum()
        Z = Z + a * P
        R = R - a * AP
        Zr = sys.proj_c(pre * R)
        rz_new = (R * Zr).sum()
        P = Zr + (rz_new / rz) * P
        rz = rz_new
    return Z, dict(iters=max_iter, resid=rel, hist=hist, converged=False)


# ---------------------------------------------------------------------------
# finite differences of omega with the ground state re-converged (W frozen)
# ---------------------------------------------------------------------------
def omega_scf(sys: KSSystem, state=0):
    sys.ground_state(n_extra=0)
    return solvers.omega_dense(sys, state)


def fd_force(sys: KSSystem, site, axis, delta, state=0):
    wp = omega_scf(displaced(sys, site, axis, +delta), state)
    wm = omega_scf(displaced(sys, site, axis, -delta), state)
    return (wp - wm) / (2 * delta)
