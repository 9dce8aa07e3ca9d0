"""Real plane-wave basis of the Gamma-point wavefunction sphere (oracle).

The paper samples only Gamma (SM Sec. IV), so orbitals are real.  The discrete
model used throughout:

* cell L = (L1, L2, L3), volume Omega = L1 L2 L3; grid points
  r_j = (j1 L1/N1, j2 L2/N2, j3 L3/N3);
* G = 2 pi (n1/L1, n2/L2, n3/L3); Fourier coefficients
  f(G) = (1/N_r) sum_j f(r_j) exp(-i G.r_j), so f(r_j) = sum_G f(G) exp(i G.r_j);
* inner product <f|g> = (Omega/N_r) sum_j f(r_j) g(r_j);
* sphere S = {G : |G|^2/2 <= ecut}, with every |n_i| < N_i/2;
* orthonormal real basis: e_0 = Omega^(-1/2) and, for every G of the half
  sphere S+ (first non-zero n_i positive), c_G = sqrt(2/Omega) cos(G.r) and
  s_G = sqrt(2/Omega) sin(G.r);
* order: G = 0 first, then S+ sorted by (|n|^2, n1, n2, n3), cos before sin.
"""
from __future__ import annotations

import numpy as np

from . import fft as _fft


class Basis:
    def __init__(self, cell, grid, ecut):
        self.cell = np.asarray(cell, dtype=np.float64)
        self.grid = tuple(int(g) for g in grid)
        self.ecut = float(ecut)
        self.omega = float(np.prod(self.cell))
        self.n_r = int(np.prod(self.grid))
        N = np.array(self.grid)
        # every n that could be in the sphere, to check it fits the grid
        big = [np.arange(-n, n + 1) for n in N]
        m = np.array(np.meshgrid(*big, indexing="ij")).reshape(3, -1).T
        g = 2 * np.pi * m / self.cell
        inside = 0.5 * (g * g).sum(1) <= self.ecut
        ok = (2 * np.abs(m) < N).all(1)
        if (inside & ~ok).any():
            raise ValueError("sphere does not fit strictly inside the grid")
        m = m[inside]
        half = np.array([self._positive(x) for x in m], dtype=bool)
        mh = m[half]
        key = np.lexsort((mh[:, 2], mh[:, 1], mh[:, 0], (mh * mh).sum(1)))
        self.mill_half = mh[key]                           # [n_half][3]
        self.n_half = len(self.mill_half)
        self.n_pw = 1 + 2 * self.n_half
        mill = np.zeros((self.n_pw, 3), dtype=np.int64)
        kind = np.zeros(self.n_pw, dtype=np.int8)
        mill[1::2] = self.mill_half
        mill[2::2] = self.mill_half
        kind[1::2] = 1
        kind[2::2] = 2
        self.miller = mill                                  # per basis function
        self.kind = kind                                    # 0 G0, 1 cos, 2 sin
        gv = 2 * np.pi * mill / self.cell
        self.gvec = gv                                      # [n_pw][3]
        self.g2 = (gv * gv).sum(1)                          # |G|^2 per function
        # grid indices (n mod N) of +G and -G for the half sphere
        self.idx_p = tuple((self.mill_half % N).T)
        self.idx_m = tuple(((-self.mill_half) % N).T)
        # minimum-image frequencies of the full grid
        f = [np.fft.fftfreq(n, 1.0 / n) for n in N]
        n1, n2, n3 = np.meshgrid(*f, indexing="ij")
        self.grid_n = np.stack([n1, n2, n3])                # [3][N1][N2][N3]
        self.grid_g = 2 * np.pi * self.grid_n / self.cell[:, None, None, None]
        self.grid_g2 = (self.grid_g ** 2).sum(0)
        nyq = np.zeros(self.grid, dtype=bool)
        for ax in range(3):
            if N[ax] % 2 == 0:
                nyq |= self.grid_n[ax] == -(N[ax] // 2)
        self.nyquist = nyq

    @staticmethod
    def _positive(m):
        for x in m:
            if x != 0:
                return x > 0
        return False

    # ---- grid transforms (numpy FFT) ------------------------------------
    def coeffs(self, x):
        """Complex Fourier coefficients on the full grid of the real basis
        expansion x[..., n_pw]:  f(0) = x0/sqrt(Omega),
        f(+G) = (xc - i xs)/sqrt(2 Omega),  f(-G) = conj(f(+G))."""
        x = np.asarray(x, dtype=np.float64)
        lead = x.shape[:-1]
        F = np.zeros(lead + self.grid, dtype=np.complex128)
        F[(...,) + (0, 0, 0)] = x[..., 0] / np.sqrt(self.omega)
        fp = (x[..., 1::2] - 1j * x[..., 2::2]) / np.sqrt(2 * self.omega)
        F[(...,) + self.idx_p] = fp
        F[(...,) + self.idx_m] = np.conj(fp)
        return F

    def to_grid(self, x):
        """Real-space values f(r_j) of x[..., n_pw] on the grid."""
        F = self.coeffs(x)
        f = _fft.ifftn(F, axes=(-3, -2, -1)) * self.n_r
        return f.real.copy()

    def from_grid(self, g):
        """Projection <e_k|g> (grid quadrature) of real grid values g."""
        G = _fft.fftn(np.asarray(g, dtype=np.float64), axes=(-3, -2, -1)) / self.n_r
        return self.from_coeffs(G)

    def from_coeffs(self, G):
        lead = G.shape[:-3]
        x = np.empty(lead + (self.n_pw,), dtype=np.float64)
        x[..., 0] = np.sqrt(self.omega) * G[(...,) + (0, 0, 0)].real
        gp = G[(...,) + self.idx_p]
        x[..., 1::2] = np.sqrt(2 * self.omega) * gp.real
        x[..., 2::2] = -np.sqrt(2 * self.omega) * gp.imag
        return x

    # ---- explicit basis matrix (independent route, small systems) -------
    def basis_matrix(self):
        """E[j][k] = e_k(r_j) built from cos/sin directly (no FFT)."""
        N = np.array(self.grid)
        j = np.array(np.meshgrid(*[np.arange(n) for n in N], indexing="ij")).reshape(3, -1).T
        phase = 2 * np.pi * (j / N) @ self.miller.T.astype(np.float64)   # G.r_j
        E = np.empty((self.n_r, self.n_pw))
        E[:, 0] = 1.0 / np.sqrt(self.omega)
        E[:, self.kind == 1] = np.sqrt(2 / self.omega) * np.cos(phase[:, self.kind == 1])
        E[:, self.kind == 2] = np.sqrt(2 / self.omega) * np.sin(phase[:, self.kind == 2])
        return E

    def grid_points(self):
        N = np.array(self.grid)
        j = np.array(np.meshgrid(*[np.arange(n) for n in N], indexing="ij")).reshape(3, -1).T
        return j / N * self.cell
