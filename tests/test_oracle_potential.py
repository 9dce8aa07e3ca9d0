"""Pin of the oracle's Gaussian-site potential against its real-space
definition.

The synthetic Hamiltonian's sites are V_I(r) = -D_I exp(-|r - R_I|^2/(2 w_I^2)),
repeated periodically.  The oracle builds V in G space on the grid's
frequencies (minimum image, Nyquist planes zero) and transforms it back.  Here
that grid potential is compared, point by point, with the direct sum of the
Gaussians over their periodic images, evaluated without any transform.

The two differ only by the Fourier components the grid cannot hold (|n_i| >=
N_i/2 in some direction, and the Nyquist planes the model zeroes).  Their sum
is bounded by sum_{G outside} |V_I(G)|, computed below from the Gaussian's
continuous transform over a box three times the grid; on a fine grid that
bound is far below 1e-10, so a wrong normalisation (1/Omega or
(2 pi w^2)^(3/2)), a w^2 / 2 w^2 slip, a sign error in exp(-i G.R) or a
transposed axis would fail by orders of magnitude.
"""
import itertools

import numpy as np
import pytest

import synth
from oracle import basis, model


def _direct_sum(b, xyz, depth, width):
    """sum_I sum_T -D_I exp(-|r_j - R_I - T|^2/(2 w_I^2)) at every grid point,
    over the lattice translations T that reach within 9 widths."""
    r = b.grid_points()                                   # [n_r][3]
    L = b.cell
    out = np.zeros(len(r))
    for R, D, w in zip(xyz, depth, width):
        reach = 9.0 * w
        ranges = [range(-int(np.ceil(reach / L[a])) - 1, int(np.ceil(reach / L[a])) + 2)
                  for a in range(3)]
        for t in itertools.product(*ranges):
            d = r - (R + np.array(t) * L)
            out += -D * np.exp(-(d * d).sum(1) / (2.0 * w * w))
    return out.reshape(b.grid)


def _alias_bound(b, depth, width):
    """sum over frequencies the grid model drops of |V_I(G)|, for a box of
    3 N_i frequencies in each direction (the tail beyond it is negligible
    against the terms kept)."""
    N = np.array(b.grid)
    f = [np.arange(-3 * n // 2, 3 * n // 2) for n in N]
    n1, n2, n3 = np.meshgrid(*f, indexing="ij")
    kept = (2 * np.abs(n1) < N[0]) & (2 * np.abs(n2) < N[1]) & (2 * np.abs(n3) < N[2])
    g2 = sum((2 * np.pi * n / L) ** 2 for n, L in zip((n1, n2, n3), b.cell))
    tot = 0.0
    for D, w in zip(depth, width):
        amp = (D / b.omega) * (2 * np.pi * w * w) ** 1.5 * np.exp(-0.5 * w * w * g2)
        tot += amp[~kept].sum()
    return tot


def _check(cell, grid, xyz, depth, width, ecut=1.0):
    b = basis.Basis(cell, grid, ecut)
    pdep = np.zeros((b.n_pw, 1))
    S = model.System(b, xyz, depth, width, pdep, np.zeros(1), 1)
    direct = _direct_sum(b, np.asarray(xyz).reshape(-1, 3), depth, width)
    bound = _alias_bound(b, depth, width)
    err = np.abs(S.Vr - direct).max()
    print(f"grid {grid}: max |V_grid - V_direct| {err:.3e}, alias bound {bound:.3e}, "
          f"max |V| {np.abs(direct).max():.3f}")
    assert err <= bound + 1e-13 * np.abs(direct).max()
    return err, bound


def test_site_potential_matches_real_space_c1_cell():
    """The tiny system's own cell, grid and sites (cubic 10 bohr, 24^3)."""
    cfg = synth.get_config("c1")
    b = basis.Basis(cfg.cell, cfg.grid, cfg.ecut)
    d = synth.make_system(cfg, b.n_pw)
    err, bound = _check(cfg.cell, cfg.grid, d["site_xyz"], d["site_depth"], d["site_width"])
    assert bound < 1e-7


def test_site_potential_matches_real_space_orthorhombic_fine_grid():
    """Three unequal cell lengths on a grid fine enough that the aliasing
    bound is ~1e-13: the G-space form must equal the real-space sum."""
    rng = np.random.default_rng(31)
    cell = (7.0, 9.0, 11.0)
    xyz = rng.random((3, 3)) * np.array(cell)
    depth = rng.uniform(1.0, 3.0, 3)
    width = rng.uniform(0.8, 1.5, 3)
    err, bound = _check(cell, (36, 44, 56), xyz, depth, width)
    assert bound < 1e-10


def test_site_potential_matches_real_space_slab_cell():
    """The slab's cell and 48 x 48 x 120 grid (vacuum along z) with the
    substitution pair and four other sites of the layer."""
    cfg = synth.get_config("c5")
    b = basis.Basis(cfg.cell, cfg.grid, 1.0)
    d = synth.make_system(cfg, b.n_pw)
    pick = np.array([108, 109, 0, 3, 57, 199])
    _check(cfg.cell, cfg.grid, d["site_xyz"][pick], d["site_depth"][pick],
           d["site_width"][pick])


@pytest.mark.parametrize("flip", ["sign", "width", "volume"])
def test_planted_mistakes_fail_the_real_space_pin(flip, monkeypatch):
    """The pin is sharp: each plausible slip in V_I(G) exceeds the bound."""
    rng = np.random.default_rng(32)
    cell = (7.0, 9.0, 11.0)
    xyz = rng.random((2, 3)) * np.array(cell)
    depth, width = np.array([2.0, 1.5]), np.array([1.0, 1.2])
    orig = model.System.site_potential_G

    def wrong(self, i):
        b = self.b
        d, w, R = self.site_depth[i], self.site_width[i], self.site_xyz[i]
        gr = np.tensordot(R, b.grid_g, axes=(0, 0))
        amp = -(d / b.omega) * (2 * np.pi * w * w) ** 1.5
        e = np.exp(-0.5 * w * w * b.grid_g2)
        ph = np.exp(-1j * gr)
        if flip == "sign":
            ph = np.exp(1j * gr)
        elif flip == "width":
            e = np.exp(-w * w * b.grid_g2)
        elif flip == "volume":
            amp = amp * b.omega
        v = amp * e * ph
        v[b.nyquist] = 0.0
        return v

    monkeypatch.setattr(model.System, "site_potential_G", wrong)
    with pytest.raises(AssertionError):
        _check(cell, (36, 44, 56), xyz, depth, width)
    monkeypatch.setattr(model.System, "site_potential_G", orig)
    _check(cell, (36, 44, 56), xyz, depth, width)
