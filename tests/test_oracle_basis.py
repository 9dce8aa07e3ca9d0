"""Pins of the oracle's plane-wave basis and grid transforms.

The grid transforms use numpy FFTs; every check here compares them with the
explicit cos/sin basis matrix built from its definition, or with properties
the definition fixes (orthonormality under grid quadrature, ordering)."""
import numpy as np
import pytest

import synth
from oracle.basis import Basis


@pytest.mark.parametrize("name,npw", [("m0", 179), ("c1", 1503), ("c2", 21079)])
def test_sphere_sizes(name, npw):
    cfg = synth.get_config(name)
    b = Basis(cfg.cell, cfg.grid, cfg.ecut)
    assert b.n_pw == npw
    # the sphere holds exactly the G with |G|^2/2 <= ecut, each G once (+G, -G in cos/sin)
    assert (0.5 * b.g2 <= cfg.ecut + 1e-12).all()


def test_ordering_and_kinds():
    cfg = synth.get_config("c1")
    b = Basis(cfg.cell, cfg.grid, cfg.ecut)
    assert b.kind[0] == 0 and (b.miller[0] == 0).all()
    assert (b.kind[1::2] == 1).all() and (b.kind[2::2] == 2).all()
    assert (b.miller[1::2] == b.miller[2::2]).all()
    n2 = (b.mill_half ** 2).sum(1)
    assert (np.diff(n2) >= 0).all()
    for m in b.mill_half:                      # half sphere: first non-zero positive
        nz = m[m != 0]
        assert nz[0] > 0


def test_sphere_must_fit():
    with pytest.raises(ValueError):
        Basis((8.0, 8.0, 8.0), (6, 6, 6), 4.0)


@pytest.mark.parametrize("name", ["m0", "c1"])
def test_grid_transforms_match_explicit_basis(name):
    cfg = synth.get_config(name)
    b = Basis(cfg.cell, cfg.grid, cfg.ecut)
    E = b.basis_matrix()
    gram = (b.omega / b.n_r) * E.T @ E
    assert np.abs(gram - np.eye(b.n_pw)).max() < 1e-13
    x = np.random.default_rng(3).standard_normal((3, b.n_pw))
    f = b.to_grid(x).reshape(3, -1)
    assert np.abs(f - x @ E.T).max() < 1e-12 * np.abs(f).max()
    # projection of an arbitrary grid function equals the quadrature <e_k|g>
    g = np.random.default_rng(4).standard_normal((2,) + b.grid)
    p = b.from_grid(g)
    p2 = (b.omega / b.n_r) * g.reshape(2, -1) @ E
    assert np.abs(p - p2).max() < 1e-12 * np.abs(p2).max()
    assert np.abs(b.from_grid(b.to_grid(x)) - x).max() < 1e-13


def test_plane_wave_values():
    """c_G and s_G evaluated at a grid point from their closed forms."""
    cfg = synth.get_config("m0")
    b = Basis(cfg.cell, cfg.grid, cfg.ecut)
    k = 7                                      # some half-sphere vector
    r = b.grid_points()
    G = 2 * np.pi * b.mill_half[k] / b.cell
    x = np.zeros(b.n_pw)
    x[1 + 2 * k] = 1.0
    assert np.allclose(b.to_grid(x).reshape(-1), np.sqrt(2 / b.omega) * np.cos(r @ G), atol=1e-14)
    x[:] = 0
    x[2 + 2 * k] = 1.0
    assert np.allclose(b.to_grid(x).reshape(-1), np.sqrt(2 / b.omega) * np.sin(r @ G), atol=1e-14)
