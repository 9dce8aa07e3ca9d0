"""Seeded synthetic inputs shared by the FP64 oracle and the HIP library.

This module draws random numbers and lays out input arrays.  It holds none of
the method's arithmetic: no basis, no Hamiltonian, no FFT, no kernel.  Every
consumer computes the plane-wave basis size itself and passes it in.

The systems stand in for the paper's workloads (which need pseudopotentials,
DFT ground states and PDEP bases that are not available): a periodic cell with
attractive Gaussian sites replaces the crystal, and a random orthonormal
G-space basis with prescribed eigenvalues replaces the PDEP eigenpotentials of
the screened interaction W (Eq. 3).

Draw order from one ``numpy.random.Generator(PCG64(seed))`` stream:
site positions -> displacements (if any) -> depths -> widths (random site
model only) -> PDEP Gaussian matrix -> trial block.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = ["Config", "CONFIGS", "get_config", "make_system", "diamond_sites",
           "honeycomb_sites", "c5_geometry", "c4_systems", "C4_GRIDS", "random_orbitals"]


@dataclasses.dataclass(frozen=True)
class Config:
    name: str
    cell: tuple            # orthorhombic lengths (bohr)
    grid: tuple            # FFT grid
    ecut: float            # Ha, sphere |G|^2/2 <= ecut
    n_val: int             # occupied orbitals N_v
    n_pdep: int            # PDEP rank
    lam_scale: float       # lambda_i = lam_scale * exp(-i / lam_decay), i = 0..n_pdep-1
    lam_decay: float
    sites: str             # "uniform:<n>", "diamond:<cells>", "honeycomb"
    depth: tuple = (1.0, 3.0)   # U(lo, hi) Ha
    width: tuple = (0.8, 1.5)   # U(lo, hi) bohr
    seed: int = 0
    n_states: int = 1      # excitons requested
    n_block: int = 8       # trial vectors per apply block in throughput runs
    # "random": depth ~ U(depth), width ~ U(width); "dimer": honeycomb
    # sublattices A / B with depths depth[0] / depth[1], width width[0], and one
    # nearest-neighbour A-B pair (the substitution) with depth 2.0, width 1.1
    site_model: str = "random"
    displace: float = 0.0  # sigma (bohr) of N(0, sigma) site displacements


CONFIGS = {
    # micro system for every dense check
    "m0": Config("m0", (8.0, 8.0, 8.0), (12, 12, 12), 4.0, 4, 8, -0.8, 2.0,
                 "uniform:3", seed=11),
    # tiny plain FP64 system: 8 random Gaussian sites, N_v = 16, N_pdep = 64
    "c1": Config("c1", (10.0, 10.0, 10.0), (24, 24, 24), 10.0, 16, 64, -0.8, 16.0,
                 "uniform:8", seed=1000),
    # 2-D slab: 10 x 5 rectangular honeycomb cells (200 sites, nearest
    # neighbours 2.733 bohr) in a 110-bohr cell along z; sublattice depths
    # 1.0 / 4.0 Ha give a Kohn-Sham gap of 0.034 Ha at N_v = 400 (1.5 / 2.5
    # leaves the layer semi-metallic: gap 1.3e-6 Ha)
    "c5": Config("c5", (47.34, 40.99, 110.0), (48, 48, 120), 3.26, 400, 768, -0.85, 144.0,
                 "honeycomb", depth=(1.0, 4.0), width=(1.0, 1.0), seed=5000,
                 site_model="dimer"),
    # defect supercell: 3x3x3 diamond cells (216 sites) with one removed; the
    # seed is the first from 2000 whose Kohn-Sham gap at N_v is >= 1e-3 Ha
    # (2000: 4.7e-4, 2001: 6.5e-4, 2002: 2.1e-3)
    "c2": Config("c2", (20.2, 20.2, 20.2), (72, 72, 72), 14.2, 432, 512, -0.85, 96.0,
                 "diamond:3", seed=2002, n_states=4, n_block=8),
}


def get_config(name: str) -> Config:
    return CONFIGS[name]


def c5_geometry(g: int) -> Config:
    """Geometry g of the slab family: the sites of c5 displaced by N(0, 0.05
    bohr), seed 5000 + g (g = 0 is the undisplaced slab)."""
    base = CONFIGS["c5"]
    return dataclasses.replace(base, name=f"c5g{g}", seed=5000 + g,
                               displace=0.05 if g > 0 else 0.0)


C4_GRIDS = (32, 40, 48, 64)


def c4_systems(n: int = 32, seed: int = 4000) -> list:
    """The uneven batch: n cubic systems with the spacing of c1 (L = 10 N / 24
    bohr, E_cut 10 Ha, 8 random sites), N drawn from C4_GRIDS, N_v from
    U{32..256}, N_pdep from U{128..384}, lambda_i = -0.8 exp(-i / (N_pdep / 4)).
    System k has seed seed + 1 + k."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for k in range(n):
        N = int(rng.choice(C4_GRIDS))
        nv = int(rng.integers(32, 257))
        npdep = int(rng.integers(128, 385))
        L = 10.0 * N / 24.0
        out.append(Config(f"c4s{k}", (L, L, L), (N, N, N), 10.0, nv, npdep, -0.8, npdep / 4.0,
                          "uniform:8", seed=seed + 1 + k))
    return out


def diamond_sites(cells: int, a: float, drop_origin: bool = True) -> np.ndarray:
    """Conventional diamond cells (8 sites each) tiled cells^3, optionally
    without the site at the origin (the vacancy)."""
    basis = np.array([[0, 0, 0], [0, .5, .5], [.5, 0, .5], [.5, .5, 0],
                      [.25, .25, .25], [.25, .75, .75], [.75, .25, .75],
                      [.75, .75, .25]])
    pts = []
    for i in range(cells):
        for j in range(cells):
            for k in range(cells):
                for b in basis:
                    pts.append((np.array([i, j, k]) + b) * a)
    pts = np.array(pts)
    if drop_origin:
        keep = np.linalg.norm(pts, axis=1) > 1e-12
        pts = pts[keep]
    return pts


def honeycomb_sites(nx: int, ny: int, nn: float, z: float) -> np.ndarray:
    """Rectangular honeycomb layer: nx x ny rectangular cells of 4 sites."""
    a = nn * math.sqrt(3.0)
    bx, by = a, 3.0 * nn
    base = np.array([[0, 0], [a / 2, nn / 2], [a / 2, 1.5 * nn], [0, 2 * nn]])
    pts = []
    for i in range(nx):
        for j in range(ny):
            for b in base:
                pts.append([i * bx + b[0], j * by + b[1], z])
    return np.array(pts)


def make_system(cfg: Config | str, n_pw: int, *, seed: int | None = None,
                n_trial: int = 0) -> dict:
    """Draw one synthetic system.

    n_pw     size of the plane-wave sphere, computed by the caller.
    n_trial  number of random trial vectors [n_trial][n_val][n_pw] (N(0,1)).

    Returns a dict of float64 arrays: cell, grid, ecut, site_xyz [n][3],
    site_depth [n], site_width [n], lam [n_pdep], pdep [n_pw][n_pdep]
    (orthonormal columns, row 0 -- the G = 0 coefficient -- zero), trial.
    """
    if isinstance(cfg, str):
        cfg = get_config(cfg)
    s = cfg.seed if seed is None else seed
    rng = np.random.Generator(np.random.PCG64(s))
    cell = np.array(cfg.cell, dtype=np.float64)
    kind, _, arg = cfg.sites.partition(":")
    if kind == "uniform":
        n = int(arg)
        xyz = rng.random((n, 3)) * cell
    elif kind == "diamond":
        cells = int(arg)
        xyz = diamond_sites(cells, cell[0] / cells)
    elif kind == "honeycomb":
        xyz = honeycomb_sites(10, 5, 2.733, cell[2] / 2)
    else:
        raise ValueError(cfg.sites)
    n_sites = xyz.shape[0]
    if cfg.displace > 0:
        xyz = xyz + rng.normal(0.0, cfg.displace, xyz.shape)
    if cfg.site_model == "dimer":
        # base sites 0 and 2 of each honeycomb cell are sublattice A, 1 and 3 B;
        # the substitution pair is sites 0 and 1 (nearest neighbours) of the
        # cell nearest the slab centre
        sub = np.arange(n_sites) % 2
        depth = np.where(sub == 0, cfg.depth[0], cfg.depth[1]).astype(np.float64)
        width = np.full(n_sites, cfg.width[0])
        c = (5 * 5 + 2) * 4
        depth[c:c + 2] = 2.0
        width[c:c + 2] = 1.1
    else:
        depth = rng.uniform(cfg.depth[0], cfg.depth[1], n_sites)
        width = rng.uniform(cfg.width[0], cfg.width[1], n_sites)
    lam = cfg.lam_scale * np.exp(-np.arange(cfg.n_pdep) / cfg.lam_decay)
    if cfg.n_pdep > n_pw - 1:
        raise ValueError("n_pdep must be below n_pw - 1")
    g = rng.standard_normal((n_pw, cfg.n_pdep))
    g[0, :] = 0.0
    q, r = np.linalg.qr(g)
    q = q * np.sign(np.diag(r))[None, :]
    q[0, :] = 0.0
    out = dict(cell=cell, grid=np.array(cfg.grid, dtype=np.int32),
               ecut=float(cfg.ecut), n_val=cfg.n_val,
               site_xyz=np.ascontiguousarray(xyz, dtype=np.float64),
               site_depth=depth, site_width=width, lam=lam,
               pdep=np.ascontiguousarray(q), seed=s)
    if n_trial:
        out["trial"] = rng.standard_normal((n_trial, cfg.n_val, n_pw))
    return out


def random_orbitals(n_pw: int, n_val: int, n_extra: int = 0, seed: int = 0):
    """A made-up orbital set for operator parity at sizes where no dense
    ground state is affordable: n_val + n_extra orthonormal rows [n][n_pw]
    (Householder QR of an N(0,1) matrix, diag(R) > 0) and ascending made-up
    energies, occupied in [-1, -0.3] Ha and the extra states in [0.1, 0.5] Ha.
    They are not eigenpairs of any Hamiltonian: the operator apply takes
    orbitals and energies as inputs and does not assume that."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = n_val + n_extra
    q, r = np.linalg.qr(rng.standard_normal((n_pw, n)))
    q = q * np.sign(np.diag(r))[None, :]
    eps = np.concatenate([np.linspace(-1.0, -0.3, n_val), np.linspace(0.1, 0.5, n_extra)])
    return np.ascontiguousarray(q.T), eps
