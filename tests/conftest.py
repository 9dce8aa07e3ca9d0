import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) to run")
    config.addinivalue_line("markers", "slow: long CPU-only check")


def _oracle_system(name, n_extra=8, kmask=None, seed=None, **kw):
    import numpy as np  # noqa: F401
    import synth
    from oracle import basis, model
    cfg = synth.get_config(name)
    b = basis.Basis(cfg.cell, cfg.grid, cfg.ecut)
    d = synth.make_system(cfg, b.n_pw, seed=seed)
    S = model.System(b, d["site_xyz"], d["site_depth"], d["site_width"], d["pdep"],
                     d["lam"], cfg.n_val,
                     kmask=model.K_ALL if kmask is None else kmask, **kw)
    S.ground_state(n_extra=n_extra)
    return S, d


@pytest.fixture(scope="session")
def m0_solved():
    """Micro system, ground state, 3 lowest excitons, U, Z for exciton 1."""
    from oracle import solvers
    S, d = _oracle_system("m0")
    om, X, info = solvers.davidson(S, n_states=3, tol=1e-11, max_iter=300)
    assert info["converged"]
    U = solvers.u_vector(S, X[0])
    Z, zi = solvers.zvector_cg(S, U, tol=1e-12)
    assert zi["converged"]
    return dict(S=S, d=d, omega=om, X=X, U=U, Z=Z)


@pytest.fixture(scope="session")
def c1_solved():
    """The 24^3 system with 16 occupied orbitals: Davidson to 1e-8, Z to 1e-8."""
    from oracle import solvers
    S, d = _oracle_system("c1")
    om, X, info = solvers.davidson(S, n_states=1, tol=1e-8, max_iter=300)
    assert info["converged"]
    U = solvers.u_vector(S, X[0])
    Z, zi = solvers.zvector_cg(S, U, tol=1e-8)
    assert zi["converged"]
    return dict(S=S, d=d, omega=om, X=X, U=U, Z=Z, zinfo=zi, dinfo=info)
