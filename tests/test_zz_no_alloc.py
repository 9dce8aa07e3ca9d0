"""bse_forces_noalloc against bse_forces, through the C ABI.

The allocation-free entry point must give the forces of the allocating one
(FP64; only the GEMM reduction order differs: 1e-10 of the largest
component asserted).  Two calls in a row on one device share the static
scratch: first the 24^3 system with 16 occupied orbitals, then the 12^3
system with 4, whose call must not see anything the first left behind.
"""
import numpy as np
import pytest

import synth
from oracle import basis, model, solvers

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2607_20728_amd import bsex  # noqa: E402


def _case(name):
    cfg = synth.get_config(name)
    b = basis.Basis(cfg.cell, cfg.grid, cfg.ecut)
    d = synth.make_system(cfg, b.n_pw)
    S = model.System(b, d["site_xyz"], d["site_depth"], d["site_width"], d["pdep"], d["lam"],
                     cfg.n_val)
    S.ground_state(n_extra=8)
    w, X, _ = solvers.davidson(S, 1, tol=1e-10)
    Z, _ = solvers.zvector_cg(S, solvers.u_vector(S, X[0]), tol=1e-10)
    return S, d, X[0], Z


def test_forces_noalloc_matches_forces_two_calls():
    for name in ("c1", "m0"):
        print(f"[gpu] forces_noalloc {name}", flush=True)
        S, d, Xs, Zs = _case(name)
        ctx = bsex.init_from_synth(d, orbitals=np.vstack([S.phi, S.psi_c]),
                                   eps=np.concatenate([S.eps, S.eps_c]))
        Xd = torch.tensor(Xs, dtype=torch.float64, device="cuda")
        Zd = torch.tensor(Zs, dtype=torch.float64, device="cuda")
        ref = bsex.forces(ctx, Xd, Zd, S.n_sites)
        out = torch.full((S.n_sites, 3), float("nan"), dtype=torch.float64, device="cuda")
        bsex.forces_noalloc(ctx, Xd, Zd, out)
        torch.cuda.synchronize()
        F = out.cpu().numpy()
        err = np.abs(F - ref).max() / np.abs(ref).max()
        print(f"  max |F_noalloc - F| / max |F| = {err:.2e}", flush=True)
        assert np.isfinite(F).all() and err < 1e-10
        # the oracle's own force contraction of the same vectors
        assert np.abs(F - solvers.dwdR(S, Xs, Zs)).max() < 1e-8
        ctx.free()
