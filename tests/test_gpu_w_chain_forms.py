"""The three forms of the W-build chain give the same results.

The pair grids of the tau build (Eq. 2c with W of Eq. 3), of the U vector
and of the coupling beyond the TDA go through one chain: pair products,
forward FFT, bare Coulomb multiply, PDEP projection, inverse FFT.  The
library forms the pair products inside the first pass of the forward FFT
and takes the multiply and the PDEP sphere entries in its last pass (the
default), or only the latter (BSEX_W_PAIRS=0), or runs the separate
kernels (BSEX_W_FUSED=0).  Each form runs in its own process (the switches
are read once) on C1 with every tau block rebuilt in every apply, in FP64
and in the mixed form; the apply, the U vector and the coupling apply must
agree to rounding (1e-13 relative in FP64, 1e-6 in the mixed form, whose
FP32 tau varies with the order of its FP64 LDS sums).  Each result is also
checked against the oracle in the other GPU tests.
"""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import sys
import numpy as np
import torch
import synth
from paper_2607_20728_amd import bsex
out, prec = sys.argv[1], sys.argv[2]
cfg = synth.get_config("c1")
d = synth.make_system(cfg, bsex.basis_size(cfg.cell, cfg.grid, cfg.ecut), n_trial=2)
kw = dict(tau_policy=bsex.TAU_REBUILD)
if prec == "mixed":
    kw = dict(precision=bsex.MIXED)
ctx = bsex.init_from_synth(d, **kw)
X = torch.tensor(np.ascontiguousarray(d["trial"]), dtype=torch.float64, device="cuda")
Y = bsex.apply(ctx, X).cpu().numpy()
U = bsex.u_vector(ctx, X[0]).cpu().numpy()
res = dict(Y=Y, U=U)
if prec == "fp64":
    res["B"] = bsex.apply_coupling(ctx, X).cpu().numpy()
ctx.free()
np.savez(out, **res)
print("done", out, flush=True)
"""


def _run(tmp_path, prec, pairs, fused):
    env = dict(os.environ, BSEX_W_PAIRS=str(pairs), BSEX_W_FUSED=str(fused))
    env["PYTHONPATH"] = os.pathsep.join([ROOT, env.get("PYTHONPATH", "")])
    out = str(tmp_path / f"{prec}_{pairs}{fused}.npz")
    print(f"[gpu] W chain form: {prec}, BSEX_W_PAIRS={pairs} BSEX_W_FUSED={fused}", flush=True)
    r = subprocess.run([sys.executable, "-c", CHILD, out, prec], env=env, cwd=ROOT,
                       capture_output=True, text=True, timeout=240)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-2000:]
    return dict(np.load(out))


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-13), ("mixed", 1e-6)])
def test_w_chain_forms_agree(tmp_path, prec, tol):
    ref = _run(tmp_path, prec, 0, 0)
    for pairs, fused in ((0, 1), (1, 1)):
        got = _run(tmp_path, prec, pairs, fused)
        errs = {k: _rel(got[k], ref[k]) for k in ref}
        print(f"  pairs={pairs} fused={fused}: " + json.dumps({k: f"{v:.1e}" for k, v in
                                                              errs.items()}), flush=True)
        assert all(v < tol for v in errs.values()), errs
