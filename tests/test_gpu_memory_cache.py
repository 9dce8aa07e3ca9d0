"""Device memory kept across contexts (bse_memory_cache): contexts built
from cached blocks give the results of freshly allocated ones, a smaller
system after a larger one reuses the cache, and turning the cache off
returns the memory."""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2607_20728_amd import bsex  # noqa: E402


def _system(name):
    cfg = synth.get_config(name)
    return synth.make_system(cfg, bsex.basis_size(cfg.cell, cfg.grid, cfg.ecut), n_trial=2)


def _apply(d):
    ctx = bsex.init_from_synth(d, n_extra=4)
    X = torch.tensor(d["trial"], dtype=torch.float64, device="cuda")
    Y = bsex.apply(ctx, X).cpu().numpy()
    w, _, _ = bsex.davidson(ctx, 1, tol=1e-10)
    ctx.free()
    return Y, w[0]


def test_contexts_from_cached_memory_match_fresh_ones():
    print("[gpu] memory cache across contexts: c1, m0", flush=True)
    d1, d0 = _system("c1"), _system("m0")
    ref1, w1 = _apply(d1)
    ref0, w0 = _apply(d0)
    bsex.memory_cache(True)
    try:
        for _ in range(2):                       # the second pass runs on cached blocks
            y1, v1 = _apply(d1)
            y0, v0 = _apply(d0)                  # smaller system after the larger one
            e1 = np.abs(y1 - ref1).max() / np.abs(ref1).max()
            e0 = np.abs(y0 - ref0).max() / np.abs(ref0).max()
            print(f"  apply {e1:.1e} {e0:.1e}  omega {abs(v1 - w1):.1e} {abs(v0 - w0):.1e}",
                  flush=True)
            assert e1 < 1e-13 and e0 < 1e-13
            assert abs(v1 - w1) < 1e-12 and abs(v0 - w0) < 1e-12
    finally:
        bsex.memory_cache(False)
    y1, _ = _apply(d1)                           # and after the cache is returned
    assert np.abs(y1 - ref1).max() < 1e-13 * np.abs(ref1).max()
