"""Pins of the FP64 reference network (oracle/mlp.py) against finite
differences and closed forms, before it is used to check the GPU kernels."""
import numpy as np

from oracle import mlp


def _setup(n=37, n_in=8, n_out=2, seed=3):
    rng = np.random.default_rng(seed)
    p = rng.normal(0, 0.2, mlp.n_params(n_in, n_out))
    x = rng.normal(0, 1, (n, n_in)) * np.arange(1, n_in + 1) + 0.5
    t = rng.normal(0, 1, (n, n_out))
    w = rng.uniform(0, 1, (n, n_out))
    w[::5, 1] = 0.0
    norm = (x.mean(0), x.std(0), t.mean(0), t.std(0))
    return p, x, t, w, norm


def test_silu_grad_closed_form():
    z = np.linspace(-6, 6, 101)
    h = 1e-6
    fd = (mlp.silu(z + h) - mlp.silu(z - h)) / (2 * h)
    assert np.abs(fd - mlp.silu_grad(z)).max() < 1e-8
    assert mlp.silu(np.array([0.0]))[0] == 0.0


def test_gradient_matches_central_differences():
    n_in, n_out = 8, 2
    p, x, t, w, norm = _setup(n_in=n_in, n_out=n_out)
    L, g = mlp.loss_and_grad(p, x, t, w, n_in, n_out, norm)
    rng = np.random.default_rng(7)
    # every bias and a sample of weights in each layer
    sizes = [128 * n_in, 128, 128 * 128, 128, n_out * 128, n_out]
    offs = np.cumsum([0] + sizes)
    idx = []
    for k in range(6):
        pool = np.arange(offs[k], offs[k + 1])
        idx += list(pool if sizes[k] <= 128 else rng.choice(pool, 24, replace=False))
    h = 1e-6
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        Lp, _ = mlp.loss_and_grad(p + e, x, t, w, n_in, n_out, norm)
        Lm, _ = mlp.loss_and_grad(p - e, x, t, w, n_in, n_out, norm)
        fd = (Lp - Lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(g[i])), (i, fd, g[i])


def test_loss_zero_at_exact_targets_and_forward_consistent():
    n_in, n_out = 8, 2
    p, x, t, w, norm = _setup(n_in=n_in, n_out=n_out)
    y = mlp.forward(p, x, n_in, n_out, norm)
    L, g = mlp.loss_and_grad(p, x, y, w, n_in, n_out, norm)
    assert L < 1e-25 and np.abs(g).max() < 1e-12


def test_adam_first_step_is_signed_lr():
    # at t = 1 the bias-corrected step is lr * g / (|g| + eps) per component
    g = np.array([0.3, -2.0, 1e-3])
    p0 = np.array([1.0, 2.0, 3.0])
    p1, m, v = mlp.adam_step(p0, g, np.zeros(3), np.zeros(3), 1, 0.01)
    assert np.allclose(p1, p0 - 0.01 * g / (np.abs(g) + mlp.ADAM_EPS), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_committed_slab_network_loads_and_predicts():
    """The committed slab network (paper_2607_20728_amd/data/slab_c5_learned.npz,
    trained on 180 slab geometries): plain arrays only, the parameter count
    of an 8-128-128-2 network, finite positive standardisation, and finite
    predictions of moderate size for features drawn around the training
    means with the training spread."""
    import os
    path = os.path.join(os.path.dirname(__file__), "..", "paper_2607_20728_amd", "data",
                        "slab_c5_learned.npz")
    d = np.load(path)                                  # allow_pickle stays False
    assert set(d.files) == {"params", "mu_x", "s_x", "mu_y", "s_y"}
    assert d["params"].size == mlp.n_params(8, 2)
    for k in ("mu_x", "s_x", "mu_y", "s_y"):
        assert np.all(np.isfinite(d[k]))
    assert np.all(d["s_x"] > 0) and np.all(d["s_y"] > 0)
    rng = np.random.default_rng(0)
    x = d["mu_x"] + d["s_x"] * rng.standard_normal((256, 8))
    y = mlp.forward(d["params"], x, 8, 2, (d["mu_x"], d["s_x"], d["mu_y"], d["s_y"]))
    assert np.all(np.isfinite(y))
    assert np.abs(np.median(y, 0)).max() < 10
