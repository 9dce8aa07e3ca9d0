"""Training data, training and use of the learned preconditioner.

The network and its kernels live in the library (bse_mlp_*); this module only
drives them.  Targets come from histories of the plain method, obtained
through the C ABI:

* shift sigma_v*: the Z-vector PCG is run with each candidate shift applied
  to every band, recording the iteration at which each band's own residual
  reaches the tolerance (per-band steps make the bands independent); the
  target is the fastest candidate (ties go to the one nearest the default
  0.25 Ha), regressed as log(sigma_v*/0.25);
* initial-guess coefficient gamma_v*: the least-squares scalar along the
  preconditioned right-hand side, from a Z converged 1000x below the
  tolerance (bse_learned_features), regressed as log(max(gamma_v*, 1e-3)).

Each band gives two samples: the Z-vector one (all features) and a Davidson
one (the u-dependent features 5 and 6 and the flag 7 set to zero, gamma
weight zero), so one network serves both solvers.
"""
from __future__ import annotations

import numpy as np

from . import bsex

SHIFTS = (0.0625, 0.125, 0.25, 0.5, 1.0, 2.0)
DEFAULT_SHIFT = 0.25


def collect(ctx, Xs, *, tol=1e-6, shifts=SHIFTS, max_iter=0, two_level=False):
    """One geometry's training record from the plain solver on context ctx
    for the normalised exciton Xs [n_val][n_pw] (CUDA float64), under the
    preconditioner form the solves will use (two_level)."""
    nv = Xs.shape[0]
    its = []
    for s in shifts:
        _, st = bsex.zvector_solve(ctx, Xs, tol=tol, shifts=np.full(nv, float(s)),
                                   band_iters=True, max_iter=max_iter, two_level=two_level,
                                   check=False)
        bi = st["band_iters"].astype(np.float64)
        bi[bi < 0] = np.inf  # band not converged within max_iter
        its.append(bi)
    its = np.array(its)                                   # [n_shift][n_val]
    Zref, _ = bsex.zvector_solve(ctx, Xs, tol=min(tol * 1e-3, 1e-9), two_level=two_level)
    feat, gamma = bsex.learned_features(ctx, Xs, Zref, two_level=two_level)
    sh = np.asarray(shifts, dtype=np.float64)
    dist = np.abs(np.log(sh / DEFAULT_SHIFT))
    best = np.empty(nv)
    for v in range(nv):
        m = its[:, v].min()
        cand = np.flatnonzero(its[:, v] == m)
        best[v] = sh[cand[np.argmin(dist[cand])]]
    return dict(features=feat.astype(np.float32), log_sigma=np.log(best / DEFAULT_SHIFT),
                gamma=np.asarray(gamma, dtype=np.float64), band_iters=its, shifts=sh)


def log_gamma(g):
    return np.log(np.maximum(np.asarray(g, dtype=np.float64), 1e-3))


def training_arrays(records):
    """x [2N][8], t [2N][2], w [2N][2] (float32) from collect() records."""
    F = np.concatenate([r["features"] for r in records]).astype(np.float32)
    T = np.stack([np.concatenate([r["log_sigma"] for r in records]),
                  np.concatenate([log_gamma(r["gamma"]) for r in records])],
                 axis=1).astype(np.float32)
    Fd = F.copy()
    Fd[:, 5:8] = 0.0
    Wz = np.ones_like(T)
    Wd = np.ones_like(T)
    Wd[:, 1] = 0.0
    return (np.concatenate([F, Fd]), np.concatenate([T, T]),
            np.concatenate([Wz, Wd]).astype(np.float32))


def norm_stats(x, t, w):
    """Standardisation statistics (features, and targets over weighted rows)."""
    mu_x = x.mean(0)
    s_x = x.std(0)
    s_x[s_x < 1e-6] = 1.0
    mu_y = np.array([(t[:, o] * w[:, o]).sum() / max(w[:, o].sum(), 1.0)
                     for o in range(t.shape[1])])
    s_y = np.array([np.sqrt((w[:, o] * (t[:, o] - mu_y[o]) ** 2).sum() / max(w[:, o].sum(), 1.0))
                    for o in range(t.shape[1])])
    s_y[s_y < 1e-6] = 1.0
    return [np.asarray(a, np.float32) for a in (mu_x, s_x, mu_y, s_y)]


def train(records, *, steps=1500, lr=2e-3, seed=0, batch=4096, log=None):
    """Adam on the library's BF16 kernels: full batches when the data has at
    most `batch` rows, otherwise a fresh random mini-batch of `batch` rows
    each step (the weight-gradient products then stay short).  log(k, loss)
    is called every 250 steps.  Returns (net, norm, losses)."""
    import torch
    x, t, w = training_arrays(records)
    norm = norm_stats(x, t, w)
    net = bsex.Mlp(bsex.LEARN_NFEAT, bsex.LEARN_NOUT, seed=seed)
    net.set_norm(*norm)
    xd = torch.tensor(x, device="cuda")
    td = torch.tensor(t, device="cuda")
    wd = torch.tensor(w, device="cuda")
    n = x.shape[0]
    rng = np.random.default_rng(seed)
    losses = []
    for k in range(steps):
        if n > batch:
            idx = torch.tensor(rng.choice(n, batch, replace=False), device="cuda")
            losses.append(net.train_step(xd[idx].contiguous(), td[idx].contiguous(),
                                         wd[idx].contiguous(), lr=lr))
        else:
            losses.append(net.train_step(xd, td, wd, lr=lr))
        if log and (k % 250 == 0 or k == steps - 1):
            log(k, losses[-1])
    return net, norm, losses


def loss_of(net, norm, records):
    """Weighted mean squared error of the network on the records' samples
    (standardised targets, the training loss)."""
    import torch
    x, t, w = training_arrays(records)
    y = net.forward(torch.tensor(x, device="cuda")).cpu().numpy().astype(np.float64)
    err = (y - t) / norm[3]
    return float((w * err ** 2).sum() / max(w.sum(), 1.0))


def save(path, net, norm):
    np.savez(path, params=net.get_params(), mu_x=norm[0], s_x=norm[1], mu_y=norm[2], s_y=norm[3])


def load(path, seed=0):
    d = np.load(path)  # plain arrays only (allow_pickle stays False)
    net = bsex.Mlp(bsex.LEARN_NFEAT, bsex.LEARN_NOUT, seed=seed)
    net.set_params(d["params"])
    norm = [d["mu_x"], d["s_x"], d["mu_y"], d["s_y"]]
    net.set_norm(*norm)
    return net, norm


def predict(net, features):
    """(sigma_v, gamma_v) the solvers would use for these features."""
    import torch
    y = net.forward(torch.tensor(np.ascontiguousarray(features, np.float32),
                                 device="cuda")).cpu().numpy().astype(np.float64)
    return (DEFAULT_SHIFT * np.exp(np.clip(y[:, 0], -3, 3)), np.exp(np.clip(y[:, 1], -6, 8)))
