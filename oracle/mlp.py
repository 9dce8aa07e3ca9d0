"""Plain FP64 NumPy reference of the learned preconditioner's network.

Test infrastructure only: the library never imports this module.

The network (no counterpart in the paper; the form is this project's): three
dense layers of width 128 with SiLU activations between them,

    xh = (x - mu_x) / s_x
    h1 = silu(xh W1^T + b1),  h2 = silu(h1 W2^T + b2),  yh = h2 W3^T + b3
    y  = yh * s_y + mu_y

trained on the weighted mean-squared error in normalised output space,

    L = sum_{n,o} w_no (yh_no - (t_no - mu_y,o) / s_y,o)^2 / max(sum w, 1),

with Adam (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected).  Parameters are
one flat vector in the order W1 [128][n_in], b1 [128], W2 [128][128], b2 [128],
W3 [n_out][128], b3 [n_out].

Parity pins (tests/test_oracle_mlp.py): gradients against central finite
differences of the loss, SiLU' against its closed form, and one Adam step
against the update written out for a single scalar.
"""
from __future__ import annotations

import numpy as np

WIDTH = 128
ADAM_B1, ADAM_B2, ADAM_EPS = 0.9, 0.999, 1e-8


def n_params(n_in: int, n_out: int, width: int = WIDTH) -> int:
    return width * n_in + width + width * width + width + n_out * width + n_out


def unpack(p, n_in, n_out, width=WIDTH):
    p = np.asarray(p, dtype=np.float64)
    o = 0
    shapes = [(width, n_in), (width,), (width, width), (width,), (n_out, width), (n_out,)]
    out = []
    for s in shapes:
        k = int(np.prod(s))
        out.append(p[o:o + k].reshape(s))
        o += k
    assert o == p.size
    return out


def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_grad(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(p, x, n_in, n_out, norm):
    """y [n][n_out] for x [n][n_in]; norm = (mu_x, s_x, mu_y, s_y)."""
    W1, b1, W2, b2, W3, b3 = unpack(p, n_in, n_out)
    mu_x, s_x, mu_y, s_y = norm
    xh = (np.asarray(x, np.float64) - mu_x) / s_x
    h1 = silu(xh @ W1.T + b1)
    h2 = silu(h1 @ W2.T + b2)
    return (h2 @ W3.T + b3) * s_y + mu_y


def loss_and_grad(p, x, t, w, n_in, n_out, norm):
    """Loss L and dL/dp (flat) by the chain rule of the layers above."""
    W1, b1, W2, b2, W3, b3 = unpack(p, n_in, n_out)
    mu_x, s_x, mu_y, s_y = norm
    x = np.asarray(x, np.float64)
    w = np.ones_like(t, dtype=np.float64) if w is None else np.asarray(w, np.float64)
    xh = (x - mu_x) / s_x
    z1 = xh @ W1.T + b1
    h1 = silu(z1)
    z2 = h1 @ W2.T + b2
    h2 = silu(z2)
    yh = h2 @ W3.T + b3
    th = (np.asarray(t, np.float64) - mu_y) / s_y
    den = max(w.sum(), 1.0)
    e = yh - th
    L = float((w * e * e).sum() / den)
    dy = 2.0 * w * e / den
    gW3 = dy.T @ h2
    gb3 = dy.sum(0)
    dh2 = dy @ W3
    dz2 = dh2 * silu_grad(z2)
    gW2 = dz2.T @ h1
    gb2 = dz2.sum(0)
    dh1 = dz2 @ W2
    dz1 = dh1 * silu_grad(z1)
    gW1 = dz1.T @ xh
    gb1 = dz1.sum(0)
    g = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])
    return L, g


def adam_step(p, g, m, v, t, lr):
    """One Adam update at step t (1-based); returns new (p, m, v)."""
    m = ADAM_B1 * m + (1.0 - ADAM_B1) * g
    v = ADAM_B2 * v + (1.0 - ADAM_B2) * g * g
    mh = m / (1.0 - ADAM_B1 ** t)
    vh = v / (1.0 - ADAM_B2 ** t)
    return p - lr * mh / (np.sqrt(vh) + ADAM_EPS), m, v
