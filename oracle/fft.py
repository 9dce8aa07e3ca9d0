"""Discrete Fourier transforms of the oracle (test infrastructure).

Plain library FFTs (scipy's pocketfft) over the last three axes, threaded over
the batch on the host cores this process may use (capped by OMP_NUM_THREADS
when it is set).  Conventions are numpy's: fftn is sum_r f(r) e^{-iG.r},
ifftn is (1/N_r) sum_G f(G) e^{+iG.r}.
"""
from __future__ import annotations

import os

import numpy as np
import scipy.fft


def workers() -> int:
    """Host threads the oracle's transforms and timing legs use."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        n = os.cpu_count() or 1
    cap = os.environ.get("OMP_NUM_THREADS")
    if cap and cap.isdigit() and int(cap) > 0:
        n = min(n, int(cap))
    return max(1, n)


def fftn(x, axes=(-3, -2, -1)):
    return scipy.fft.fftn(np.asarray(x), axes=axes, workers=workers())


def ifftn(x, axes=(-3, -2, -1)):
    return scipy.fft.ifftn(np.asarray(x), axes=axes, workers=workers())
