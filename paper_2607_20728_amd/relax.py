"""Excited-state geometry relaxation of a synthetic system: the use the
paper puts its forces to (relaxed excited-state geometries and the
mass-weighted displacement Delta Q between the ground- and excited-state
minima).

The paper's excited-state force is the ground-state force minus d omega/d R
(the sentence introducing Eq. 4).  The synthetic model has no ion-ion term,
so on its own the occupied eigenvalue sum would pull the Gaussian sites
together without bound; each site is therefore tied to its starting position
by a harmonic spring of stiffness k (Ha/bohr^2).  The surfaces are

    E_GS(R) = f_occ sum_v eps_v(R) + k/2 sum_I |R_I - R_I^0|^2
    E_ES(R) = E_GS(R) + omega(R)

with the dielectric (PDEP) basis held fixed, as in the paper's finite-
difference protocol.  Every energy and gradient comes from the library
(bse_init_system, bse_davidson, bse_zvector_solve, bse_forces and
bse_ground_state_forces); this module only moves the sites, by BFGS with a
backtracking line search.
"""
from __future__ import annotations

import time

import numpy as np

from . import bsex


def evaluate(sysd, xyz, *, surface="es", spring=5.0, f_occ=2.0, tol=1e-9, n_extra=8,
             precision=bsex.FP64, state=None, two_level=False):
    """(E, dE/dR [n_sites][3]) of the ground- ("gs") or excited-state ("es")
    surface at site positions xyz, from a fresh context (two_level: the
    solves use the two-level preconditioner on the n_extra conduction states).

    state (a dict, optional) carries solver state between the geometries of
    a relaxation: with state["warm"] true (the default) the Davidson solve
    starts from the previous geometry's exciton and the Z-vector solve from
    its Z; the exciton and Z of this geometry are stored back, and the solver
    iterations are added to state["davidson_iters"], state["zvector_iters"]
    with state["evals"] counting the evaluations.

    Both pair each occupied band v with an orbital phi_v, whose sign (and,
    within a degenerate level, whose rotation) a fresh ground-state solve
    fixes arbitrarily.  The guesses are therefore re-expressed on this
    geometry's orbitals through the transition density matrix,
    a_v <- Delta rho_old phi_v = sum_v' <phi_v'^old|phi_v> a_v'^old (the same
    for Z), and the library then projects them onto the new conduction
    space."""
    if surface not in ("gs", "es"):
        raise ValueError(f"surface {surface!r}: 'gs' or 'es'")
    d = dict(sysd)
    d["site_xyz"] = np.ascontiguousarray(xyz, dtype=float)
    x0 = np.asarray(sysd["site_xyz"], dtype=float)
    n = x0.shape[0]
    t0 = time.perf_counter()
    ctx = bsex.init_from_synth(d, n_extra=n_extra, precision=precision)
    if state is not None:
        state["s_init"] = state.get("s_init", 0.0) + time.perf_counter() - t0
    try:
        phi, eps = bsex.get_orbitals(ctx)
        E = f_occ * float(np.sum(eps)) + 0.5 * spring * float(np.sum((d["site_xyz"] - x0) ** 2))
        G = f_occ * bsex.ground_state_forces(ctx, n) + spring * (d["site_xyz"] - x0)
        if surface == "es":
            warm = state is not None and state.get("warm", True)
            x0 = z0 = None
            phi_h = phi.cpu().numpy()
            if warm and state.get("X") is not None:
                import torch
                S = state["phi"] @ phi_h.T                    # <phi_v'^old|phi_v>
                x0 = torch.tensor((S.T @ state["X"])[None], dtype=torch.float64,
                                  device=phi.device)
                z0 = torch.tensor(S.T @ state["Z"], dtype=torch.float64, device=phi.device)
            t1 = time.perf_counter()
            w, X, ds = bsex.davidson(ctx, 1, tol=tol, x0=x0, two_level=two_level)
            t2 = time.perf_counter()
            Z, zs = bsex.zvector_solve(ctx, X[0], tol=tol, z0=z0, two_level=two_level)
            t3 = time.perf_counter()
            E += float(w[0])
            G = G + bsex.forces(ctx, X[0], Z, n)
            if state is not None:
                state["phi"] = phi_h
                state["X"], state["Z"] = X[0].cpu().numpy(), Z.cpu().numpy()
                state["davidson_iters"] = state.get("davidson_iters", 0) + ds["iters"]
                state["davidson_applies"] = state.get("davidson_applies", 0) + ds["applies"]
                state["zvector_iters"] = state.get("zvector_iters", 0) + zs["iters"]
                state["s_davidson"] = state.get("s_davidson", 0.0) + t2 - t1
                state["s_zvector"] = state.get("s_zvector", 0.0) + t3 - t2
        if state is not None:
            state["evals"] = state.get("evals", 0) + 1
    finally:
        ctx.free()
    return E, G


def bfgs(fun, x0, *, gtol=1e-5, max_steps=50, max_step=0.2):
    """Minimise fun(x) -> (f, grad) by BFGS on the inverse Hessian with an
    Armijo backtracking line search; steps are capped at max_step (bohr) per
    coordinate.  A line search that finds no decrease resets the Hessian to
    the identity and tries again from the same point; if that fails too the
    minimisation stops there (the energies carry no more information), so
    the accepted energies never increase.  Returns (x, f, grad, history of
    (f, |grad|_max))."""
    x = np.asarray(x0, dtype=float).copy()
    f, g = fun(x)
    H = np.eye(x.size)
    reset = True
    hist = [(f, float(np.abs(g).max()))]
    for _ in range(max_steps):
        if np.abs(g).max() < gtol:
            break
        p = -H @ g
        scale = max_step / max(np.abs(p).max(), 1e-300)
        if scale < 1.0:
            p *= scale
        slope = float(g @ p)
        if slope >= 0:  # not a descent direction: restart from steepest descent
            H = np.eye(x.size)
            p = -g * min(1.0, max_step / max(np.abs(g).max(), 1e-300))
            slope = float(g @ p)
        t = 1.0
        while True:
            xn = x + t * p
            fn, gn = fun(xn)
            if fn <= f + 1e-4 * t * slope:
                break
            t *= 0.5
            if t < 1e-4:
                xn = None
                break
        if xn is None:
            if reset:
                break
            H = np.eye(x.size)
            reset = True
            continue
        reset = False
        s, y = xn - x, gn - g
        sy = float(s @ y)
        if sy > 1e-12:
            rho = 1.0 / sy
            V = np.eye(x.size) - rho * np.outer(s, y)
            H = V @ H @ V.T + rho * np.outer(s, s)
        x, f, g = xn, fn, gn
        hist.append((f, float(np.abs(g).max())))
    return x, f, g, hist


def relax(sysd, *, surface="es", start=None, gtol=1e-5, max_steps=50, evaluator=None,
          keep_memory=None, **kw):
    """Relax the sites of a synth.make_system dict on one surface.
    evaluator(sysd, xyz, surface=..., **kw) -> (E, dE/dR) defaults to
    evaluate (the library).  keep_memory (default: with the library's own
    evaluator): the library keeps each geometry's device memory for the next
    (bse_memory_cache) while the relaxation runs.  Returns (xyz [n_sites][3],
    E, history)."""
    if keep_memory is None:
        keep_memory = evaluator is None
    ev = evaluator or evaluate
    x0 = np.asarray(sysd["site_xyz"] if start is None else start, dtype=float)
    shape = x0.shape

    def fun(x):
        E, G = ev(sysd, x.reshape(shape), surface=surface, **kw)
        return E, np.asarray(G, dtype=float).reshape(-1)

    if keep_memory:
        bsex.memory_cache(True)
    try:
        x, E, _, hist = bfgs(fun, x0.reshape(-1), gtol=gtol, max_steps=max_steps)
    finally:
        if keep_memory:
            bsex.memory_cache(False)
    return x.reshape(shape), E, hist


def delta_q(xyz_a, xyz_b, masses=None):
    """Mass-weighted displacement sqrt(sum_I M_I |R_I^a - R_I^b|^2) (unit
    masses when none are given)."""
    d2 = np.sum((np.asarray(xyz_a) - np.asarray(xyz_b)) ** 2, axis=1)
    m = np.ones_like(d2) if masses is None else np.asarray(masses, dtype=float)
    return float(np.sqrt(np.sum(m * d2)))
