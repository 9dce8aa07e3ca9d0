#!/usr/bin/env python3
"""Throughput of the DMPT BSE operator apply (A.X applications per second).

One step = one bse_apply of a block of N_b = 8 trial vectors on the defect
supercell workload: cubic 20.2 bohr cell, 72^3 grid, 21,079 plane waves,
N_v = 432 occupied orbitals, N_pdep = 512, 215 Gaussian sites on a 3x3x3
diamond lattice with one site removed, plain FP64.  The ground state is
solved on the device first (Chebyshev-filtered subspace iteration); the
pair potentials tau = W(phi_v phi_v') are cached as far as device memory
allows and the rest are rebuilt inside every apply (part of the timed work).

Prints ONE JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HERE = os.path.dirname(os.path.abspath(__file__))
HBM_PEAK_GBS = 8000.0
METRIC = "A·X applies/s at N_v=432"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def pair_count(nv, blocks):
    """Unordered occupied pairs (v <= v') inside a list of 8x8 blocks (I, J)."""
    n = 0
    for I, J in blocks:
        for i in range(8):
            for j in range(8):
                v, w = 8 * I + i, 8 * J + j
                if v < nv and w < nv and (I < J or i <= j):
                    n += 1
    return n


def cpu_model():
    """The host CPU's model name (Linux /proc/cpuinfo), or 'unknown'."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(cfg_name, n_b):
    """The FP64 oracle timed on a bounded sample of one apply block, on every
    host core this process may use (transforms and BLAS threaded).

    Sample: the full per-vector work of ONE trial vector (projector, the N_v
    inverse and forward grid transforms, K1e, the diagonal term), plus
    tau_{v'v} = W(phi_v' phi_v) for every v' of ONE output band v (N_v pairs:
    a whole band row of the pair matrix) and its contraction with one
    vector's a(r).  The block is extrapolated as
        n_b t_vector + (P / N_v) (t_band_tau + n_b t_band_contract),
    P = N_v (N_v + 1)/2 pairs.  Orbitals are a random orthonormal set with
    made-up energies (the apply does the same work for any orbitals).
    """
    from threadpoolctl import threadpool_limits

    import synth
    from oracle import basis, model
    from oracle.fft import workers
    nw = workers()
    cfg = synth.get_config(cfg_name)
    b = basis.Basis(cfg.cell, cfg.grid, cfg.ecut)
    d = synth.make_system(cfg, b.n_pw, n_trial=1)
    nv = cfg.n_val
    with threadpool_limits(limits=nw):
        S = model.System(b, d["site_xyz"], d["site_depth"], d["site_width"], d["pdep"],
                         d["lam"], nv)
        orbs, eps = synth.random_orbitals(b.n_pw, nv, 0, seed=7)
        S.set_orbitals(orbs, eps)
        X = d["trial"][0]
        t0 = time.perf_counter()
        A = S.proj_c(X)
        ar = b.to_grid(A)
        z = S.Vr * ar
        drho = (S.phir * ar).sum(0)
        z += S.spin * S.poisson(drho) * S.phir
        Z = b.from_grid(z) + (S.T[None, :] - S.eps[:, None]) * A
        S.proj_c(Z)
        t_vec = time.perf_counter() - t0
        v = nv // 2
        t1 = time.perf_counter()
        tau = S.apply_W(S.phir * S.phir[v])          # tau_{v'v} for every v'
        t_tau = time.perf_counter() - t1
        t2 = time.perf_counter()
        np.einsum("uxyz,uxyz->xyz", tau, ar)          # y_v = sum_v' tau_{v'v} a_v'
        t_con = time.perf_counter() - t2
    n_pairs = nv * (nv + 1) // 2
    rows = n_pairs / nv
    t_block = n_b * t_vec + rows * (t_tau + n_b * t_con)
    return dict(value=n_b / t_block, unit="applies/s", cores=nw, kind="oracle",
                cpu=cpu_model(),
                sample=(f"1 vector's full work without K1d ({t_vec:.2f} s) + tau for all {nv} "
                        f"pairs of one output band ({t_tau:.2f} s) and its contraction with "
                        f"one vector ({t_con:.2f} s); block of {n_b} extrapolated to "
                        f"{t_block:.0f} s with {n_pairs} pairs"))


def stream_kernel_sha():
    """Hash of the tau-stream kernel's source: traffic counters taken on an
    older kernel are not reported."""
    import hashlib
    src = open(os.path.join(HERE, "paper_2607_20728_amd", "csrc", "kernels.hip")).read()
    a = src.index("// LDS rows (one per orbital v)")
    b = src.index("// potential, Coulomb kernel, forces")
    return hashlib.sha256(src[a:b].encode()).hexdigest()[:16]


def stream_traffic(mixed):
    """HBM bytes per k_tau_stream launch from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE runs, scaled by the same counters on a plain
    copy of known size), or None when absent or taken on another kernel."""
    f = os.path.join(HERE, "profiles", f"traffic_tau_stream_{'f32' if mixed else 'f64'}.json")
    if not os.path.exists(f):
        return None
    d = json.load(open(f))
    if d.get("source_sha") != stream_kernel_sha():
        return None
    return (d["fetch_kib_per_launch"] * d["copy_fetch_factor"] +
            d["write_kib_per_launch"] * d["copy_write_factor"]) * 1024.0


def loc_kw(args):
    """Wannier-localised pruning options of the library (--prune T)."""
    if args.prune is None:
        return {}
    return dict(localize=1, prune_threshold=args.prune, loc_max_sweeps=args.loc_sweeps)


def loc_info(info):
    return dict(threshold=None, tau_blocks_kept=info["tau_blocks"],
                tau_blocks_all=info["tau_blocks_all"], spread_bohr2=info["loc_spread"],
                sweeps=info["loc_sweeps"])


def copy_rate(n_bytes=4 << 30, reps=5):
    """Measured device-to-device copy rate (read + write bytes per second) of
    a plain torch copy of n_bytes, the practical HBM ceiling beside the 8
    TB/s peak."""
    import torch
    n = n_bytes // 8
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        y.copy_(x)
    e1.record()
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) / 1e3 / reps
    del x, y
    return dict(gbs=round(2 * 8 * n / t / 1e9, 1), bytes_per_copy=2 * 8 * n,
                frac_of_peak=round(2 * 8 * n / t / 1e9 / HBM_PEAK_GBS, 4))


def read_rate(n_bytes=4 << 30, reps=5):
    """Measured read rate of the device: torch's sum over n_bytes of float64
    (a read-only stream, the practical ceiling of a kernel that mostly
    reads)."""
    import torch
    x = torch.ones(n_bytes // 8, dtype=torch.float64, device="cuda")
    x.sum()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        x.sum()
    e1.record()
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) / 1e3 / reps
    del x
    return dict(gbs=round(n_bytes / t / 1e9, 1), bytes_per_read=n_bytes,
                frac_of_peak=round(n_bytes / t / 1e9 / HBM_PEAK_GBS, 4))


def copy_calibration(args):
    """A plain device copy of known size, for scaling the FETCH_SIZE and
    WRITE_SIZE counters: each launch reads and writes 2 GiB."""
    import torch
    torch.cuda.set_device(0)
    n = 2 ** 28  # 2 GiB of float64
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(args.steps):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps(dict(copy_bytes_read=8 * n, copy_bytes_written=8 * n,
                          launches=args.steps)), flush=True)


def config_of(name):
    """A named configuration, or system k of the uneven batch as "c4s<k>"."""
    import synth
    if name.startswith("c4s"):
        return synth.c4_systems()[int(name[3:])]
    return synth.get_config(name)


def beyond_tda(args):
    """Beyond the TDA on one system (default the defect supercell): the
    coupling apply P_c (s K2e - K2d) P_c X timed on --nb vectors after one
    warm-up, then (--full-bse) the lowest root of the coupled problem to
    --tol, with the TDA root of the same context for comparison."""
    import torch

    import synth
    from paper_2607_20728_amd import bsex

    torch.cuda.set_device(0)
    cfg = config_of(args.config)
    n_pw = bsex.basis_size(cfg.cell, cfg.grid, cfg.ecut)
    d = synth.make_system(cfg, n_pw, n_trial=args.nb, seed=args.seed)
    ctx = bsex.init_from_synth(d, n_extra=args.n_extra, gs_tol=1e-10)
    X = torch.tensor(d["trial"], dtype=torch.float64, device="cuda")
    Y = torch.empty_like(X)
    bsex.apply_coupling(ctx, X[:1], Y[:1])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bsex.apply_coupling(ctx, X, Y)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    log(f"[coupling] {cfg.name}: {dt / args.nb:.4f} s per vector")
    # the TDA apply of the same block, for scale
    bsex.apply(ctx, X, Y)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bsex.apply(ctx, X, Y)
    torch.cuda.synchronize()
    dt_a = time.perf_counter() - t0
    nv, nr = cfg.n_val, int(np.prod(cfg.grid))
    out = dict(metric="coupling applies/s (beyond the TDA)", value=round(args.nb / dt, 4),
               unit="applies/s", higher_is_better=True, dtype="f64", data="synthetic",
               config=dict(workload=cfg.name, n_val=nv, n_pw=n_pw, grid=list(cfg.grid),
                           n_pdep=cfg.n_pdep, n_b=args.nb),
               s_per_vector=round(dt / args.nb, 5),
               tda_s_per_vector=round(dt_a / args.nb, 6),
               coupling_over_tda=round(dt / dt_a, 1),
               w_pair_grids_per_vector=nv * nv)
    if args.full_bse:
        t1 = time.perf_counter()
        w, Xf, Yf, st = bsex.full_bse(ctx, 1, tol=args.tol)
        t2 = time.perf_counter()
        wt, _, dst = bsex.davidson(ctx, 1, tol=args.tol)
        t3 = time.perf_counter()
        out["full_bse"] = dict(omega=float(w[0]), iters=st["iters"], vectors=st["applies"],
                               s=round(t2 - t1, 2), resid=st["resid"][0],
                               y_norm2=float((Yf[0] ** 2).sum()),
                               tda_omega=float(wt[0]), tda_s=round(t3 - t2, 2))
    ctx.free()
    print(json.dumps(out), flush=True)


def relaxation(args):
    """Excited-state relaxation on one system (default C1): BFGS on the
    excited-state surface to |dE/dR| < --relax-gtol, once with every
    geometry solved from scratch and once warm started (each geometry's
    Davidson from the previous exciton, its Z-vector solve from the previous
    Z), then the ground-state relaxation for the displacement Delta Q."""
    import torch

    import synth
    from paper_2607_20728_amd import bsex, relax

    torch.cuda.set_device(0)
    cfg = config_of(args.config)
    n_pw = bsex.basis_size(cfg.cell, cfg.grid, cfg.ecut)
    d = synth.make_system(cfg, n_pw, seed=args.seed)
    prec = bsex.MIXED if args.precision == "mixed" else bsex.FP64
    bsex.warm_up()
    runs = {}
    order = (("warm", True), ("cold", False)) if args.relax_warm_first else \
        (("cold", False), ("warm", True))
    for label, warm in order:
        state = dict(warm=warm)

        def ev(sysd, xyz, state=state, label=label, **kw):
            r = relax.evaluate(sysd, xyz, state=state, **kw)
            log(f"[relax] {label}: evaluation {state['evals']}, E {r[0]:.10f}, "
                f"max |dE/dR| {np.abs(r[1]).max():.2e}")
            return r

        t0 = time.perf_counter()
        xyz, E, hist = relax.relax(d, surface="es", gtol=args.relax_gtol,
                                   max_steps=args.relax_steps, evaluator=ev, tol=args.relax_tol,
                                   precision=prec, two_level=args.two_level,
                                   n_extra=args.n_extra, keep_memory=not args.relax_free)
        dt = time.perf_counter() - t0
        runs[label] = dict(s=round(dt, 2), bfgs_steps=len(hist) - 1, evaluations=state["evals"],
                           davidson_iters=state["davidson_iters"],
                           davidson_applies=state["davidson_applies"],
                           zvector_iters=state["zvector_iters"],
                           s_init=round(state["s_init"], 2),
                           s_davidson=round(state["s_davidson"], 2),
                           s_zvector=round(state["s_zvector"], 2), E_es=E,
                           max_abs_grad=hist[-1][1], xyz=xyz)
        log(f"[relax] {label}: {dt:.1f} s, {len(hist) - 1} steps, {state['evals']} evaluations, "
            f"Davidson {state['davidson_iters']} / Z {state['zvector_iters']} iterations")
    dxyz = float(np.abs(runs["warm"]["xyz"] - runs["cold"]["xyz"]).max())
    gs = None
    dq = None
    if not args.relax_no_gs:
        t0 = time.perf_counter()
        xg, Eg, hg = relax.relax(d, surface="gs", gtol=args.relax_gtol,
                                 max_steps=args.relax_steps, precision=prec,
                                 n_extra=args.n_extra)
        gs = dict(s=round(time.perf_counter() - t0, 2), bfgs_steps=len(hg) - 1, E_gs=Eg)
        dq = relax.delta_q(xg, runs["warm"]["xyz"])
    for r in runs.values():
        del r["xyz"]
    out = dict(metric=f"excited-state relaxation, |dE/dR| < {args.relax_gtol:g} Ha/bohr "
                      f"(at most {args.relax_steps} BFGS steps)",
               value=runs["warm"]["s"], unit="s", higher_is_better=False,
               dtype="f32+f64" if prec == bsex.MIXED else "f64",
               data="synthetic",
               config=dict(workload=cfg.name, n_val=cfg.n_val, n_pw=n_pw, grid=list(cfg.grid),
                           n_sites=len(d["site_depth"]), spring_ha_bohr2=5.0),
               cold=runs["cold"], warm=runs["warm"],
               max_site_difference_warm_vs_cold_bohr=dxyz,
               ground_state=gs, delta_q_bohr=dq)
    print(json.dumps(out), flush=True)


def batch(args):
    """The uneven batch: the 32 systems of synth.c4_systems, lowest exciton and
    forces each, once one system at a time (one stream, no graphs, default
    kernels) and once batched (4 streams, HIP graphs, autotuned kernels)."""
    import torch

    import synth
    from paper_2607_20728_amd import bsex
    torch.cuda.set_device(0)
    cfgs = synth.c4_systems(args.batch_n)
    systems = []
    for cfg in cfgs:
        n_pw = bsex.basis_size(cfg.cell, cfg.grid, cfg.ecut)
        systems.append(synth.make_system(cfg, n_pw))
    prec = bsex.MIXED if args.precision == "mixed" else bsex.FP64
    runs = {}
    for name, kw in (("sequential", dict(n_streams=1, autotune=False, use_graph=False)),
                     ("batched", dict(n_streams=4, autotune=True, use_graph=True))):
        bsex.tune_cache_clear()
        t0 = time.perf_counter()
        res = bsex.batch_run(systems, tol=args.tol, precision=prec, check=False, **kw)
        dt = time.perf_counter() - t0
        bad = [r["message"] for r in res if r["status"] != 0]
        runs[name] = dict(seconds=round(dt, 2), systems_per_s=round(len(res) / dt, 4),
                          failed=len(bad), first_error=bad[0] if bad else None,
                          davidson_iters=sum(r["davidson_iters"] for r in res),
                          z_iters=sum(r["z_iters"] for r in res),
                          sum_stage_s={k: round(sum(r["t_" + k + "_ms"] for r in res) / 1e3, 2)
                                       for k in ("init", "davidson", "z", "force")},
                          variants=[r["variant"] for r in res], res=res)
        log(f"[batch] {name}: {dt:.1f} s, {len(bad)} failed")
    a, b = runs["sequential"]["res"], runs["batched"]["res"]
    dw = max(abs(x["omega"] - y["omega"]) for x, y in zip(a, b))
    dF = max(float(np.abs(x["dwdR"] - y["dwdR"]).max()) for x, y in zip(a, b))
    for r in runs.values():
        r.pop("res")
    out = dict(metric="uneven batch: systems/s (lowest exciton + forces each)",
               value=runs["batched"]["systems_per_s"], unit="systems/s", higher_is_better=True,
               dtype="f32+f64" if prec == bsex.MIXED else "f64", data="synthetic",
               config=dict(workload="32 cubic systems, grids {32,40,48,64}^3, N_v U{32..256}, "
                                    "N_pdep U{128..384}, 8 Gaussian sites (seed 4000)",
                           tol=args.tol, grids=[c.grid[0] for c in cfgs],
                           n_val=[c.n_val for c in cfgs]),
               runs=runs, max_abs_domega=dw, max_abs_ddwdR=dF,
               speedup=round(runs["sequential"]["seconds"] / runs["batched"]["seconds"], 3))
    print(json.dumps(out), flush=True)


def time_to_force(args):
    """Time to force on one system (default the defect supercell): device
    ground state and tau cache (init), Davidson for the lowest n_states
    excitons to --tol, U and the Z-vector solve to --tol, forces for exciton 1.
    --precision mixed runs the mixed-precision operator (residuals still judged
    by the FP64 operator); --learned attaches a trained preconditioner."""
    import torch

    import synth
    from paper_2607_20728_amd import bsex

    torch.cuda.set_device(0)
    cfg = config_of(args.config)
    n_pw = bsex.basis_size(cfg.cell, cfg.grid, cfg.ecut)
    d = synth.make_system(cfg, n_pw, seed=args.seed)
    # one-time process start-up (HIP runtime, the library's code objects) is
    # timed apart: a relaxation pays it once, not per geometry
    ts = time.perf_counter()
    bsex.warm_up()
    t_start = time.perf_counter() - ts
    t0 = time.perf_counter()
    prec = bsex.MIXED if args.precision == "mixed" else bsex.FP64
    ctx = bsex.init_from_synth(d, n_extra=args.n_extra, gs_tol=1e-10, gap_min=args.gap_min,
                               precision=prec, ks_model=args.ks_model, **loc_kw(args))
    net = None
    if args.learned:
        from paper_2607_20728_amd import learned
        net, _ = learned.load(args.learned)
        bsex.set_learned(ctx, net)
    use = net is not None
    torch.cuda.synchronize()
    t_init = time.perf_counter() - t0
    info = bsex.get_info(ctx)
    log(f"[ttf] init {t_init:.1f} s, gap {info['ks_gap']:.3e}, cached "
        f"{info['tau_blocks_cached']}/{info['tau_blocks']}")
    if args.phases:
        bsex.set_profiling(ctx, True)
        bsex.phase_times(ctx, reset=True)
    t1 = time.perf_counter()
    tl = args.two_level
    w, X, ds = bsex.davidson(ctx, cfg.n_states, tol=args.tol, use_learned=use, two_level=tl,
                             check=False, max_subspace=args.max_subspace)
    t2 = time.perf_counter()
    ph_dav = bsex.phase_times(ctx, reset=True) if args.phases else None
    log(f"[ttf] davidson {t2 - t1:.1f} s, {ds['iters']} iters, {ds['applies']} applies "
        f"({ds['applies_fp64']} FP64), "
        f"omega {w}, resid {ds['resid'][:cfg.n_states]}")
    Z, zs = bsex.zvector_solve(ctx, X[0], tol=args.tol, use_learned=use, two_level=tl,
                               check=False)
    t3 = time.perf_counter()
    ph_uz = bsex.phase_times(ctx, reset=True) if args.phases else None
    log(f"[ttf] U + Z {t3 - t2:.1f} s, {zs['iters']} iters, resid {zs['resid'][0]:.2e}")
    F = bsex.forces(ctx, X[0], Z, len(d["site_depth"]))
    t4 = time.perf_counter()
    mode = (args.precision + ("+learned" if use else "") + ("+two-level" if tl else "")
            + ("+ks" if args.ks_model else ""))
    out = dict(metric=f"time-to-force @{args.tol:g} resid ({mode})",
               value=round(t4 - t0, 2), unit="s", higher_is_better=False,
               dtype="f32+f64" if prec == bsex.MIXED else "f64", data="synthetic",
               seed=d["seed"],
               config=dict(workload=cfg.name, n_states=cfg.n_states, n_extra=args.n_extra,
                           tau_blocks_cached=info["tau_blocks_cached"],
                           tau_blocks=info["tau_blocks"], ks_gap_ha=info["ks_gap"]),
               split_s=dict(init=round(t_init, 2), davidson=round(t2 - t1, 2),
                            u_z=round(t3 - t2, 2), u=round(zs["t_u_ms"] / 1e3, 2),
                            z=round(t3 - t2 - zs["t_u_ms"] / 1e3, 2), forces=round(t4 - t3, 3)),
               init_s=dict(ground_state=round(info["t_ground_state_ms"] / 1e3, 2),
                           gs_sweeps=info["gs_sweeps"], tau=round(info["t_tau_ms"] / 1e3, 2),
                           tau_alloc=round(info["t_tau_alloc_ms"] / 1e3, 2),
                           library=round(info["t_init_ms"] / 1e3, 2)),
               process_start_s=round(t_start, 2),
               davidson=dict(iters=ds["iters"], applies=ds["applies"],
                             max_subspace=args.max_subspace or None,
                             applies_fp64=ds["applies_fp64"], rc=ds["rc"],
                             learned=ds["learned"], fallback=ds["fallback"],
                             omega=list(map(float, w)), resid=ds["resid"][:cfg.n_states]),
               zvector=dict(iters=zs["iters"], applies_fp64=zs["applies_fp64"],
                            learned=zs["learned"], fallback=zs["fallback"],
                            resid=zs["resid"][0], rc=zs["rc"]),
               max_abs_dwdR=float(np.abs(F).max()), sum_dwdR=list(map(float, F.sum(0))))
    if args.prune is not None:
        out["config"]["localized"] = dict(loc_info(info), threshold=args.prune)
    if args.ks_model:
        out["config"]["ks_model"] = dict(scf_iters=info["scf_iters"], alpha_exx=0.0)
    if args.phases:
        # device time per phase (ms, launches) with profiling on (no graphs)
        out["phases_ms"] = dict(
            davidson={k: [round(v[0], 1), v[1]] for k, v in ph_dav.items() if v[1]},
            u_z={k: [round(v[0], 1), v[1]] for k, v in ph_uz.items() if v[1]})
    if args.forces_out:
        np.save(args.forces_out, F)
    ctx.free()
    if net is not None:
        net.free()
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default=None,
                    help="system (default: the defect supercell c2; c1 for --relax)")
    ap.add_argument("--nb", type=int, default=8)
    # an explicit budget lets the tau cache use the memory a Davidson subspace
    # would otherwise keep in reserve (this run only applies the operator)
    ap.add_argument("--tau-budget-gb", type=float, default=1000.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--ttf", action="store_true", help="time-to-force run instead")
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--seed", type=int, default=None)
    ap.add_argument("--gap-min", type=float, default=0.0)
    ap.add_argument("--precision", choices=("fp64", "mixed"), default="fp64")
    ap.add_argument("--prune", type=float, default=None,
                    help="Wannier-localised frame with 8x8 blocks of occupied-pair W integrals "
                         "kept when their pair measure reaches this threshold")
    ap.add_argument("--loc-sweeps", type=int, default=0, help="Jacobi sweep cap (0: library default)")
    ap.add_argument("--forces-out", default=None, help="--ttf: save d omega/d R here (.npy)")
    ap.add_argument("--ks-model", type=int, default=0, choices=(0, 1),
                    help="--ttf: 1 = self-consistent KS ground state, with its response "
                         "kernels in U and the Z-vector equation (semilocal, no exact exchange)")
    ap.add_argument("--max-subspace", type=int, default=0,
                    help="--ttf: Davidson subspace size (0: the library default, 16 blocks)")
    ap.add_argument("--phases", action="store_true",
                    help="--ttf: device time per library phase (profiling on) in the JSON")
    ap.add_argument("--two-level", action="store_true",
                    help="two-level preconditioner on the conduction states held (--ttf)")
    ap.add_argument("--n-extra", type=int, default=8,
                    help="conduction states the ground-state solve computes (--ttf)")
    ap.add_argument("--batch", action="store_true", help="uneven batch run instead")
    ap.add_argument("--relax", action="store_true",
                    help="excited-state relaxation (cold and warm-started) instead")
    ap.add_argument("--relax-gtol", type=float, default=1e-5)
    ap.add_argument("--relax-steps", type=int, default=60, help="--relax: BFGS step cap")
    ap.add_argument("--relax-tol", type=float, default=1e-9,
                    help="--relax: Davidson and Z-vector residual per geometry")
    ap.add_argument("--relax-free", action="store_true",
                    help="--relax: free each geometry's device memory (no bse_memory_cache)")
    ap.add_argument("--relax-no-gs", action="store_true",
                    help="--relax: skip the ground-state relaxation (and Delta Q)")
    ap.add_argument("--relax-warm-first", action="store_true",
                    help="--relax: run the warm-started relaxation before the cold one")
    ap.add_argument("--coupling", action="store_true",
                    help="beyond the TDA: time the coupling apply (and --full-bse the root)")
    ap.add_argument("--full-bse", action="store_true", help="--coupling: also the coupled root")
    ap.add_argument("--batch-n", type=int, default=32)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="plain 2 GiB device copies, for scaling HBM counters")
    ap.add_argument("--learned", default=None,
                    help="trained preconditioner weights (.npz) for the --ttf run")
    args = ap.parse_args()
    if args.config is None:
        args.config = "c1" if args.relax else "c2"
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU "
              "sharding of this path is a design note, not a measured run.", file=sys.stderr)
        sys.exit(2)

    if args.ttf:
        time_to_force(args)
        return
    if args.copy_calibration:
        copy_calibration(args)
        return
    if args.relax:
        relaxation(args)
        return
    if args.batch:
        batch(args)
        return
    if args.coupling:
        beyond_tda(args)
        return

    import torch

    import synth
    from paper_2607_20728_amd import bsex

    torch.cuda.set_device(0)
    cfg = synth.get_config(args.config)
    n_pw = bsex.basis_size(cfg.cell, cfg.grid, cfg.ecut)
    d = synth.make_system(cfg, n_pw, n_trial=args.nb)
    log(f"[bench] {cfg.name}: grid {cfg.grid}, n_pw {n_pw}, n_val {cfg.n_val}, "
        f"n_pdep {cfg.n_pdep}, sites {len(d['site_depth'])}")
    # trial block first: the library sizes its tau cache from the memory left
    X = torch.tensor(d["trial"], dtype=torch.float64, device="cuda")
    Y = torch.empty_like(X)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mixed = args.precision == "mixed"
    ctx = bsex.init_from_synth(d, n_extra=8, gs_tol=1e-10,
                               tau_budget_bytes=int(args.tau_budget_gb * 1e9),
                               precision=bsex.MIXED if mixed else bsex.FP64, **loc_kw(args))
    torch.cuda.synchronize()
    t_init = time.perf_counter() - t0
    info = bsex.get_info(ctx)
    log(f"[bench] init {t_init:.1f} s; gs resid {info['gs_resid']:.2e}, KS gap "
        f"{info['ks_gap']:.3e} Ha; tau blocks cached {info['tau_blocks_cached']}/"
        f"{info['tau_blocks']}")
    for i in range(args.warmup):
        bsex.apply(ctx, X, Y)
        log(f"[bench] warmup {i + 1}/{args.warmup}")
    bsex.set_profiling(ctx, True)
    bsex.phase_times(ctx, reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        bsex.apply(ctx, X, Y)
        log(f"[bench] step {i + 1}/{args.steps}")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ph = bsex.phase_times(ctx)
    bsex.set_profiling(ctx, False)
    ms_step = 1e3 * dt / args.steps
    value = args.nb * args.steps / dt

    # roofline of the dominant phase: the tau contraction over the cache
    nv, nr = cfg.n_val, int(np.prod(cfg.grid))
    nB = (nv + 7) // 8
    blocks = [(I, J) for I in range(nB) for J in range(I, nB)]
    ncached = info["tau_blocks_cached"]
    esz = 4.0 if mixed else 8.0
    if mixed:  # the FP32 cache holds every block
        ncached = info["tau_blocks"]
    tau_bytes = esz * pair_count(nv, blocks[:ncached]) * nr
    if args.prune is not None:
        # kept blocks: every diagonal block (36 pairs) and the rest whole (64)
        if nv % 8 or ncached != info["tau_blocks"]:
            sys.exit("pruned roofline needs N_v divisible by 8 and the whole cache")
        tau_bytes = esz * (36 * nB + 64 * (ncached - nB)) * nr
    av_bytes = 2 * esz * args.nb * nv * nr          # a read + y write
    ms_stream, n_stream = ph.get("tau_stream", (0.0, 0))
    roofline = None
    if n_stream:
        dur = ms_stream / n_stream / 1e3
        ach = (tau_bytes + av_bytes) / dur / 1e9
        tr = stream_traffic(mixed)
        roofline = dict(bound="hbm", achieved=round(ach, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                        frac=round(ach / HBM_PEAK_GBS, 4),
                        traffic=None if tr is None else round(tr),
                        kernel=f"k_tau_stream_qs ({'FP32' if mixed else 'FP64'} cached blocks)",
                        bytes_per_launch=tau_bytes + av_bytes,
                        avg_launch_ms=round(1e3 * dur, 3))
    phases = {k: dict(ms_per_step=round(v[0] / args.steps, 3), launches=v[1])
              for k, v in ph.items() if v[1]}
    out = dict(metric=METRIC, value=round(value, 3), unit="applies/s", n_gpus=1,
               steps=args.steps, warmup=args.warmup, ms_per_step=round(ms_step, 2),
               higher_is_better=True, scaling="weak", vs_baseline=None,
               dtype="f32+f64" if mixed else "f64", data="synthetic",
               config=dict(workload=("defect supercell: cubic 20.2 bohr, 72^3 grid, "
                                     "21,079 plane waves, N_v=432, N_pdep=512, 215 Gaussian "
                                     "sites (3x3x3 diamond minus one), " +
                                     ("mixed: FP32 grids, FFTs and tau cache, FP64 projector "
                                      "and diagonal" if mixed else "FP64")),
                           n_b=args.nb, n_pw=n_pw, tau_blocks=info["tau_blocks"],
                           tau_blocks_cached=ncached,
                           tau_policy={0: "auto", 1: "cache", 2: "rebuild"}[info["tau_policy"]],
                           init_s=round(t_init, 1), ks_gap_ha=info["ks_gap"]),
               roofline=roofline, phases=phases)
    if args.prune is not None:
        out["config"]["localized"] = dict(loc_info(info), threshold=args.prune)
    ctx.free()
    del X, Y
    out["hbm_copy"] = copy_rate()
    out["hbm_read"] = read_rate()
    out["roofline"]["frac_of_read"] = round(out["roofline"]["achieved"] / out["hbm_read"]["gbs"], 4)
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle sample)")
        out["cpu_baseline"] = cpu_baseline(args.config, args.nb)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
