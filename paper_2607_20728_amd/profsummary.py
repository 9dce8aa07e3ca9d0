"""Summaries of rocprofv3 output.

    python -m paper_2607_20728_amd.profsummary kernels <results.db> [rows]
        per-kernel time from a --kernel-trace run (rocpd database), grouped
        by kernel and launch shape;

    python -m paper_2607_20728_amd.profsummary apply <results.db>
        the kernels of the last apply in a bench trace (those launched after
        the next-to-last k_tau_stream, up to the last one), in launch order;

    python -m paper_2607_20728_amd.profsummary stages <results.db> --grid N1 N2 N3
            --planes N1S --npw NPW --nv NV --nb NB --prec f64|f32 --stream-bytes B
        every stage of the applies in a bench trace against its own roof: the
        mean duration over the applies (segments between consecutive
        k_tau_stream launches) and the algorithmic bytes of the stage (N1S =
        planes along axis 1 that hold sphere modes; B = the stream's bytes
        per launch as bench.py reports them);

    python -m paper_2607_20728_amd.profsummary busy <results.db> [after] [rows] [before]
        device-busy fraction of a --kernel-trace run: from the end of the last
        launch whose name contains `after` (default: the first launch; NAME@k
        for the k-th launch, counting from 1) to the start of the launch
        `before` names (default: the end of the trace), the union of kernel
        intervals against the window, the gaps between kernels by size, and
        the kernels of the window by time;

    python -m paper_2607_20728_amd.profsummary counters <dir> [match]
        mean and largest value per dispatch of every counter of a --pmc run
        (--output-format csv), per kernel whose name contains match;

    python -m paper_2607_20728_amd.profsummary traffic --fetch DIR --write DIR
            --copy-fetch DIR --copy-write DIR --match k_tau_stream --out FILE
            [--dram DIR] [--command TEXT]
        HBM bytes per launch of the kernels whose name contains --match, from
        the FETCH_SIZE and WRITE_SIZE counter runs (--output-format csv),
        each scaled by the same counter on a plain 2 GiB copy
        (bench.py --copy-calibration); writes the JSON bench.py reads.
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import json
import os
import re
import sqlite3
import statistics
import sys


def kernels(db, rows=30):
    con = sqlite3.connect(db)
    cur = con.cursor()
    q = ("select name, grid_x, workgroup_x, lds_size, vgpr_count, accum_vgpr_count, duration "
         "from kernels")
    g = collections.defaultdict(list)
    for n, gx, wx, lds, vg, ag, du in cur.execute(q).fetchall():
        m = re.search(r'(k_[a-z_0-9]+(<[^>]*>)?|__amd_rocclr_\w+)', n)
        short = m.group(1) if m else n[:40]
        g[(short, gx, lds, vg, ag)].append(du)
    tot = sum(sum(v) for v in g.values())
    print(f"{'kernel':34s} {'grid_x':>10s} {'lds':>6s} {'calls':>6s} {'avg_us':>10s} "
          f"{'tot_ms':>9s} {'%':>5s}")
    for k, v in sorted(g.items(), key=lambda kv: -sum(kv[1]))[:rows]:
        print(f"{k[0]:34s} {k[1]:10d} {k[2]:6d} {len(v):6d} {sum(v) / len(v) / 1e3:10.1f} "
              f"{sum(v) / 1e6:9.1f} {100 * sum(v) / tot:5.1f}")


def _launch(ks, spec, last_default):
    """(start, end) of the launch `spec` names: NAME (the last launch, or the
    first when last_default is false) or NAME@k (the k-th, from 1)."""
    name, _, k = spec.partition("@")
    hits = [(s, e) for n, s, e in ks if name in n]
    if not hits:
        sys.exit(f"no launch matches {name!r}")
    if k:
        if int(k) > len(hits):
            sys.exit(f"{name!r} has {len(hits)} launches")
        return hits[int(k) - 1]
    return hits[-1] if last_default else hits[0]


def busy(db, after="", rows=20, before=""):
    con = sqlite3.connect(db)
    ks = con.execute("select name, start, end from kernels order by start").fetchall()
    if not ks:
        sys.exit("no kernels in the trace")
    t0 = _launch(ks, after, True)[1] if after else ks[0][1]
    tb = _launch(ks, before, False)[0] if before else None
    win = [(n, max(s, t0), e if tb is None else min(e, tb)) for n, s, e in ks
           if e > t0 and (tb is None or s < tb)]
    if not win:
        sys.exit("empty window")
    t1 = max(e for _, _, e in win) if tb is None else tb
    busy_ns, cur_s, cur_e = 0, None, None
    gaps = []
    for _, s, e in sorted(win, key=lambda r: r[1]):
        if cur_e is None:
            cur_s, cur_e = s, e
        elif s > cur_e:
            busy_ns += cur_e - cur_s
            gaps.append(s - cur_e)
            cur_s, cur_e = s, e
        else:
            cur_e = max(cur_e, e)
    busy_ns += cur_e - cur_s
    span = t1 - t0
    print(f"window {span / 1e6:.1f} ms, kernels busy {busy_ns / 1e6:.1f} ms "
          f"({100 * busy_ns / max(span, 1):.1f}%), {len(win)} launches")
    edges = [(0, 10e3), (10e3, 100e3), (100e3, 1e6), (1e6, float("inf"))]
    for lo, hi in edges:
        g = [x for x in gaps if lo <= x < hi]
        print(f"  gaps {lo / 1e3:g}-{hi / 1e3:g} us: {len(g):6d}, {sum(g) / 1e6:9.1f} ms")
    g = collections.defaultdict(list)
    for n, s, e in win:
        g[_short(n)].append(e - s)
    print(f"{'kernel':48s} {'calls':>7s} {'avg_us':>9s} {'tot_ms':>9s}")
    for k, v in sorted(g.items(), key=lambda kv: -sum(kv[1]))[:rows]:
        print(f"{k:48s} {len(v):7d} {sum(v) / len(v) / 1e3:9.1f} {sum(v) / 1e6:9.1f}")


def last_apply(db):
    con = sqlite3.connect(db)
    rows = con.execute("select name, grid_x, duration from kernels order by start").fetchall()
    idx = [i for i, r in enumerate(rows) if "k_tau_stream" in r[0]]
    if len(idx) < 2:
        sys.exit("fewer than two k_tau_stream launches in the trace")
    print(f"{'kernel':48s} {'grid_x':>10s} {'us':>9s}")
    for n, gx, du in rows[idx[-2] + 1:idx[-1] + 1]:
        m = re.search(r'(k_[a-z_0-9]+(<[^>]*>)?|__amd_rocclr_\w+)', n)
        print(f"{(m.group(1) if m else n[:40]):48s} {gx:10d} {du / 1e3:9.1f}")


_SHORT = re.compile(r'(k_[a-z_0-9]+(<[^>]*>)?|__amd_rocclr_\w+)')
HBM_PEAK = 8.0e12
FP64_MFMA_PEAK = 78.6e12


def _short(n):
    m = _SHORT.search(n)
    return m.group(1) if m else n[:40]


def stages(a):
    """Per-stage rooflines of the applies in a bench trace."""
    con = sqlite3.connect(a.db)
    rows = [(_short(n), gx, du) for n, gx, du in
            con.execute("select name, grid_x, duration from kernels order by start").fetchall()]
    idx = [i for i, r in enumerate(rows) if r[0].startswith("k_tau_stream")]
    if len(idx) < 2:
        sys.exit("fewer than two k_tau_stream launches in the trace")
    N1, N2, N3 = a.grid
    nr, p2 = N1 * N2 * N3, N2 * N3
    c = 16 if a.prec == "f64" else 8
    G = a.nb * ((a.nv + 1) // 2)
    xb = a.nb * a.nv * a.npw * 8
    model = [
        ("inverse plane pass, sphere -> planes", r"k_sphere_inv_ct|k_fft_plane_ct<\d+, \d+, 1, 1, 0>",
         xb + G * a.planes * p2 * c),
        ("inverse axis-1 pass", r"k_fft_axis_(ct|gd)<\d+, 1>", G * nr * c * (a.planes / N1 + 1)),
        ("transition density (K1e)", r"k_transition_density",
         (G + (a.nv + 1) // 2 + (a.nb + 1) // 2) * nr * c),
        ("tau stream + combine", r"k_tau_stream", a.stream_bytes),
        ("forward axis-1 pass", r"k_fft_axis_(ct|gd)<\d+, -1>", G * nr * c * (1 + a.planes / N1)),
        ("forward plane pass, planes -> sphere", r"k_sphere_fwd_ct|k_sphere_fwd_whole|k_fft_plane_ct<\d+, \d+, -1, 0, 1>",
         G * a.planes * p2 * c + G * a.npw * c),
        ("gather + diagonal", r"k_gather", G * a.npw * c + 2 * xb),
    ]
    gemm = [("S = Phi^T X", "k_dgemm<0, 1,"), ("Y = X - Phi S", "k_dgemm<1, 0,")]
    segs = [rows[idx[k - 1] + 1:idx[k] + 1] for k in range(1, len(idx))]

    def pick(seg, pat):
        # the stage's launch: the largest grid among the matching launches
        # (the K1e Poisson transforms reuse the FFT kernels on a few grids)
        m = [r for r in seg if re.match(pat, r[0])]
        if not m:
            return None, []
        big = max(r[1] for r in m)
        return m[0][0], [r[2] for r in m if r[1] == big]

    print(f"{len(segs)} applies; {a.prec}, N_b = {a.nb}, N_v = {a.nv}, grid {N1}x{N2}x{N3}, "
          f"{a.planes} planes hold sphere modes\n")
    print("| stage (kernel) | algorithmic bytes | ms | achieved | of 8 TB/s |")
    print("|---|---|---|---|---|")
    for label, pat, byt in model:
        ds, name = [], None
        for seg in segs:
            n, d = pick(seg, pat)
            if n:
                name = n
                ds.extend(d)
        if not ds:
            continue
        t = statistics.mean(ds) / 1e9
        print(f"| {label} (`{name}`) | {byt / 1e9:.2f} GB | {t * 1e3:.2f} | "
              f"{byt / t / 1e12:.2f} TB/s | {byt / t / HBM_PEAK:.2f} |")
    flops = 2.0 * a.nv * a.nb * a.nv * a.npw
    print("\n| GEMM (2 of each per apply) | flops | ms | achieved | of 78.6 TFLOP/s FP64 MFMA |")
    print("|---|---|---|---|---|")
    for label, prefix in gemm:
        ds, name = [], None
        for seg in segs:
            m = [r for r in seg if r[0].startswith(prefix)]
            if m:
                big = max(r[1] for r in m)
                name = m[0][0]
                ds.extend(r[2] for r in m if r[1] == big)
        if not ds:
            continue
        t = statistics.mean(ds) / 1e9
        print(f"| {label} (`{name}`) | {flops / 1e9:.1f} G | {t * 1e3:.2f} | "
              f"{flops / t / 1e12:.1f} TFLOP/s | {flops / t / FP64_MFMA_PEAK:.2f} |")
    seg_ms = [sum(r[2] for r in seg) / 1e6 for seg in segs]
    print(f"\nkernel time per apply (sum of its launches): {statistics.mean(seg_ms):.2f} ms")


def _counter_rows(d, counter):
    """(kernel name, value) per dispatch of one counter, from rocprofv3 CSVs."""
    out = []
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        with open(f, newline="") as fh:
            for r in csv.DictReader(fh):
                if r.get("Counter_Name") == counter:
                    out.append((r.get("Kernel_Name", ""), float(r["Counter_Value"])))
    if not out:
        sys.exit(f"no {counter} rows under {d}")
    return out


def counters(d, match=""):
    """Mean of each counter per dispatch, per kernel (name contains match)."""
    vals = collections.defaultdict(list)
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        with open(f, newline="") as fh:
            for r in csv.DictReader(fh):
                n = r.get("Kernel_Name", "")
                if match in n:
                    m = re.search(r'(k_[a-z_0-9]+(<[^>]*>)?|__amd_rocclr_\w+)', n)
                    vals[((m.group(1) if m else n[:60]), r["Counter_Name"])].append(
                        float(r["Counter_Value"]))
    if not vals:
        sys.exit(f"no counter rows under {d}")
    for (k, c), v in sorted(vals.items()):
        print(f"{k:48s} {c:36s} dispatches {len(v):4d} mean {statistics.mean(v):.6g} "
              f"max {max(v):.6g}")


def _copy_factor(d, counter, expected_kib):
    # the 2 GiB copy (and, for WRITE_SIZE, the 2 GiB fill before it) are the
    # only dispatches of that size in the calibration run
    vals = [v for _, v in _counter_rows(d, counter) if v > 0.5 * expected_kib]
    if not vals:
        sys.exit(f"no 2 GiB dispatch in {d}")
    return expected_kib / statistics.median(vals), vals


def traffic(a):
    gib_kib = 2.0 * 1024 * 1024
    ff, fvals = _copy_factor(a.copy_fetch, "FETCH_SIZE", gib_kib)
    wf, wvals = _copy_factor(a.copy_write, "WRITE_SIZE", gib_kib)
    fk = [(n, v) for n, v in _counter_rows(a.fetch, "FETCH_SIZE") if a.match in n]
    wk = [(n, v) for n, v in _counter_rows(a.write, "WRITE_SIZE") if a.match in n]
    if not fk or not wk:
        sys.exit(f"no dispatch of {a.match}")
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import bench
    out = dict(kernel=sorted({n for n, _ in fk})[0][:120], source_sha=bench.stream_kernel_sha(),
               launches=len(fk), fetch_kib_per_launch=statistics.mean(v for _, v in fk),
               write_kib_per_launch=statistics.mean(v for _, v in wk),
               copy_fetch_factor=ff, copy_write_factor=wf,
               copy_fetch_kib=fvals, copy_write_kib=wvals, command=a.command)
    if a.dram:
        # second route: DRAM-bound requests counted in 32-byte units
        # (a 64-byte request counts 2, a 128-byte one 4)
        rd = [v for n, v in _counter_rows(a.dram, "TCC_EA0_RDREQ_DRAM_32B_sum") if a.match in n]
        wr = [v for n, v in _counter_rows(a.dram, "TCC_EA0_WRREQ_WRITE_DRAM_32B_sum")
              if a.match in n]
        if rd and wr:
            out["dram_read_bytes_per_launch"] = 32.0 * statistics.mean(rd)
            out["dram_write_bytes_per_launch"] = 32.0 * statistics.mean(wr)
    with open(a.out, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out))


def main():
    if len(sys.argv) > 1 and sys.argv[1] == "apply":
        last_apply(sys.argv[2])
        return
    if len(sys.argv) > 1 and sys.argv[1] == "counters":
        counters(sys.argv[2], sys.argv[3] if len(sys.argv) > 3 else "")
        return
    if len(sys.argv) > 1 and sys.argv[1] == "busy":
        busy(sys.argv[2], sys.argv[3] if len(sys.argv) > 3 else "",
             int(sys.argv[4]) if len(sys.argv) > 4 else 20,
             sys.argv[5] if len(sys.argv) > 5 else "")
        return
    if len(sys.argv) > 1 and sys.argv[1] == "kernels":
        kernels(sys.argv[2], int(sys.argv[3]) if len(sys.argv) > 3 else 30)
        return
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("traffic")
    for k in ("fetch", "write", "copy_fetch", "copy_write", "out"):
        t.add_argument("--" + k.replace("_", "-"), dest=k, required=True)
    t.add_argument("--match", default="k_tau_stream")
    t.add_argument("--dram", default=None,
                   help="run with TCC_EA0_RDREQ_DRAM_32B_sum and TCC_EA0_WRREQ_WRITE_DRAM_32B_sum")
    t.add_argument("--command", default="")
    g = sub.add_parser("stages")
    g.add_argument("db")
    g.add_argument("--grid", type=int, nargs=3, required=True)
    g.add_argument("--planes", type=int, required=True)
    for k in ("npw", "nv", "nb"):
        g.add_argument("--" + k, type=int, required=True)
    g.add_argument("--prec", choices=("f64", "f32"), required=True)
    g.add_argument("--stream-bytes", dest="stream_bytes", type=float, required=True)
    a = ap.parse_args()
    if a.cmd == "stages":
        stages(a)
    else:
        traffic(a)


if __name__ == "__main__":
    main()
