#!/usr/bin/env python
"""Benchmark of the matching-AMG preconditioned CG on one MI355X.

Workload: 3D Poisson, 7-point Laplacian on the 160^3 interior grid
(n = 4 096 000, nnz = 28 518 400), b = A u with u ~ U(-1, 1) (seed 1),
x0 = 0, PCG to a relative residual of 1e-8. Hierarchy: 3 pairwise matching
sweeps per level with w = 1, unsmoothed prolongator, 1 + 1 l1-Jacobi sweeps,
coarsest level (<= 200 unknowns) solved by dense Cholesky.

One step is one complete PCG solve (the hierarchy is built once, before the
timed region, as the solver reuses it across right-hand sides). The headline
value is the p99 solve time with the FP64 hierarchy; the same system solved
with the FP32 hierarchy (FP64 outer CG) is reported beside it, as are the
V-cycle bandwidths, the dominant kernel's roofline position and the FP64 CPU
oracle timed on the host.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "AMG-PCG solve ms & V-cycle HBM GB/s (160^3 Poisson), FP32-prec vs FP64; p99"
HBM_PEAK_GBS = 8000.0
KERNEL_NAMES = {0: "pre-smoothing + residual + restriction", 1: "post-smoothing + CG dot",
                2: "level-1 post-smoothing + prolongation", 4: "outer-CG SpMV + dot"}


def source_hash() -> str:
    """Hash of the HIP sources (ties stored counter readings to a build)."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2006_16147_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def vcycle_bytes(sizes, nnzs, V, nL, a0=None, s0=None):
    """Algorithmic HBM bytes of one V-cycle with this library's kernel set.

    n_l rows, z_l entries per level; V value bytes; Vr = 8 on level 0, whose
    right-hand side and output are the FP64 CG vectors. Every array is read
    or written once per kernel (matrix values + int32 columns + int32 row
    offsets per SpMV):
      pre-smoothing + residual + restriction (l < L):
          z_l (V + 4) + 4 (n_l + 1) + n_l (Vr + 3 V) + n_{l+1} (V + 4)
      post-smoothing of level c (0 < c < L), fused with prolongation:
          z_c (V + 4) + 4 (n_c + 1) + 3 V n_c
      prolongation into level l (l < L):  n_l (3 V + 4)
      coarsest solve (dense A_L^-1):      8 n_L^2 + V n_L
      level-0 post-smoothing:             z_0 (A0 + 4) + 4 (n_0 + 1) + n_0 (16 + 2 V)
    A0 = a0 is the byte width of level 0's stored values there (4 when the
    FP64 hierarchy reads the exact FP32 copy of A; V otherwise). s0 is the
    byte width of the values level 0's down step reads: the scaled A M^-1 in
    the hierarchy precision (V), or 4 where an FP64 hierarchy forms M^-1 r
    in LDS and reads the exact FP32 copy of A.
    """
    a0 = V if a0 is None else a0
    s0 = V if s0 is None else s0
    L = len(sizes) - 1
    if L == 0:
        return 8.0 * nL * nL + 16.0 * nL
    total = 0.0
    for l in range(L):
        n, z, nc = sizes[l], nnzs[l], sizes[l + 1]
        Vr = 8.0 if l == 0 else V
        Vs = s0 if l == 0 else V
        total += z * (Vs + 4) + 4 * (n + 1) + n * (Vr + 3 * V) + nc * (V + 4)
        total += n * (3 * V + 4)
    for c in range(1, L):
        total += nnzs[c] * (V + 4) + 4 * (sizes[c] + 1) + 3 * V * sizes[c]
    total += 8.0 * nL * nL + V * nL
    total += nnzs[0] * (a0 + 4) + 4 * (sizes[0] + 1) + sizes[0] * (16 + 2 * V)
    return total


def percentile(a, q):
    return float(np.percentile(np.asarray(a), q))


def load_traffic(kernel_key):
    """HBM traffic per launch from the committed rocprofv3 counter summary, if
    it was taken on the current sources; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    if d.get("source_hash") != source_hash():
        return None
    k = d.get("kernels", {}).get(kernel_key)
    if not k:
        return None
    return float(k["bytes_per_launch"])


CALIB_BYTES = 512 << 20  # plain device copy used to scale the HBM counters
TRAFFIC_KERNELS = {  # kernel-name pattern (its largest launches are level 0's) -> key
    "fp64_level0_0": r"k_pre_restrict(_lds)?<double, double, [02],",
    "fp64_level0_1": r"k_post(_lds)?<double, double, double, true,",
    "fp64_level0_4": r"k_spmv_dot(_lds)?<",
}


def profile_pass(N=160):
    """Short run for counter collection: one FP64 setup, two solves, and a
    plain device copy of CALIB_BYTES (read and written once)."""
    import torch

    from paper_2006_16147_amd import amg, inputs

    dev = torch.device("cuda:0")
    case = inputs.headline_case(N, seed=1)
    A = case["A"]
    h = amg.amg_setup(torch.from_numpy(A.row_ptr).to(dev), torch.from_numpy(A.col).to(dev),
                      torch.from_numpy(A.val).to(dev))
    b = torch.from_numpy(case["b"]).to(dev)
    for _ in range(2):
        x = torch.zeros_like(b)
        amg.amg_pcg_solve(h, b, x, rtol=case["rtol"], maxit=1000)
    src = torch.ones(CALIB_BYTES // 8, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    h.close()
    print(json.dumps({"profile_pass": "done", "n": A.n}), flush=True)


def _counter_rows(path):
    import csv

    with open(path) as f:
        return list(csv.DictReader(f))


def ingest_pmc(fetch_csv, write_csv):
    """Writes profiles/traffic.json from rocprofv3 FETCH_SIZE and WRITE_SIZE
    counter CSVs of the profile pass: per-dispatch KiB averaged per kernel,
    scaled by the same counter's reading for the calibration copy."""
    out = {"source_hash": source_hash(), "calibration_bytes": CALIB_BYTES, "kernels": {}}
    per = {}
    for counter, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        rows = [r for r in _counter_rows(path) if r.get("Counter_Name") == counter]
        # the calibration copy is the largest device copy of the pass
        copies = [float(r["Counter_Value"]) for r in rows if "copyBuffer" in r["Kernel_Name"]]
        if not copies:
            raise SystemExit("no calibration copy dispatch found for %s" % counter)
        kib_copy = max(copies)
        scale = kib_copy * 1024.0 / CALIB_BYTES  # counter bytes per real byte moved
        out["%s_scale" % counter] = scale
        for key, frag in TRAFFIC_KERNELS.items():
            match = [r for r in rows if re.search(frag, r["Kernel_Name"])]
            top = max((int(r.get("Grid_Size", 0)) for r in match), default=0)
            vals = [float(r["Counter_Value"]) * 1024.0 / scale for r in match
                    if int(r.get("Grid_Size", 0)) == top]
            if vals:
                per.setdefault(key, {})[counter] = sum(vals) / len(vals)
                per[key]["dispatches"] = len(vals)
    for key, d in per.items():
        if "FETCH_SIZE" in d and "WRITE_SIZE" in d:
            out["kernels"][key] = {"fetch_bytes": d["FETCH_SIZE"], "write_bytes": d["WRITE_SIZE"],
                                   "bytes_per_launch": d["FETCH_SIZE"] + d["WRITE_SIZE"],
                                   "dispatches": d["dispatches"]}
    path = os.path.join(ROOT, "profiles", "traffic.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


def _grid(r):
    for key in ("Grid_Size", "Grid_Size_X"):
        if r.get(key) not in (None, ""):
            return int(r[key])
    return 0


def _short(name):
    """Kernel name without return type, namespaces and argument list."""
    if name.startswith("void "):
        name = name[5:]
    depth, cut, ns = 0, len(name), 0
    for i, ch in enumerate(name):
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0 and not name.startswith("(anonymous", i):
            cut = i
            break
        elif ch == ":" and depth == 0 and name[i:i + 2] == "::":
            ns = i + 2
    return name[ns:cut] if ns < cut else name[:cut]


def kernel_summary(trace_csv):
    """Markdown summary of a rocprofv3 kernel trace: per kernel the calls and
    the average / min / max duration, and, for the level-0 solve kernels, the
    average over their full launches only (largest grid, and not the early
    exits that the iterations queued past convergence take, which last a few
    microseconds: durations below half the median of those launches)."""
    rows = _counter_rows(trace_csv)
    per = {}
    for r in rows:
        d = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3  # us
        per.setdefault(r["Kernel_Name"], []).append((d, _grid(r)))
    tot = sum(d for v in per.values() for d, _ in v)
    out = ["| kernel | calls | avg us | min us | max us | total ms | % |",
           "|---|---|---|---|---|---|---|"]
    for name, v in sorted(per.items(), key=lambda kv: -sum(d for d, _ in kv[1]))[:40]:
        ds = [d for d, _ in v]
        out.append("| `%s` | %d | %.1f | %.1f | %.1f | %.2f | %.1f |" % (
            _short(name), len(ds), sum(ds) / len(ds), min(ds), max(ds), sum(ds) / 1e3, 100 * sum(ds) / tot))
    out += ["", "Level-0 solve kernels, full launches only (largest grid, early exits left out):",
            "", "| kernel | full launches | avg us | min us | max us |", "|---|---|---|---|---|"]
    level0 = re.compile(r"^(k_pre_restrict|k_post|k_spmv_dot)(_lds)?<")
    for name, v in sorted(per.items(), key=lambda kv: -sum(d for d, _ in kv[1])):
        if not level0.match(_short(name)):
            continue
        top = max(g for _, g in v)
        ds = sorted(d for d, g in v if g == top)
        med = ds[len(ds) // 2]
        full = [d for d in ds if d >= 0.5 * med]
        if sum(full) / len(full) < 20.0:  # a coarse level's launches, not level 0's
            continue
        out.append("| `%s` | %d | %.2f | %.1f | %.1f |" % (
            _short(name), len(full), sum(full) / len(full), min(full), max(full)))
    # The same kernels inside CG iterations only: the launches that follow a
    # finalize (the down step after the CG update's sum) or p = z + beta p
    # (the outer SpMV), or that a finalize follows (the post-smoothing and
    # its CG dot). The back-to-back timing loops, whose launches find their
    # data in L2, and the V-cycle timing loop (bracketed by the permutations)
    # are left out; this is what the benchmark's in-solve figure times.
    seqs = {}
    for r in rows:
        q = r.get("Queue_Id") or r.get("Stream_Id") or "0"
        seqs.setdefault(q, []).append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]),
                                       _short(r["Kernel_Name"]), _grid(r)))
    insolve = {}
    for seq in seqs.values():
        seq.sort()
        for i, (t0, t1, name, g) in enumerate(seq):
            if not level0.match(name):
                continue
            prev = seq[i - 1][2] if i > 0 else ""
            nxt = seq[i + 1][2] if i + 1 < len(seq) else ""
            if prev.startswith(("k_finalize", "k_xpay")) or nxt.startswith("k_finalize"):
                insolve.setdefault(name, []).append(((t1 - t0) / 1e3, g))
    out += ["", "The same kernels inside CG iterations (launches next to the iteration's "
            "finalize or p update; full launches only):", "",
            "| kernel | launches | avg us | min us | max us |", "|---|---|---|---|---|"]
    for name, v in sorted(insolve.items(), key=lambda kv: -sum(d for d, _ in kv[1])):
        top = max(g for _, g in v)
        ds = sorted(d for d, g in v if g == top)
        med = ds[len(ds) // 2]
        full = [d for d in ds if d >= 0.5 * med]
        if sum(full) / len(full) < 20.0:
            continue
        out.append("| `%s` | %d | %.2f | %.1f | %.1f |" % (
            name, len(full), sum(full) / len(full), min(full), max(full)))
    print("\n".join(out))


def counter_summary(fetch_csv, write_csv):
    """Markdown table of rocprofv3 FETCH_SIZE / WRITE_SIZE counter runs: per
    kernel, the mean over its largest-grid dispatches, in MB, each counter
    scaled as profiles/traffic.json records for the calibration copy."""
    scale = {"FETCH_SIZE": 1.0, "WRITE_SIZE": 1.0}
    tpath = os.path.join(ROOT, "profiles", "traffic.json")
    if os.path.exists(tpath):
        with open(tpath) as f:
            t = json.load(f)
        for c in scale:
            scale[c] = t.get("%s_scale" % c, 1.0)
    per = {}
    for counter, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        for r in _counter_rows(path):
            if r.get("Counter_Name") != counter:
                continue
            d = per.setdefault(_short(r["Kernel_Name"]), {}).setdefault(counter, [])
            d.append((_grid(r), float(r["Counter_Value"]) * 1024.0 / scale[counter]))
    out = ["| kernel | largest-grid dispatches | fetched MB | written MB |", "|---|---|---|---|"]
    rows = []
    for name, d in per.items():
        vals = {}
        for counter, v in d.items():
            top = max(g for g, _ in v)
            sel = [b for g, b in v if g == top]
            # levels with the same (capped) grid: keep the largest level's dispatches
            big = max(sel)
            sel = [b for b in sel if b >= 0.5 * big]
            vals[counter] = (len(sel), sum(sel) / len(sel))
        f = vals.get("FETCH_SIZE", (0, 0.0))
        w = vals.get("WRITE_SIZE", (0, 0.0))
        rows.append((f[1] + w[1], name, max(f[0], w[0]), f[1], w[1]))
    for _, name, nd, fb, wb in sorted(rows, reverse=True)[:30]:
        out.append("| `%s` | %d | %.1f | %.1f |" % (name, nd, fb / 1e6, wb / 1e6))
    print("\n".join(out))


def overlap_summary(trace_csv):
    """GPU busy fraction and cross-stream overlap of a rocprofv3 kernel trace:
    the time covered by at least one kernel, and by kernels of at least two
    different queues at once, over the span from the first kernel's start to
    the last one's end (a serving run: each slot has its own stream)."""
    rows = _counter_rows(trace_csv)
    ev = []
    for r in rows:
        q = r.get("Queue_Id") or r.get("Stream_Id") or "0"
        s0, s1 = int(r["Start_Timestamp"]), int(r["End_Timestamp"])
        if s1 > s0:
            ev.append((s0, 1, q))
            ev.append((s1, -1, q))
    ev.sort()
    active = {}
    busy = multi = 0
    t_prev = ev[0][0]
    for t, d, q in ev:
        if t > t_prev:
            live = sum(1 for c in active.values() if c > 0)
            if live >= 1:
                busy += t - t_prev
            if live >= 2:
                multi += t - t_prev
            t_prev = t
        active[q] = active.get(q, 0) + d
    span = ev[-1][0] - ev[0][0]
    out = {"kernels": len(rows), "queues": len({e[2] for e in ev}), "span_ms": span / 1e6,
           "busy_ms": busy / 1e6, "busy_fraction": busy / span,
           "overlap_ms": multi / 1e6, "overlap_fraction_of_busy": multi / busy if busy else 0.0}
    print(json.dumps(out))
    return out


def bench_kcycle(args):
    """160^3 Poisson (b = A u): flexible CG with the K-cycle (Section 3.1)
    against CG with the V-cycle, both hierarchy precisions, same run."""
    import torch

    from paper_2006_16147_amd import amg, inputs

    dev = torch.device("cuda:0")
    case = inputs.headline_case(args.N, seed=1)
    A = case["A"]
    rp = torch.from_numpy(A.row_ptr).to(dev)
    ci = torch.from_numpy(A.col).to(dev)
    va = torch.from_numpy(A.val).to(dev)
    b = torch.from_numpy(case["b"]).to(dev)
    out = {"mode": "kcycle", "workload": "poisson7_%d^3_b=Au_seed1_rtol1e-8" % args.N,
           "n": A.n, "nnz": A.nnz}
    for cyc, cname in ((amg.CYCLE_K, "K"), (amg.CYCLE_V, "V")):
        for prec, pname in ((amg.FP64, "fp64"), (amg.FP32, "fp32_prec")):
            h = amg.amg_setup(rp, ci, va, precision=prec, cycle=cyc)
            x = torch.zeros_like(b)
            times = []
            for k in range(args.warmup + args.steps):
                x.zero_()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                st, info = amg.amg_pcg_solve(h, b, x, rtol=1e-8, maxit=500)
                if k >= args.warmup:
                    times.append((time.perf_counter() - t0) * 1e3)
            p50 = percentile(times, 50)
            out["%s_%s" % (cname, pname)] = {
                "p50_ms": round(p50, 3), "p99_ms": round(percentile(times, 99), 3),
                "iterations": info["iterations"], "rel_res_true": info["rel_res_true"],
                "ms_per_iteration": round(p50 / max(1, info["iterations"]), 4),
                "setup_ms": round(h.setup_times()["total"], 1)}
            h.close()
    print(json.dumps(out), flush=True)


def bench_coarse(args):
    """160^3 Poisson (b = A u): the coarsest solve by CG with the l1-Jacobi
    diagonal (rtol 1e-4, at most 30 iterations) against the dense Cholesky
    solve. V-cycle with 4 l1-Jacobi pre/post sweeps and the CG coarsest
    solve is the paper's GPU preconditioner (Section 5); flexible CG is the
    outer solver whenever the coarsest solve is iterative. Outer tolerance
    1e-6 (Section 5) and 1e-8."""
    import torch

    from paper_2006_16147_amd import amg, inputs

    dev = torch.device("cuda:0")
    case = inputs.headline_case(args.N, seed=1)
    A = case["A"]
    rp = torch.from_numpy(A.row_ptr).to(dev)
    ci = torch.from_numpy(A.col).to(dev)
    va = torch.from_numpy(A.val).to(dev)
    b = torch.from_numpy(case["b"]).to(dev)
    out = {"mode": "coarse", "workload": "poisson7_%d^3_b=Au_seed1" % args.N}
    configs = [("V_l1x1_cholesky", amg.CYCLE_V, 1, amg.COARSE_CHOLESKY, amg.FP64),
               ("V_l1x1_cg", amg.CYCLE_V, 1, amg.COARSE_PCG, amg.FP64),
               ("V_l1x4_cholesky", amg.CYCLE_V, 4, amg.COARSE_CHOLESKY, amg.FP64),
               ("V_l1x4_cg", amg.CYCLE_V, 4, amg.COARSE_PCG, amg.FP64),
               ("V_l1x4_cg_fp32_prec", amg.CYCLE_V, 4, amg.COARSE_PCG, amg.FP32),
               ("K_l1x1_cg", amg.CYCLE_K, 1, amg.COARSE_PCG, amg.FP64)]
    for name, cyc, sw, cs, prec in configs:
        h = amg.amg_setup(rp, ci, va, precision=prec, cycle=cyc, pre=sw, post=sw,
                          coarse_solver=cs)
        res = {"setup_ms": round(h.setup_times()["total"], 1)}
        for rtol in (1e-6, 1e-8):
            x = torch.zeros_like(b)
            times = []
            for k in range(args.warmup + args.steps):
                x.zero_()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                st, info = amg.amg_pcg_solve(h, b, x, rtol=rtol, maxit=500)
                if k >= args.warmup:
                    times.append((time.perf_counter() - t0) * 1e3)
            p50 = percentile(times, 50)
            res["rtol%g" % rtol] = {
                "p50_ms": round(p50, 3), "p99_ms": round(percentile(times, 99), 3),
                "iterations": info["iterations"], "rel_res_true": info["rel_res_true"],
                "ms_per_iteration": round(p50 / max(1, info["iterations"]), 4)}
        if cyc == amg.CYCLE_V:
            ms, _ = h.time_kernel(5, 0, reps=args.vcycles)
            res["vcycle_ms"] = round(ms, 4)
        out[name] = res
        h.close()
    print(json.dumps(out), flush=True)


def bench_smoothed(args):
    """160^3 Poisson (b = A u): smoothed aggregation (Pbar = (I - omega D^-1 A) P,
    the alternative to the K-cycle in Section 3.2) against the unsmoothed
    hierarchy; with 4 l1-Jacobi pre/post sweeps and the CG coarsest solve it
    is the paper's GPU preconditioner (Section 5). Outer tolerance 1e-6
    (Section 5) and 1e-8."""
    import torch

    from paper_2006_16147_amd import amg, inputs

    dev = torch.device("cuda:0")
    case = inputs.headline_case(args.N, seed=1)
    A = case["A"]
    rp = torch.from_numpy(A.row_ptr).to(dev)
    ci = torch.from_numpy(A.col).to(dev)
    va = torch.from_numpy(A.val).to(dev)
    b = torch.from_numpy(case["b"]).to(dev)
    out = {"mode": "smoothed", "workload": "poisson7_%d^3_b=Au_seed1" % args.N}
    configs = [("V_unsmoothed_l1x1_cholesky", 0, 1, amg.COARSE_CHOLESKY, amg.FP64),
               ("V_smoothed_l1x1_cholesky", 1, 1, amg.COARSE_CHOLESKY, amg.FP64),
               ("V_smoothed_l1x4_cg", 1, 4, amg.COARSE_PCG, amg.FP64),
               ("V_smoothed_l1x4_cg_fp32_prec", 1, 4, amg.COARSE_PCG, amg.FP32),
               ("V_smoothed_l1x1_cholesky_fp32_prec", 1, 1, amg.COARSE_CHOLESKY, amg.FP32)]
    for name, sm, sw, cs, prec in configs:
        setup_ms = []
        for _ in range(2):
            h = amg.amg_setup(rp, ci, va, precision=prec, pre=sw, post=sw, coarse_solver=cs,
                              smooth_p=sm)
            setup_ms.append(h.setup_times()["total"])
        res = {"setup_ms_min": round(min(setup_ms), 1), "levels": h.sizes(),
               "opc": round(h.opc(), 4), "footprint_GB": round(h.footprint_bytes() / 1e9, 3)}
        for rtol in (1e-6, 1e-8):
            x = torch.zeros_like(b)
            times = []
            for k in range(args.warmup + args.steps):
                x.zero_()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                st, info = amg.amg_pcg_solve(h, b, x, rtol=rtol, maxit=500)
                if k >= args.warmup:
                    times.append((time.perf_counter() - t0) * 1e3)
            p50 = percentile(times, 50)
            res["rtol%g" % rtol] = {
                "p50_ms": round(p50, 3), "p99_ms": round(percentile(times, 99), 3),
                "iterations": info["iterations"], "rel_res_true": info["rel_res_true"],
                "ms_per_iteration": round(p50 / max(1, info["iterations"]), 4)}
        ms, by = h.time_kernel(5, 0, reps=args.vcycles)
        res["vcycle_ms"] = round(ms, 4)
        res["vcycle_GBs"] = round(by / ms / 1e6, 1)
        out[name] = res
        h.close()
    print(json.dumps(out), flush=True)


def bench_variants(args):
    """160^3 Poisson (b = A u), V-cycle PCG in FP64: 3 or 4 pairwise sweeps
    per level, w = ones or an algebraically smooth w (4 l1-Jacobi sweeps on
    A w = 0 from ones)."""
    import torch

    from paper_2006_16147_amd import amg, inputs

    dev = torch.device("cuda:0")
    case = inputs.headline_case(args.N, seed=1)
    A = case["A"]
    rp = torch.from_numpy(A.row_ptr).to(dev)
    ci = torch.from_numpy(A.col).to(dev)
    va = torch.from_numpy(A.val).to(dev)
    b = torch.from_numpy(case["b"]).to(dev)
    out = {"mode": "variants", "workload": "poisson7_%d^3_b=Au_seed1_rtol1e-8" % args.N}
    for sweeps in (3, 4):
        for nu in (0, 4):
            h = amg.amg_setup(rp, ci, va, sweeps=sweeps, w_sweeps=nu)
            x = torch.zeros_like(b)
            times = []
            for k in range(args.warmup + args.steps):
                x.zero_()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                st, info = amg.amg_pcg_solve(h, b, x, rtol=1e-8, maxit=500)
                if k >= args.warmup:
                    times.append((time.perf_counter() - t0) * 1e3)
            out["sweeps%d_wsweeps%d" % (sweeps, nu)] = {
                "levels": h.sizes(), "opc": round(h.opc(), 5),
                "setup_ms": round(h.setup_times()["total"], 1),
                "iterations": info["iterations"], "rel_res_true": info["rel_res_true"],
                "p50_ms": round(percentile(times, 50), 3)}
            h.close()
    print(json.dumps(out), flush=True)


def bench_aniso(args):
    """256^3 block-anisotropic diffusion: FP64 vs FP32 hierarchy (outer CG FP64)."""
    import torch

    from paper_2006_16147_amd import amg, inputs

    dev = torch.device("cuda:0")
    N = args.N if args.N != 160 else 256
    ex, ey, bh = inputs.aniso_blocks_coefficients(N, 16, seed=2)
    rp, ci, va = inputs.diffusion7_torch(N, torch.from_numpy(ex).to(dev),
                                         torch.from_numpy(ey).to(dev), 1.0, dev)
    b = torch.from_numpy(bh).to(dev)
    out = {"mode": "aniso", "workload": "aniso7_%d^3_blocks16_seed2_rtol1e-8" % N,
           "n": int(rp.numel() - 1), "nnz": int(ci.numel())}
    xs = {}
    for prec, name in ((amg.FP64, "fp64"), (amg.FP32, "fp32_prec")):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h = amg.amg_setup(rp, ci, va, precision=prec)
        torch.cuda.synchronize()
        setup_ms = (time.perf_counter() - t0) * 1e3
        x = torch.zeros_like(b)
        times = []
        for k in range(args.warmup + args.steps):
            x.zero_()
            t0 = time.perf_counter()
            st, info = amg.amg_pcg_solve(h, b, x, rtol=1e-8, maxit=1000)
            if k >= args.warmup:
                times.append((time.perf_counter() - t0) * 1e3)
        xs[name] = x.cpu().numpy()
        out[name] = {"setup_ms": round(setup_ms, 1), "levels": h.sizes(), "opc": round(h.opc(), 4),
                     "p50_ms": round(percentile(times, 50), 3),
                     "p99_ms": round(percentile(times, 99), 3),
                     "iterations": info["iterations"], "rel_res_true": info["rel_res_true"]}
        h.close()
    out["fp32_vs_fp64_rel_diff"] = float(np.linalg.norm(xs["fp32_prec"] - xs["fp64"])
                                         / np.linalg.norm(xs["fp64"]))
    out["fp32_prec_speedup_p50"] = round(out["fp64"]["p50_ms"] / out["fp32_prec"]["p50_ms"], 3)
    print(json.dumps(out), flush=True)


def bench_batch(args):
    """128^3 Poisson with k = 32 right-hand sides: one batched solve (block
    V-cycle, FP32 hierarchy, per-column FP64 CG) vs k single solves."""
    import torch

    from paper_2006_16147_amd import amg, inputs

    dev = torch.device("cuda:0")
    N = args.N if args.N != 160 else 128
    k = 32
    A = inputs.laplacian7(N)
    B = np.random.default_rng(3).uniform(-1.0, 1.0, (A.n, k))
    Bd = torch.from_numpy(B).to(dev)
    h = amg.amg_setup(torch.from_numpy(A.row_ptr).to(dev), torch.from_numpy(A.col).to(dev),
                      torch.from_numpy(A.val).to(dev), precision=amg.FP32)
    X = torch.zeros_like(Bd)
    for _ in range(max(1, args.warmup)):
        X.zero_()
        amg.amg_pcg_solve_batch(h, Bd, X, rtol=1e-8, maxit=1000)
    times = []
    for _ in range(args.steps):
        X.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, infos = amg.amg_pcg_solve_batch(h, Bd, X, rtol=1e-8, maxit=1000)
        times.append((time.perf_counter() - t0) * 1e3)
    its = [i["iterations"] for i in infos]
    # the same 32 right-hand sides one at a time
    single = 0.0
    x = torch.zeros(A.n, dtype=torch.float64, device=dev)
    cols = [Bd[:, j].contiguous() for j in range(k)]
    amg.amg_pcg_solve(h, cols[0], x, rtol=1e-8, maxit=1000)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for j in range(k):
        x.zero_()
        amg.amg_pcg_solve(h, cols[j], x, rtol=1e-8, maxit=1000)
    torch.cuda.synchronize()
    single = (time.perf_counter() - t0) * 1e3
    out = {"mode": "batch", "workload": "poisson7_%d^3_k%d_seed3_rtol1e-8_fp32prec" % (N, k),
           "n": A.n, "k": k, "status": st, "tile": h.batch_tiles()[0],
           "vector_tile_shift": h.batch_tiles()[1],
           "batch_p50_ms": round(percentile(times, 50), 3),
           "batch_p99_ms": round(percentile(times, 99), 3),
           "ms_per_rhs": round(percentile(times, 50) / k, 3),
           "single_solves_ms": round(single, 3), "ms_per_rhs_single": round(single / k, 3),
           "batch_speedup": round(single / percentile(times, 50), 3),
           "iterations_min_max": [min(its), max(its)],
           "max_rel_res_true": max(i["rel_res_true"] for i in infos)}
    h.close()
    print(json.dumps(out), flush=True)


def bench_serve(args):
    from paper_2006_16147_amd import serve

    serve.main(["--rates", args.rates, "--count", str(args.count), "--warmup",
                str(max(0, args.count // 20)), "--slots", str(args.slots)]
               + ([] if args.budget_gb is None else ["--budget-gb", str(args.budget_gb)]))


def physical_cores():
    """Physical cores of the host (lscpu's CORE,SOCKET pairs), else None."""
    import subprocess

    try:
        out = subprocess.run(["lscpu", "-p=CORE,SOCKET"], capture_output=True, text=True,
                             timeout=10).stdout
    except (OSError, subprocess.SubprocessError):
        return None
    pairs = {l for l in out.splitlines() if l and not l.startswith("#")}
    return len(pairs) or None


_NATIVE_TIMING = r"""
import json, sys, time
sys.path.insert(0, sys.argv[1])
import numpy as np
import oracle
from paper_2006_16147_amd import inputs
case = inputs.headline_case(int(sys.argv[2]), seed=1)
t0 = time.perf_counter()
ho = oracle.Hierarchy(case["A"])
t_setup = time.perf_counter() - t0
t0 = time.perf_counter()
x, info = ho.pcg(case["b"], rtol=case["rtol"], maxit=1000)
t_solve = time.perf_counter() - t0
print(json.dumps({"setup_ms": t_setup * 1e3, "solve_ms": t_solve * 1e3,
                  "iterations": info["iterations"], "x_sha": __import__("hashlib").sha256(
                      x.tobytes()).hexdigest()}))
"""


def cpu_baseline(case, gpu_iters, N):
    """The FP64 oracle's solve of the same system on the host, serial (one
    thread): the -O3 -march=native timing build (built here for this host,
    run in a child process) is the reported value; the -O2 test build is
    timed beside it in this process and its solution kept for the
    comparisons. Both builds give the same bits (checked by hash)."""
    import hashlib
    import subprocess

    import oracle

    t0 = time.perf_counter()
    ho = oracle.Hierarchy(case["A"])
    t_setup = time.perf_counter() - t0
    t0 = time.perf_counter()
    x, info = ho.pcg(case["b"], rtol=case["rtol"], maxit=1000)
    t_solve = time.perf_counter() - t0
    native = None
    try:
        lib = oracle.build_oracle(native=True)
        env = dict(os.environ, ORACLE_LIB=lib, OMP_NUM_THREADS="1")
        r = subprocess.run([sys.executable, "-c", _NATIVE_TIMING, ROOT, str(N)], env=env,
                           capture_output=True, text=True, timeout=300)
        if r.returncode == 0:
            native = json.loads(r.stdout.strip().splitlines()[-1])
    except (OSError, subprocess.SubprocessError, ValueError):
        native = None
    same = native is not None and native["x_sha"] == hashlib.sha256(x.tobytes()).hexdigest()
    value = native["solve_ms"] if native and same else t_solve * 1e3
    build = "gcc -O3 -march=native -ffp-contract=off" if native and same else "gcc -O2"
    return {
        "value": round(value, 1),
        "unit": "ms",
        "cores": 1,
        "kind": "oracle",
        "sample": ("one complete FP64 oracle PCG solve of the same 160^3 system to rtol 1e-8 "
                   "(%d iterations; GPU: %d), serial, %s; oracle setup not included"
                   % (info["iterations"], gpu_iters, build)),
        "host_physical_cores": physical_cores(),
        "setup_ms": round(native["setup_ms"] if native and same else t_setup * 1e3, 1),
        "O2_solve_ms": round(t_solve * 1e3, 1),
        "O2_setup_ms": round(t_setup * 1e3, 1),
        "native_bit_identical": same,
        "iterations": info["iterations"],
        "rel_res_true": info["rel_res_true"],
    }, x


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--N", type=int, default=160)
    ap.add_argument("--vcycles", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--mode", default="headline",
                    choices=["headline", "aniso", "batch", "serve", "kcycle", "variants", "coarse",
                             "smoothed"],
                    help="headline (default): the 160^3 benchmark line; the others print "
                         "their own JSON lines")
    ap.add_argument("--rates", default="10,20,50,100,200,500",
                    help="serve mode: arrival rates /s")
    ap.add_argument("--budget-gb", type=float, default=None,
                    help="serve mode: GiB the server may reserve (default: the device's "
                         "memory less 32 GiB)")
    ap.add_argument("--count", type=int, default=200, help="serve mode: requests per rate")
    ap.add_argument("--slots", type=int, default=4, help="serve mode: concurrent slots")
    ap.add_argument("--profile-pass", action="store_true",
                    help="short run for rocprofv3 counter collection")
    ap.add_argument("--ingest-pmc", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write profiles/traffic.json from two counter runs")
    ap.add_argument("--kernel-summary", metavar="KERNEL_TRACE_CSV",
                    help="print a markdown summary of a rocprofv3 kernel trace")
    ap.add_argument("--counter-summary", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="print per-kernel HBM MB from two rocprofv3 counter runs")
    ap.add_argument("--overlap-summary", metavar="KERNEL_TRACE_CSV",
                    help="print the GPU busy fraction and cross-queue overlap of a trace")
    args = ap.parse_args()
    if args.kernel_summary:
        kernel_summary(args.kernel_summary)
        return
    if args.counter_summary:
        counter_summary(*args.counter_summary)
        return
    if args.overlap_summary:
        overlap_summary(args.overlap_summary)
        return
    if args.ingest_pmc:
        ingest_pmc(*args.ingest_pmc)
        return
    if args.profile_pass:
        profile_pass(args.N)
        return
    if args.mode != "headline":
        import torch

        torch.cuda.set_device(0)
        {"aniso": bench_aniso, "batch": bench_batch, "serve": bench_serve,
         "kcycle": bench_kcycle, "variants": bench_variants,
         "coarse": bench_coarse, "smoothed": bench_smoothed}[args.mode](args)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2006_16147_amd import amg, inputs

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    amg.load_library()
    log = lambda *a: print("[bench]", *a, file=sys.stderr, flush=True)  # noqa: E731

    case = inputs.headline_case(args.N, seed=1)
    A = case["A"]
    log("problem %d^3: n=%d nnz=%d" % (args.N, A.n, A.nnz))
    rp = torch.from_numpy(A.row_ptr).to(dev)
    ci = torch.from_numpy(A.col).to(dev)
    va = torch.from_numpy(A.val).to(dev)
    b = torch.from_numpy(case["b"]).to(dev)
    rtol = case["rtol"]

    res = {}
    hier = {}
    for prec, name in ((amg.FP64, "fp64"), (amg.FP32, "fp32_prec")):
        setup_ms = []
        for rep in range(3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            h = amg.amg_setup(rp, ci, va, precision=prec)
            torch.cuda.synchronize()
            setup_ms.append((time.perf_counter() - t0) * 1e3)
            if rep < 2:
                h.close()
        hier[name] = h
        res[name] = {"setup_ms_min": round(min(setup_ms), 2),
                     "setup_stages_ms": {k: round(v, 2) for k, v in h.setup_times().items()},
                     "levels": h.sizes(), "opc": round(h.opc(), 5)}
        log(name, "setup %.1f ms, levels %s" % (min(setup_ms), h.sizes()))

    x = torch.zeros_like(b)

    def one_solve(h):
        x.zero_()
        st, info = amg.amg_pcg_solve(h, b, x, rtol=rtol, maxit=1000)
        if st != amg.Status.OK:
            raise RuntimeError("solve failed: %s" % info)
        return info

    for name in ("fp64", "fp32_prec"):
        h = hier[name]
        for _ in range(args.warmup):
            one_solve(h)
        times = []
        torch.cuda.synchronize()
        t_all = time.perf_counter()
        for _ in range(args.steps):
            t0 = time.perf_counter()
            info = one_solve(h)
            times.append((time.perf_counter() - t0) * 1e3)
        torch.cuda.synchronize()
        total = (time.perf_counter() - t_all) * 1e3
        xg = x.cpu().numpy()
        err_u = float(np.linalg.norm(xg - case["u"]) / np.linalg.norm(case["u"]))
        res[name].update({
            "p50_ms": round(percentile(times, 50), 3), "p99_ms": round(percentile(times, 99), 3),
            "mean_ms": round(total / args.steps, 3), "iterations": info["iterations"],
            "rel_res_true": info["rel_res_true"], "err_vs_u": err_u,
            "ms_per_iteration": round(percentile(times, 50) / max(info["iterations"], 1), 4),
        })
        res[name]["_x"] = xg
        log(name, "solve p50 %.2f ms p99 %.2f ms, %d it, true rel res %.2e" % (
            res[name]["p50_ms"], res[name]["p99_ms"], info["iterations"], info["rel_res_true"]))

    # V-cycle bandwidth: one cycle as the solve runs it, HIP events over
    # back-to-back cycles on the hierarchy's stream (algorithmic bytes /
    # time); the time of a whole amg_vcycle_apply call (permutation to and
    # from the caller's order, host launch cost) is reported beside it
    r = torch.from_numpy(np.random.default_rng(7).uniform(-1, 1, A.n)).to(dev)
    z = torch.zeros_like(r)
    for name, V in (("fp64", 8.0), ("fp32_prec", 4.0)):
        h = hier[name]
        amg.amg_vcycle_apply(h, r, z)  # leaves a live right-hand side in the cycle's input
        ms, by = h.time_kernel(5, 0, reps=args.vcycles)
        for _ in range(3):
            amg.amg_vcycle_apply(h, r, z)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.vcycles):
            amg.amg_vcycle_apply(h, r, z)
        torch.cuda.synchronize()
        ms_apply = (time.perf_counter() - t0) * 1e3 / args.vcycles
        res[name]["vcycle_ms"] = round(ms, 4)
        res[name]["vcycle_gbs"] = round(by / ms / 1e6, 1)
        res[name]["vcycle_bytes"] = by
        res[name]["vcycle_apply_call_ms"] = round(ms_apply, 4)
        log(name, "V-cycle %.3f ms, %.0f GB/s algorithmic (apply call %.3f ms)" % (
            ms, by / ms / 1e6, ms_apply))

    # dominant level-0 kernel of the FP64 solve: each of the three level-0
    # kernels that launch once per iteration timed inside the CG iterations
    # as the solve runs them (HIP events stamped at the start and end of its
    # own dispatch on the hierarchy's stream, three times as many iterations
    # as the solve takes, so that the mean is over 3 x 38 launches at 160^3);
    # the back-to-back loop of the same kernel is reported beside it
    h = hier["fp64"]
    one_solve(h)  # the in-solve timing starts from this right-hand side
    iters = res["fp64"]["iterations"]
    kt, kt_loop = {}, {}
    for k in KERNEL_NAMES:
        kt_loop[k] = h.time_kernel(k, 0, reps=20)
        if k != 2:
            kt[k] = h.time_kernel(k | amg.TIME_IN_SOLVE, 0, reps=3 * iters)
    dom = max(kt, key=lambda k: kt[k][0])
    ms, by = kt[dom]
    achieved = by / ms / 1e6
    traffic = load_traffic("fp64_level0_%d" % dom)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic, "kernel": KERNEL_NAMES[dom] + " (level 0, FP64)",
                "kernel_ms": round(ms, 4),
                "kernel_ms_timing": "in solve, mean of %d launches" % (3 * iters),
                "kernel_ms_back_to_back": round(kt_loop[dom][0], 4), "algorithmic_bytes": by}
    res["level0_kernels"] = {KERNEL_NAMES[k]: {
        "ms_in_solve": round(kt[k][0], 4) if k in kt else None,
        "GB/s_in_solve": round(kt[k][1] / kt[k][0] / 1e6, 1) if k in kt else None,
        "ms_back_to_back": round(v[0], 4), "GB/s_back_to_back": round(v[1] / v[0] / 1e6, 1)}
        for k, v in kt_loop.items()}
    log("dominant kernel:", roofline)

    # the FP64 hierarchy without the exact FP32 copy of level 0's values
    # (AMG_FLAG_NO_VALUE_COMPRESSION): same bits, FP64 value traffic
    hn = amg.amg_setup(rp, ci, va, precision=amg.FP64, flags=amg.FLAG_NO_VALUE_COMPRESSION)
    for _ in range(args.warmup):
        one_solve(hn)
    times = []
    for _ in range(args.steps):
        t0 = time.perf_counter()
        info = one_solve(hn)
        times.append((time.perf_counter() - t0) * 1e3)
    res["fp64_fp64_values_level0"] = {"p50_ms": round(percentile(times, 50), 3),
                                      "p99_ms": round(percentile(times, 99), 3),
                                      "iterations": info["iterations"],
                                      "same_solution": bool(np.array_equal(
                                          x.cpu().numpy(), res["fp64"]["_x"]))}
    hn.close()
    log("fp64 without the FP32 copy of A_0:", res["fp64_fp64_values_level0"])

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle ...")
        cpu, xo = cpu_baseline(case, res["fp64"]["iterations"], args.N)
        for name in ("fp64", "fp32_prec"):
            xg = res[name]["_x"]
            res[name]["rel_diff_vs_oracle"] = float(np.linalg.norm(xg - xo) /
                                                    np.linalg.norm(xo))
        res["fp32_prec"]["rel_diff_vs_oracle_note"] = (
            "FP32 hierarchy and V-cycle, FP64 CG, against the FP64 oracle's solution of the "
            "same system to the same rtol")
        log("cpu baseline:", cpu)
    for name in ("fp64", "fp32_prec"):
        res[name].pop("_x", None)

    line = {
        "metric": METRIC,
        "value": res["fp64"]["p99_ms"],
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res["fp64"]["mean_ms"],
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "poisson7_%d^3_b=Au_seed1_rtol1e-8" % args.N, "n": A.n,
                   "nnz": A.nnz, "rtol": rtol,
                   "hierarchy": "matching, 3 sweeps, w=1, l1-Jacobi 1+1, dense Cholesky <=200",
                   "level0_values": ("FP64 products of level 0 read A from an exact FP32 "
                                     "copy (every value of this A is an FP32 number; same "
                                     "bits): see fp64_fp64_values_level0 for the solve "
                                     "without it")},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "fp64": res["fp64"],
        "fp32_prec": res["fp32_prec"],
        "fp32_prec_speedup_p50": round(res["fp64"]["p50_ms"] / res["fp32_prec"]["p50_ms"], 3),
        "fp64_fp64_values_level0": res["fp64_fp64_values_level0"],
        "level0_kernels": res["level0_kernels"],
        "source_hash": source_hash(),
    }
    for hh in hier.values():
        hh.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
