#!/usr/bin/env python3
"""Throughput of the batch-wise Hamiltonian integration + density update on one MI355X.

A step is one density update n = phi D phi (eq. Density) followed by one Hamiltonian
integration H = phi^T (w v) phi (eq. H_int_aims) over every octree batch of the workload,
with v, D, H and n resident in device memory.  The work measure is the paper's #ops
(Section "GPGPU Acceleration Across Materials and Architectures"): U = sum over batches
of |B| * nnz(B)^2 per operation, so value = 2 U / step time in 1e9 point*basis^2/s.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload slab375|block100|cube8]
                    [--precision fp64] [--no-cpu-baseline]

Prints one JSON line.  Only one GPU is supported: --gpus above 1 exits with a message.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "H-integration + density-update Gpt·basis²/s vs plain FP64; p50/p99 latency"
PEAK = {"fp64": 78.6, "fp32": 157.3, "bf16x3": 2500.0, "bf16x6": 2500.0}  # TFLOP/s, dense MFMA, MI355X
KERNELS_SRC = os.path.join(ROOT, "paper_1912_06636_amd", "csrc", "kernels.hip")
# HBM bytes per launch of the contraction kernels on the default workload, from two rocprofv3
# --pmc passes (FETCH_SIZE, WRITE_SIZE) over "bench.py --steps 1 --warmup 0 --h-tile 64
# --no-cpu-baseline --no-plain --serve-seconds 0 --calibrate-copy 1024", each counter scaled by
# its reading of the 1 GiB plain copy made in that run.  Valid only for the kernel source it was
# taken on (sha256).
TRAFFIC = {"sha256": "cc43f530885cf44543ea0c8c1b09478f283a858a8e67926968cc404d174f67f4",
           "workload": "slab375", "precision": "fp64", "h_tile": 64, "group_max": 256,
           "bytes_per_launch": {"n_f64": 5.800e9, "h_f64": 6.019e9}}
WORKLOADS = {
    "slab375": (4, "375-atom layered slab, 28 NAO/atom (10,500 basis functions, l<=3, 6 A cutoff), "
                   "60x434 grid/atom = 9,765,000 points, octree batches <= 256"),
    "block100": (2, "100-atom jittered simple-cubic block, 14 NAO/atom (1,400 basis functions, 5 A "
                    "cutoff), 50x302 grid/atom = 1,510,000 points, octree batches <= 256"),
    "cube8": (1, "8 atoms in a 6 A cube, 5 NAO/atom (40 basis functions), 30x110 grid/atom = "
                 "26,400 points, octree batches <= 200"),
    "many64": (3, "64 independent structures, 10-200 atoms log-uniform on a jittered simple-cubic "
                  "lattice, 14 NAO/atom, 50x302 grid/atom, octree batches <= 256, all in one "
                  "hipGraph-captured launch sequence (nao_run_many)"),
}


def measured_traffic(workload, prec, h_tile, group_max, kernel, batcher="octree", max_batch=256):
    """Counter-derived HBM bytes per launch of `kernel`, or None when the kernel source or the
    launch configuration differ from the ones the counters were taken on."""
    import hashlib
    with open(KERNELS_SRC, "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()
    t = TRAFFIC
    if (t["sha256"] != sha or t["workload"] != workload or t["precision"] != prec or t["h_tile"] != h_tile
            or t["group_max"] != group_max or batcher != "octree" or max_batch != 256):
        return None
    return t["bytes_per_launch"].get(kernel)


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def batch_measures(sysm):
    """Per-batch |B| and m from the system's batches and lists."""
    perm, bp, lp, li = sysm.get_batches()
    B = np.diff(bp).astype(np.float64)
    m = np.diff(lp).astype(np.float64)
    return perm, bp, lp, li, B, m


def cpu_baseline(work, perm, bp, lp, li, budget_s):
    """The FP64 oracle's batched forms (as they stand) on an evenly spaced sample of batches,
    timed on this host; returns (Gpt*basis^2/s, cores, description)."""
    from oracle import basis as ob
    from oracle import integrals as oi
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info() if i.get("user_api") == "blas"] or [1])
    except Exception:
        cores = os.cpu_count() or 1
    B = ob.Basis(work["basis"])
    nb = len(bp) - 1
    sizes = np.diff(bp)
    ms = np.diff(lp)
    live = np.nonzero(ms > 0)[0]
    # double the sample until one pass (both operations) takes about budget_s / 2
    stride = max(1, len(live) // 64)
    done_units, done_t, used = 0.0, 0.0, 0
    while True:
        sel = live[::stride][:max(1, min(len(live), 64 * (1 + used)))]
        sub_bp = np.concatenate([[0], np.cumsum(sizes[sel])])
        sub_perm = np.concatenate([perm[bp[b]:bp[b + 1]] for b in sel])
        sub_lp = np.concatenate([[0], np.cumsum(ms[sel])])
        sub_li = np.concatenate([li[lp[b]:lp[b + 1]] for b in sel])
        t0 = time.perf_counter()
        oi.hamiltonian_batched(B, work["xyz"], work["w"], work["v"], sub_perm, sub_bp, sub_lp, sub_li)
        oi.density_batched(B, work["xyz"], work["D"], sub_perm, sub_bp, sub_lp, sub_li)
        t = time.perf_counter() - t0
        units = float(np.sum(sizes[sel].astype(np.float64) * ms[sel].astype(np.float64) ** 2))
        done_units, done_t = units, t
        used += 1
        if t >= budget_s / 2 or len(sel) >= len(live) or used > 7:
            break
        stride = max(1, stride // 2)
    rate = 2.0 * done_units / done_t / 1e9
    desc = ("oracle hamiltonian_batched + density_batched (numpy FP64) on %d of %d batches "
            "(every %d-th non-empty batch), %.1f s" % (len(sel), nb, stride, done_t))
    return rate, cores, desc


def bench_many(args, desc):
    """64 structures per step through one captured launch sequence (config-3 shapes)."""
    import torch
    from paper_1912_06636_amd import nao
    from workloads import config_workload
    from workloads.generate import CONFIG3_N_STRUCTURES

    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(device=dev)
    ctx = nao.Context(0, stream=stream.cuda_stream)
    t0 = time.time()
    systems, tens, U, sum_Bm = [], [], 0.0, 0.0
    sample = None  # one structure's inputs and batches for the CPU baseline
    for k in range(CONFIG3_N_STRUCTURES):
        w = config_workload(3, k)
        sysm = nao.build_batches(ctx, w["basis"], w["xyz"], w["w"], w["max_batch"])
        perm, bp, lp, li, Bsz, msz = batch_measures(sysm)
        sum_Bm += float(np.sum(Bsz * msz))
        if sample is None or len(w["xyz"]) > len(sample[0]["xyz"]):
            sample = (w, perm, bp, lp, li)
        if k == 0 and not args.h_tile:
            ht, gm, ms = sysm.autotune(w["v"], w["D"], precision=args.precision, force=True)
            log("autotuned on structure 0: h_tile %d, group_max %d" % (ht, gm))
        elif not args.h_tile:
            sysm.autotune(w["v"], w["D"], precision=args.precision)
        U += sysm.work_units()
        with torch.cuda.stream(stream):
            t = (torch.from_numpy(w["v"]).to(dev), torch.from_numpy(w["D"]).to(dev),
                 torch.empty((sysm.n_basis, sysm.n_basis), dtype=torch.float64, device=dev),
                 torch.empty(sysm.n_points, dtype=torch.float64, device=dev))
        systems.append(sysm)
        tens.append(t)
    torch.cuda.synchronize()
    log("%d structures built in %.1f s (U = %.3g per operation)" % (len(systems), time.time() - t0, U))
    work = []
    for sysm, (v, D, H, n) in zip(systems, tens):
        work += [(sysm, "n", D, n), (sysm, "h", v, H)]

    def timed(fn, steps):
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            ev0.record(stream)
            for _ in range(steps):
                fn()
            ev1.record(stream)
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1) / steps

    def separate():
        for sysm, (v, D, H, n) in zip(systems, tens):
            sysm.update_density(D, precision=args.precision, out=n)
            sysm.integrate_h(v, precision=args.precision, out=H)

    for _ in range(args.warmup):
        ctx.run_many(work, precision=args.precision, capture_graph=True)
    ms_graph = timed(lambda: ctx.run_many(work, precision=args.precision, capture_graph=True), args.steps)
    ms_eager = timed(lambda: ctx.run_many(work, precision=args.precision, capture_graph=False), max(1, args.steps // 2))
    ms_sep = timed(separate, max(1, args.steps // 2))
    value = 2.0 * U / (ms_graph * 1e-3) / 1e9
    log("graph %.2f ms, eager run_many %.2f ms, separate calls %.2f ms" % (ms_graph, ms_eager, ms_sep))
    profs = {}
    for name, fn in (("run_many", lambda: ctx.run_many(work, precision=args.precision, capture_graph=False)),
                     ("separate", separate)):
        ctx.profile(True)
        fn()
        profs[name] = ctx.profile_read()
        ctx.profile(False)
        log("kernels (%s): " % name + ", ".join("%s %d x %.2f ms" % (k, c, t) for k, (c, t) in profs[name].items()))
    # credited work as for the single structure: 2|B|m^2 + 2|B|m (n), |B|m(m+1) + |B|m (H)
    sfx = {"fp64": "f64", "fp32": "f32", "bf16x3": "bf16x3", "bf16x6": "bf16x6"}[args.precision]
    credit = {"h_" + sfx: U + 2.0 * sum_Bm, "n_" + sfx: 2.0 * U + 2.0 * sum_Bm}
    peak = PEAK.get(args.precision, PEAK["fp64"])
    cands = {k: v for k, v in profs["run_many"].items() if k in credit}
    roofline = None
    if cands:
        dom = max(cands, key=lambda k: cands[k][1])
        launches, tot_ms = cands[dom]
        achieved = credit[dom] / (tot_ms * 1e-3) / 1e12
        roofline = {"bound": "mfma", "kernel": dom, "achieved": round(achieved, 3), "peak": peak,
                    "unit": "TFLOP/s", "frac": round(achieved / peak, 4), "traffic": None,
                    "launches": launches, "avg_launch_ms": round(tot_ms / launches, 4),
                    "flops_per_launch": credit[dom] / launches,
                    "kernels": {k: {"launches": c, "ms": round(t, 3),
                                    "frac": round(credit[k] / (t * 1e-3) / 1e12 / peak, 4)}
                                for k, (c, t) in cands.items()}}
    step_flops = sum(credit.values())
    roofline_step = {"flops": step_flops, "achieved": round(step_flops / (ms_graph * 1e-3) / 1e12, 3),
                     "peak": peak, "unit": "TFLOP/s",
                     "frac": round(step_flops / (ms_graph * 1e-3) / 1e12 / peak, 4)}
    cpu = None
    if not args.no_cpu_baseline:
        sw, perm, bp, lp, li = sample
        rate, cores, sdesc = cpu_baseline(sw, perm, bp, lp, li, args.cpu_seconds)
        cpu = {"value": round(rate, 4), "unit": "Gpt·basis²/s", "cores": cores, "kind": "oracle",
               "sample": sdesc + " of the largest structure (%d atoms)" % len(sw["basis"]["atom_xyz"])}
        log("cpu baseline %.4f Gpt*basis^2/s on %d threads" % (rate, cores))
    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "Gpt·basis²/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_graph, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": {"fp64": "f64", "fp32": "f32", "bf16x3": "bf16x3", "bf16x6": "bf16x6"}[args.precision],
        "data": "synthetic (seeded generator; shapes of the paper's workloads)",
        "config": {"workload": "many64", "description": desc, "structures": len(systems), "units_per_op": U,
                   "precision": args.precision},
        "ms_eager_run_many": round(ms_eager, 3), "ms_separate_calls": round(ms_sep, 3),
        "roofline": roofline, "roofline_step": roofline_step, "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    for sysm in systems:
        sysm.close()
    ctx.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="slab375", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default="fp64")
    ap.add_argument("--group-max", type=int, default=256)
    ap.add_argument("--batcher", default="octree", choices=["octree", "cutplane"],
                    help="batching method (the workload's own is the octree)")
    ap.add_argument("--max-batch", type=int, default=0, help="batch size; 0 = the workload's (256)")
    ap.add_argument("--h-tile", type=int, default=0, help="Hamiltonian tile width (64 or 128); 0 = autotune")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true", help="skip timing the plain FP64 per-batch path")
    ap.add_argument("--gradient", action="store_true",
                    help="also time the extended operations: the density with its gradient, the Hamiltonian "
                         "with a vector field and with the kinetic term, and the local Pulay forces")
    ap.add_argument("--resident", action="store_true",
                    help="also time steps with the basis values kept resident across operations (SCF form)")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--serve-seconds", type=float, default=20.0,
                    help="seconds of Poisson arrivals (8 per s) for each serving path; 0 skips serving")
    ap.add_argument("--calibrate-copy", type=int, default=0,
                    help="MiB copied once by a plain device copy (reference for counter scaling)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the grid operations of one structure run on a single "
              "MI355X here (multi-GPU sharding is a design note, not built)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1912_06636_amd import nao
    from workloads import config_workload

    cfg, desc = WORKLOADS[args.workload]
    if args.workload == "many64":
        return bench_many(args, desc)
    t0 = time.time()
    work = config_workload(cfg)
    log("workload %s generated in %.1f s" % (args.workload, time.time() - t0))
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(device=dev)
    ctx = nao.Context(0, stream=stream.cuda_stream)
    t0 = time.time()
    max_batch = args.max_batch or work["max_batch"]
    sysm = nao.build_batches(ctx, work["basis"], work["xyz"], work["w"], max_batch, batcher=args.batcher)
    if args.group_max != 256:
        sysm.set_group_max(args.group_max)
    if args.h_tile:
        sysm.set_h_tile(args.h_tile)
    log("system built in %.1f s: %d %s batches (max %d points), N_b=%d" % (
        time.time() - t0, sysm.n_batches, args.batcher, max_batch, sysm.n_basis))
    perm, bp, lp, li, Bsz, msz = batch_measures(sysm)
    U = float(np.sum(Bsz * msz * msz))
    sum_Bm = float(np.sum(Bsz * msz))
    with torch.cuda.stream(stream):
        v = torch.from_numpy(work["v"]).to(dev)
        D = torch.from_numpy(work["D"]).to(dev)
        H = torch.empty((sysm.n_basis, sysm.n_basis), dtype=torch.float64, device=dev)
        n = torch.empty(sysm.n_points, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    tuned = None
    h_tile_used, group_max_used = args.h_tile or 64, args.group_max
    if not args.h_tile:
        t0 = time.time()
        ht, gm, ms = sysm.autotune(v, D, precision=args.precision, force=True)
        tuned = {"h_tile": ht, "group_max": gm, "best_ms": round(ms, 3)}
        h_tile_used, group_max_used = ht, gm
        log("autotuned in %.1f s: %s" % (time.time() - t0, tuned))

    def step():
        sysm.update_density(D, precision=args.precision, out=n)
        sysm.integrate_h(v, precision=args.precision, out=H)

    if args.calibrate_copy:
        nelem = args.calibrate_copy * (1 << 20) // 8
        src = torch.ones(nelem, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("plain copy of %d MiB done" % args.calibrate_copy)
        del src, dst

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    mid = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    with torch.cuda.stream(stream):
        ev[0].record(stream)
        for k in range(args.steps):
            sysm.update_density(D, precision=args.precision, out=n)
            mid[k].record(stream)
            sysm.integrate_h(v, precision=args.precision, out=H)
            ev[k + 1].record(stream)
    torch.cuda.synchronize()
    t_wall = time.perf_counter() - t_wall
    step_ms = [ev[k].elapsed_time(ev[k + 1]) for k in range(args.steps)]
    n_ms = [ev[k].elapsed_time(mid[k]) for k in range(args.steps)]
    h_ms = [mid[k].elapsed_time(ev[k + 1]) for k in range(args.steps)]
    ms_per_step = ev[0].elapsed_time(ev[-1]) / args.steps
    value = 2.0 * U / (ms_per_step * 1e-3) / 1e9
    log("step %.2f ms (n %.2f, H %.2f), %.1f Gpt*basis^2/s" % (ms_per_step, np.mean(n_ms), np.mean(h_ms), value))

    # per-kernel timing (separate pass: events around every launch, on the stream it runs on); the
    # basis launches run beside the contractions (the library's default), so a contraction's time
    # includes its share of the GPU with them; a second pass with the overlap off times every
    # kernel alone
    ctx.profile(True)
    step()
    prof = ctx.profile_read()
    ctx.profile(False)
    log("kernels: " + ", ".join("%s %d x %.2f ms" % (k, c, t) for k, (c, t) in prof.items()))
    ctx.set_overlap(False)
    ctx.profile(True)
    step()
    prof_alone = ctx.profile_read()
    ctx.profile(False)
    ctx.set_overlap(os.environ.get("NAO_OVERLAP", "1") != "0")  # back to the context's setting
    log("kernels alone: " + ", ".join("%s %d x %.2f ms" % (k, c, t) for k, (c, t) in prof_alone.items()))
    prec = args.precision
    sfx = {"fp64": "f64", "fp32": "f32", "bf16x3": "bf16x3", "bf16x6": "bf16x6"}[prec]
    # algorithmic flops of one call, summed over the octree batches, as the method counts them:
    # the paper's symmetric rank-2k triangle for H and its symmetric product and row dot for n
    credit = {
        "h_" + sfx: U + 2.0 * sum_Bm,        # |B| m (m+1) + |B| m
        "n_" + sfx: 2.0 * U + 2.0 * sum_Bm,  # 2 |B| m^2 + 2 |B| m
    }
    # the density as this library forms it (off-diagonal tiles of D once, doubled), a second,
    # labelled figure: |B| m (m+1) + 3 |B| m
    credit_n_half = U + 3.0 * sum_Bm
    peak = PEAK.get(prec, PEAK["fp64"])
    cands = {k: v for k, v in prof.items() if k in credit}
    dom = max(cands, key=lambda k: cands[k][1]) if cands else None
    roofline = None
    if dom:
        launches, tot_ms = cands[dom]
        achieved = credit[dom] / (tot_ms * 1e-3) / 1e12
        roofline = {"bound": "mfma", "kernel": dom, "achieved": round(achieved, 3), "peak": peak,
                    "unit": "TFLOP/s", "frac": round(achieved / peak, 4),
                    "traffic": measured_traffic(args.workload, prec, h_tile_used, group_max_used, dom,
                                                args.batcher, max_batch),
                    "launches": launches, "avg_launch_ms": round(tot_ms / launches, 4),
                    "flops_per_launch": credit[dom] / launches,
                    "kernels": {k: {"launches": c, "ms": round(t, 3),
                                    "frac": round(credit[k] / (t * 1e-3) / 1e12 / peak, 4)}
                                for k, (c, t) in cands.items()}}
        if "n_" + sfx in cands:
            t = cands["n_" + sfx][1]
            roofline["kernels"]["n_" + sfx]["frac_half_credit"] = round(credit_n_half / (t * 1e-3) / 1e12 / peak, 4)
        roofline["kernels_alone"] = {k: {"launches": c, "ms": round(t, 3),
                                         "frac": round(credit[k] / (t * 1e-3) / 1e12 / peak, 4)}
                                     for k, (c, t) in prof_alone.items() if k in credit}
    # the whole step (basis evaluation included) against the same peak
    step_flops = credit["h_" + sfx] + credit["n_" + sfx]
    roofline_step = {"flops": step_flops, "achieved": round(step_flops / (ms_per_step * 1e-3) / 1e12, 3),
                     "peak": peak, "unit": "TFLOP/s",
                     "frac": round(step_flops / (ms_per_step * 1e-3) / 1e12 / peak, 4)}
    log("step at %.1f %% of the %s MFMA peak (credited work)" % (100 * roofline_step["frac"], prec))

    # the plain FP64 per-batch path on the same inputs (every octree batch its own unit, FP64),
    # outside the timed region: the reference the metric's "vs plain FP64" compares with
    plain = None
    if not args.no_plain:
        sysm.set_group_max(0)
        if h_tile_used != 64:
            sysm.set_h_tile(64)
        def plain_step():
            sysm.update_density(D, precision="fp64", out=n)
            sysm.integrate_h(v, precision="fp64", out=H)
        plain_step()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        with torch.cuda.stream(stream):
            e0.record(stream)
            for _ in range(2):
                plain_step()
            e1.record(stream)
        torch.cuda.synchronize()
        plain_ms = e0.elapsed_time(e1) / 2
        plain = {"ms_per_step": round(plain_ms, 3), "value": round(2.0 * U / (plain_ms * 1e-3) / 1e9, 3),
                 "speedup": round(plain_ms / ms_per_step, 3)}
        log("plain FP64 per-batch path: %.2f ms per step (%.2fx slower)" % (plain_ms, plain_ms / ms_per_step))

    resident = None
    if args.resident:
        # the SCF form: the geometry is fixed, so the basis values are evaluated once and reused
        sysm.set_group_max(group_max_used)
        sysm.set_h_tile(h_tile_used)
        sysm.set_resident_basis(True)
        step()  # evaluates and stores the basis values
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        with torch.cuda.stream(stream):
            e0.record(stream)
            for _ in range(args.steps):
                step()
            e1.record(stream)
        torch.cuda.synchronize()
        r_ms = e0.elapsed_time(e1) / args.steps
        resident = {"ms_per_step": round(r_ms, 3), "value": round(2.0 * U / (r_ms * 1e-3) / 1e9, 3),
                    "vs_step": round(ms_per_step / r_ms, 3),
                    "device_bytes": int(sysm.info()[3])}
        log("resident basis values: %.2f ms per step (%.2fx the full step)" % (r_ms, ms_per_step / r_ms))
        sysm.set_resident_basis(False)

    grad = None
    if args.gradient and prec in ("fp64", "fp32"):
        # the extended operations on the same inputs and grouping as the timed step
        sysm.set_group_max(group_max_used)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

        def time_op(op):
            """Mean of two calls on the library's stream, then one profiled call (ms per kernel)."""
            op()
            torch.cuda.synchronize()
            with torch.cuda.stream(stream):
                e0.record(stream)
                for _ in range(2):
                    op()
                e1.record(stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / 2
            ctx.profile(True)
            op()
            prof = ctx.profile_read()
            ctx.profile(False)
            return ms, {k: round(t, 3) for k, (c, t) in prof.items()}

        n_mean, h_mean = float(np.mean(n_ms)), float(np.mean(h_ms))
        peak = PEAK.get(prec, PEAK["fp64"])

        def mfma_rate(kern, name, flops):
            """Credited TFLOP/s of one contraction kernel and its fraction of the MFMA peak."""
            t = kern.get(name)
            if not t:
                return None
            tf = flops / (t * 1e-3) / 1e12
            return {"kernel": name, "achieved": round(tf, 3), "peak": peak, "unit": "TFLOP/s",
                    "frac": round(tf / peak, 4), "flops": flops}

        gn = torch.empty((sysm.n_points, 3), dtype=torch.float64, device=dev)
        g_ms, kern = time_op(lambda: sysm.update_density_gradient(D, precision=prec, out=n, out_grad=gn))
        # full product Phi D (2|B|m^2) and four row dots (8|B|m)
        grad = {"ms": round(g_ms, 3), "vs_density": round(g_ms / n_mean, 3),
                "gpt_basis2_per_s": round(U / (g_ms * 1e-3) / 1e9, 3), "kernels_ms": kern,
                "mfma": mfma_rate(kern, "ngrad_" + sfx, 2.0 * U + 8.0 * sum_Bm)}
        log("density + gradient: %.2f ms (%.2fx the density alone); kernels: %s" % (g_ms, g_ms / n_mean, kern))
        del gn
        # Hamiltonian with a seeded vector field (the GGA term), and with the kinetic term
        a = torch.from_numpy(0.3 * np.random.default_rng(99).normal(size=(sysm.n_points, 3))).to(dev)
        ms, kern = time_op(lambda: sysm.integrate_h_gga(v, a, precision=prec, out=H))
        # two products per upper-triangle tile pair: 2 |B| m (m+1)
        grad["hamiltonian_with_field"] = {"ms": round(ms, 3), "vs_hamiltonian": round(ms / h_mean, 3),
                                          "kernels_ms": kern,
                                          "mfma": mfma_rate(kern, "hgga_" + sfx, 2.0 * U + 2.0 * sum_Bm)}
        log("hamiltonian with a vector field: %.2f ms (%.2fx the local one); kernels: %s" % (ms, ms / h_mean, kern))
        ms, kern = time_op(lambda: sysm.integrate_h_ks(v, precision=prec, out=H))
        grad["hamiltonian_kinetic"] = {"ms": round(ms, 3), "vs_hamiltonian": round(ms / h_mean, 3),
                                       "kernels_ms": kern,
                                       "mfma": mfma_rate(kern, "hks_" + sfx, 2.0 * U + 2.0 * sum_Bm)}
        log("hamiltonian with the kinetic term: %.2f ms (%.2fx the local one); kernels: %s" % (ms, ms / h_mean, kern))
        del a
        # local Pulay forces with a seeded energy-weighted density matrix
        from workloads.generate import energy_weighted_for
        Q = torch.from_numpy(energy_weighted_for(work, 1)).to(dev)
        F = torch.empty((sysm.n_atoms, 3), dtype=torch.float64, device=dev)
        ms, kern = time_op(lambda: sysm.pulay_forces(D, Q, v, precision=prec, out=F))
        # two full products (4|B|m^2), row weights (2|B|m) and three column dots (6|B|m)
        grad["pulay_forces"] = {"ms": round(ms, 3), "vs_density": round(ms / n_mean, 3), "kernels_ms": kern,
                                "mfma": mfma_rate(kern, "nforce_" + sfx, 4.0 * U + 8.0 * sum_Bm)}
        log("local Pulay forces: %.2f ms (%.2fx the density alone); kernels: %s" % (ms, ms / n_mean, kern))
        del Q, F

    n_points, n_basis, n_batches = int(sysm.n_points), int(sysm.n_basis), int(sysm.n_batches)
    serving = None
    if args.serve_seconds > 0:
        # continuous-batching serving of SCF-iteration requests (density update then H) for a pool
        # of 20-400-atom structures: request latency p50/p99 of the plain FP64 path and of the
        # batched reduced-precision path at the same arrival rate
        from paper_1912_06636_amd import serve
        del D, v, H, n
        sysm.close()
        torch.cuda.synchronize()
        t0 = time.time()
        pool = serve.make_pool(6)
        serve.measure_pool(nao, pool)
        log("serving pool (%s atoms) ready in %.1f s" % ([len(w["basis"]["atom_xyz"]) for w in pool],
                                                         time.time() - t0))
        serving = {"lambda_per_s": 8.0, "seconds": args.serve_seconds}
        for path, sprec in (("plain", "fp64"), ("batched", "fp32")):
            r = serve.run(nao, torch, pool, 8.0, args.serve_seconds, 10 ** 6, path, precision=sprec,
                          hbm_budget=160 << 30, log=log)
            serving[path] = {k: r[k] for k in ("precision", "completed", "requests_per_s", "gpt_basis2_per_s",
                                               "p50_ms", "p99_ms", "backlog_at_end")}
        sysm = None

    cpu = None
    if not args.no_cpu_baseline:
        rate, cores, sdesc = cpu_baseline(work, perm, bp, lp, li, args.cpu_seconds)
        cpu = {"value": round(rate, 4), "unit": "Gpt·basis²/s", "cores": cores, "kind": "oracle",
               "sample": sdesc}
        log("cpu baseline %.4f Gpt*basis^2/s on %d threads" % (rate, cores))

    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "Gpt·basis²/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "bf16x3": "bf16x3", "bf16x6": "bf16x6"}[prec],
        "data": "synthetic (seeded generator; shapes of the paper's workloads)",
        "config": {"workload": args.workload, "description": desc, "n_points": n_points,
                   "n_basis": n_basis, "n_batches": n_batches, "units_per_op": U,
                   "group_max": args.group_max, "h_tile": args.h_tile, "precision": prec,
                   "batcher": args.batcher, "max_batch": max_batch,
                   "mean_batch": round(float(n_points) / max(1, n_batches), 2),
                   "autotuned": tuned},
        "latency_ms": {"p50": round(float(np.percentile(step_ms, 50)), 3),
                       "p99": round(float(np.percentile(step_ms, 99)), 3)},
        "ops_ms": {"density": round(float(np.mean(n_ms)), 3), "hamiltonian": round(float(np.mean(h_ms)), 3)},
        "wall_s_timed": round(t_wall, 3),
        "plain_fp64_per_batch": plain,
        "density_gradient": grad,
        "resident_basis": resident,
        "roofline": roofline,
        "roofline_step": roofline_step,
        "serving": serving,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    if sysm is not None:
        sysm.close()
    ctx.close()


if __name__ == "__main__":
    main()
