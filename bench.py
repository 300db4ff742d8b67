#!/usr/bin/env python3
"""Benchmark: per-tree split search on one MI355X.

Default (`--workload headline`): the 50M-row, 10-class MultiClass workload
(the largest configuration, depth 10, 230 histogram columns at 255 bins) is
the headline; the 1M-row RMSE workload follows as a second block of the same
JSON line. `--workload c2|c3|c5` runs one workload alone, `--workload c4` the
batching workload (64 independent problems, and the 1M-row problem as
cross-validation folds and as ordered-boosting permutations), `apply` and
`combine` the model-apply and feature-combination workloads.

A step is one boosting iteration: every level's histogram build, scoring,
argmax and leaf update, then the leaf solve and the model/gradient update.
The once-per-dataset steps (borders, bins, ordered statistics) are timed in
the same run and reported beside it. Inputs are resident in HBM before the
timed region starts.

The data are prepared once; then every histogram form is timed on them in
turn: the headline form (float64 LDS accumulation, the fastest float form on
gfx950, which meets the 1e-5 error bar) and, beside it on the same launch
plan, plain float32 accumulation, compensated float32 (TwoSum pairs) and
int16 codes. Each form is autotuned first where the workload asks for it
(untimed), then warm-up trees run, one tree per permutation is captured into
a HIP graph, and the timed trees are replayed with events around the whole
loop (the comparison forms with fewer trees). The histogram build is then
timed inside trees: more trees are replayed from graphs that hold
device-clock stamps around every build. After timing, one more tree is grown
level by level and its histograms on sampled features are kept; the oracle
leg at the end (with the CPU timing of the oracle) compares them with FP64
and reports the largest normalised error.

Prints one JSON line. `value` is the headline form's whole-step throughput
in 1e9 (rows x features x levels) per second; `roofline` gives the
histogram build's algorithmic HBM bytes over its stamp-timed duration
against 8 TB/s, and beside it (`lds_issue`) the fraction of that duration
the build's LDS atomics need at the measured per-CU issue rates.
"""
from __future__ import annotations

import argparse
import copy
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "sec/tree and histogram G row-features/s vs plain FP32, ≤1e-5 rel err"
PEAK_HBM_GBS = 8000.0
PRECISIONS = {"fp32": 0, "twofloat": 1, "int16": 2, "f64": 3}
DTYPES = {"fp32": "f32", "twofloat": "f32x2", "int16": "i16->i64", "f64": "f64"}


def hist_bytes_per_level(n, F, K, level, rmse, precision, bin_bits=8):
    """Algorithmic bytes one histogram build must read: the bin of every
    (row, feature) (a byte, or bin_bits bits when packed), the row's gradient
    statistics and (after level 0) its leaf."""
    if precision == 2:
        grad = 4 * K                       # int16 (g, h) code pair
    else:
        grad = 4 * K if rmse else 8 * K    # g (and h) float32
    leaf = 2 if level > 0 else 0
    return n * F * bin_bits // 8 + n * grad + n * leaf


# LDS atomic issue rates (lane updates per clock per CU, the 64 lanes of a
# wave on distinct banks), measured in the same run by cbh_probe_lds_rates;
# 256 CUs at 2.4 GHz.
LDS_RATE = {}
CU_CLOCKS_PER_S = 256 * 2.4e9


def measure_lds_rates():
    """Fill LDS_RATE once from the library's probe."""
    if not LDS_RATE:
        from paper_1810_11363_amd import cbhip as cb
        ctx = cb.cbh_create(0)
        try:
            LDS_RATE.update({k: round(v, 3) for k, v in cb.cbh_probe_lds_rates(ctx).items()})
        finally:
            cb.cbh_destroy(ctx)
    return dict(LDS_RATE)


def lds_ops_per_level(n, F, K, rmse, precision):
    """LDS atomics one full-rows histogram build issues, by instruction (the
    float64 and int16 forms; the compare-and-swap forms have no fixed count)."""
    if precision == 3:
        return {"ds_add_f64": n * F * K, "ds_add_u32": n * F} if rmse else \
            {"ds_add_f64": n * F * 2 * K}
    if precision == 2:
        return {"ds_add_u64": n * F * K}
    return None


def lds_floor_s(ops):
    """Seconds the LDS needs for `ops` at the measured issue rates."""
    return sum(c / (LDS_RATE[op] * CU_CLOCKS_PER_S) for op, c in ops.items())


def cpu_info():
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count()
    return {"cpu_model": model, "logical_cpus": os.cpu_count(), "cpus_available": avail}


# Workloads: "headline" runs c5 then c2 (see the module docstring).
WORKLOADS = {
    "c2": dict(tag="c2_1m_rmse", n=1_000_000, steps=200, cpu_rows=1_000_000, cpu_trees=20),
    "c3": dict(tag="c3_10m_logloss", n=10_000_000, steps=20, cpu_rows=250_000, cpu_trees=2),
    "c4": dict(tag="c4_batch_rmse", n=0, steps=20, cpu_rows=1_000_000, cpu_trees=1),
    "c5": dict(tag="c5_50m_multiclass", n=50_000_000, steps=20, cpu_rows=100_000, cpu_trees=1,
               warmup=5, hist_trees=2, autotune="off", compare="fp32,twofloat,int16",
               warmup_s=0.0, compare_steps=2),
    "apply": dict(tag="apply_100k_8000_trees", n=100_000, steps=20, cpu_rows=20_000, cpu_trees=0),
    "combine": dict(tag="combine_10m_pairs", n=10_000_000, steps=10, cpu_rows=1_000_000,
                    cpu_trees=0),
    "packed": dict(tag="packed_10m_logloss", n=10_000_000, steps=20, cpu_rows=0, cpu_trees=0,
                   hist_trees=4, autotune="off", warmup_s=0.5),
    "combotrees": dict(tag="combo_trees_1m_rmse", n=1_000_000, steps=10, warmup=2,
                       cpu_rows=20_000, cpu_trees=0),
}
# per-run defaults a workload may override
RUN_DEFAULTS = dict(warmup=5, hist_trees=40, autotune="run", compare="fp32,twofloat,int16",
                    warmup_s=1.0, compare_steps=None)


def describe(workload, p, bst):
    n, F, depth = bst.n, bst.F, bst.depth
    if workload == "c2":
        return (f"1M-row RMSE: n={n}, 100 numeric features at 128 bins + 10 categorical -> "
                f"{F - 100} ordered-statistic columns per tree, 4 permutations, depth {depth}, "
                f"lr 0.1, l2 3")
    if workload == "c5":
        return (f"50M-row MultiClass: n={n}, 50 numeric features at {bst.B} bins + 20 "
                f"categorical (cardinality 10..1e6, Zipf 1.05) -> {F - 50} one-vs-rest "
                f"ordered-statistic columns, K={bst.K} classes, depth {depth}, lr 0.1, l2 3")
    return (f"10M-row precision Logloss: n={n}, {F} uniform numeric features at {bst.B} bins "
            f"(5% exact duplicates), 1% positives, depth {depth}, lr 0.1, l2 3")


def counters_path(workload):
    return os.path.join(ROOT, "profiles", f"hist_{WORKLOADS[workload]['tag']}_counters.json")


COUNTERS = counters_path("c2")
COUNTED_SOURCES = ("paper_1810_11363_amd/csrc/kernels_dev.h",
                   "paper_1810_11363_amd/csrc/histogram.hip",
                   "paper_1810_11363_amd/csrc/partition.hip")


def measured_traffic(form: str, workload: str = "c2"):
    """HBM bytes per histogram build (fetch + write, hardware counters scaled
    by a plain copy's reading), as recorded beside the kernel sources they
    were taken on; None when the sources have changed since or when no
    counters were recorded for the workload."""
    import hashlib
    try:
        rec = json.load(open(counters_path(workload)))
        h = hashlib.sha256()
        for f in COUNTED_SOURCES:
            h.update(open(os.path.join(ROOT, f), "rb").read())
        if h.hexdigest() != rec["source_sha256"]:
            return None
        return int(rec["forms"][form]["build_hbm_bytes"])
    except (OSError, KeyError, ValueError):
        return None


def cpu_baseline(p, rows: int, trees: int):
    """The oracle as it stands, on a row sample of the same workload."""
    import numpy as np

    import oracle
    from oracle import boost
    n_full = p.n
    rows = min(rows, n_full)
    sub = np.sort(np.random.default_rng(0).choice(n_full, rows, replace=False))
    p.x_num = np.ascontiguousarray(p.x_num[:, sub])
    p.cat = np.ascontiguousarray(p.cat[:, sub])
    p.label = np.ascontiguousarray(p.label[sub])
    p.y_num = np.ascontiguousarray(p.y_num[:, sub])
    # each permutation restricted to the sample, rows renumbered 0..rows-1
    if p.perms.shape[0]:
        p.perms = np.stack([np.searchsorted(sub, perm[np.isin(perm, sub)]).astype(np.int32)
                            for perm in p.perms])
    else:
        p.perms = np.zeros((0, rows), np.int32)
    prep = boost.prepare(p)
    approx = np.zeros((p.K, p.n))
    B = max(int(prep.nb_num.max()), prep.nb_ts)
    bins, nb = prep.tree_features(0)
    boost.fit_tree(bins, nb, approx, p.label, p.loss, p.K, p.depth, p.lr, p.l2, B)   # warm
    t0 = time.perf_counter()
    for t in range(trees):
        bins, nb = prep.tree_features(t)
        boost.fit_tree(bins, nb, approx, p.label, p.loss, p.K, p.depth, p.lr, p.l2, B)
    dt = (time.perf_counter() - t0) / trees
    F = bins.shape[0]
    return {"value": round(rows * F * p.depth / dt / 1e9, 6), "unit": "G row-features/s",
            "cores": oracle.num_threads(), "kind": "oracle",
            "sample": (f"{rows} of {n_full} rows" + (" (uniform sample)" if rows < n_full
                                                         else " (the whole workload)") +
                       f", {trees} trees after 1 warm tree; oracle sec/tree {dt:.3f}; "
                       f"borders/bins/statistics before it are not timed"),
            "sec_per_tree": round(dt, 4)}


def hist_f64(raw, L, F, B, K, precision, rmse):
    """Device histogram bytes -> float64 [L][F][B][2K] (counts as integers)."""
    import numpy as np
    import torch
    if precision == 0:
        u = raw[: L * F * B * 2 * K * 4].view(torch.int32).cpu().numpy()
        out = u.view(np.float32).astype(np.float64).reshape(L, F, B, 2 * K)
        if rmse:
            out[..., 1::2] = u.reshape(L, F, B, 2 * K)[..., 1::2].astype(np.uint32)
        return out
    if precision in (1, 3):
        u = raw[: L * F * B * 2 * K * 8].view(torch.int32).cpu().numpy()
        pair = u.view(np.float32).reshape(L, F, B, 2 * K, 2).astype(np.float64)
        out = pair[..., 0] + pair[..., 1]
        if rmse:
            out[..., 1::2] = u.reshape(L, F, B, 2 * K, 2)[..., 0][..., 1::2].astype(np.uint32)
        return out
    return raw[: L * F * B * 2 * K * 8].view(torch.int64).cpu().numpy().reshape(L, F, B, 2 * K)


def snapshot_tree(bst, t, rng, n_feat=4):
    """Grow tree t level by level with the booster's own calls and keep, for
    sampled features, every level's GPU histogram with the inputs that define
    it (bins, the GPU's float32 gradients, leaf indices); the oracle leg
    compares them with FP64 later."""
    import numpy as np
    import torch

    from paper_1810_11363_amd import cbhip as cb
    pr = bst.probs[t % bst.s]
    if bst.precision == 2:
        cb.cbh_quantize_gradients(bst.ctx, pr, bst.stream)
    torch.cuda.synchronize()
    bins = bst.bins_host(t % bst.s)
    g = bst.g.cpu().numpy().astype(np.float64)
    h = bst.h.cpu().numpy().astype(np.float64) if bst.loss != 0 else np.ones_like(g)
    levels = []
    # leaf indices on the host from the chosen splits (the device may keep the
    # rows in leaf order until the last level)
    leaf = np.zeros(bst.n, np.uint16)
    for lvl in range(bst.depth):
        L = 1 << lvl
        bst.build_level_histograms(pr, lvl)
        cb.cbh_score_splits(bst.ctx, pr, lvl, bst.hist_ptr(lvl), bst.precision, bst.l2,
                            bst.split_ptr(lvl), None, bst.stream)
        torch.cuda.synchronize()
        got = hist_f64(bst.hists[lvl % 2], L, bst.F, bst.B, bst.K, bst.precision, bst.loss == 0)
        if bst.precision == 2:
            sc = bst.grad_scale.cpu().numpy().astype(np.float64)
            got = got.astype(np.float64)
            got[..., 0::2] *= sc[:, 0]
            if bst.loss != 0:
                got[..., 1::2] *= sc[:, 1]
        fs = np.sort(rng.choice(bst.F, n_feat, replace=False))
        levels.append((L, fs, leaf.copy(), got[:, fs]))
        f, k = (int(v) for v in bst.best[lvl, :2].cpu().numpy())
        if 0 <= f < bst.F:
            leaf |= ((bins[f] > k).astype(np.uint16) << lvl)
        bst.advance(pr, lvl)
    cb.cbh_update_approx(bst.ctx, pr, bst.hist_ptr(bst.depth - 1), bst.precision,
                         bst.split_ptr(bst.depth - 1), bst.lr, bst.l2, bst.leaf_values, None,
                         bst.stream)
    torch.cuda.synchronize()
    scale = bst.grad_scale.cpu().numpy().astype(np.float64) if bst.precision == 2 else None
    return {"bins": bins, "g": g, "h": h, "B": bst.B, "levels": levels, "scale": scale,
            "rmse": bst.loss == 0}


def oracle_error(snap):
    """Largest error of the snapshot's histograms against the FP64 oracle,
    normalised by the sum of magnitudes of each bin's terms; for int16 codes
    also the largest g-sum error over its quantisation bound
    n_bin * s_g * (1/2 + 2^-9), which must be <= 1: each code is
    rint(fl(g / s_g)), and the float32 quotient is within 2^-24 |g / s_g| <=
    2^-9 of g / s_g."""
    import numpy as np

    import oracle
    worst, worst_q = 0.0, None
    for L, fs, leaf, got in snap["levels"]:
        bins = snap["bins"][fs]
        want = oracle.histogram(bins, snap["g"], snap["h"], leaf, L, snap["B"])
        mag = oracle.histogram(bins, np.abs(snap["g"]), np.abs(snap["h"]), leaf, L, snap["B"])
        m = mag > 0
        worst = max(worst, float((np.abs(got - want)[m] / mag[m]).max()))
        if snap["scale"] is not None:
            one = np.ones_like(snap["g"])
            cnt = oracle.histogram(bins, one, one, leaf, L, snap["B"])[..., 1::2]
            bound = cnt * snap["scale"][:, 0] * (0.5 + 2.0**-9)
            err = np.abs(got[..., 0::2] - want[..., 0::2])
            q = float((err[bound > 0] / bound[bound > 0]).max())
            worst_q = q if worst_q is None else max(worst_q, q)
    return worst, worst_q


def warm_for(bst, seconds, t0, eager):
    """Replay (or grow, if eager) trees for `seconds` of wall time."""
    import torch
    t_end = time.perf_counter() + seconds
    k = t0
    while time.perf_counter() < t_end:
        for _ in range(8):
            if eager:
                bst.fit_tree(k)
            else:
                bst.replay_tree(k)
            k += 1
        torch.cuda.synchronize()


def time_form(bst, name, args, rmse):
    import numpy as np
    import torch

    from paper_1810_11363_amd import cbhip as cb
    prec = PRECISIONS[name]
    # every form on the headline form's plan (histogram subtraction on or
    # off for all), so that the forms differ in their arithmetic only
    bst.set_precision(prec, subtract=args.subtract)
    n, F, K, depth, stream = bst.n, bst.F, bst.K, bst.depth, bst.stream
    bst.init_gradients()
    t_tune = 0.0
    if args.autotune == "run":
        t_tune = time.perf_counter()
        if prec == 2:
            cb.cbh_quantize_gradients(bst.ctx, bst.probs[0], stream)
        cb.cbh_autotune(bst.ctx, bst.probs[0], prec, bst.subtract, args.autotune_save, stream)
        t_tune = time.perf_counter() - t_tune
    elif args.autotune != "off":
        cb.cbh_autotune_load(bst.ctx, args.autotune)
    for t in range(args.warmup):
        bst.fit_tree(t)
    torch.cuda.synchronize()
    # timed region: whole trees replayed from HIP graphs (one per permutation),
    # after `--warmup-s` seconds of the same replays: the clocks settle below
    # their first-burst level within about a second of sustained work, and the
    # timed figure is the sustained one
    if not args.no_graph:
        bst.capture_trees()
    warm_for(bst, args.warmup_s, args.warmup, args.no_graph)
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        start.record(stream)
        t_wall = time.perf_counter()
        for s in range(args.steps):
            if args.no_graph:
                bst.fit_tree(args.warmup + s)
            else:
                bst.replay_tree(args.warmup + s)
        stop.record(stream)
    torch.cuda.synchronize()
    t_wall = time.perf_counter() - t_wall
    cb.cbh_sync(bst.ctx, stream)
    total_ms = start.elapsed_time(stop)
    # the histogram build alone, inside real trees: one more graph per tree
    # with device-clock stamps around every build, the trees replayed back to
    # back as in the timed loop, the stamps read once at the end
    n_hist = max(1, args.hist_trees)
    hist_ms = np.zeros((n_hist, depth))
    if not args.no_graph:
        timing = "device-clock stamps around every build, captured in the tree graphs"
        khz = cb.cbh_device_clock_khz(bst.ctx)
        buf = torch.zeros(n_hist * depth * 2, dtype=torch.int64, device=bst.device)
        timed = [bst.capture_tree(args.warmup + args.steps + s,
                                  stamps=buf.data_ptr() + 8 * 2 * depth * s)
                 for s in range(n_hist)]
        warm_for(bst, args.warmup_s, args.warmup, False)   # settle again after the captures
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        with torch.cuda.stream(stream):
            e0.record(stream)
            for g in timed:
                cb.cbh_graph_launch(g, stream)
            e1.record(stream)
        torch.cuda.synchronize()
        stamped_tree_ms = e0.elapsed_time(e1) / n_hist
        v = buf.view(n_hist, depth, 2).cpu().numpy()
        hist_ms[:] = (v[:, :, 1] - v[:, :, 0]) / khz
        for g in timed:
            cb.cbh_graph_destroy(g)
    else:
        stamped_tree_ms = None
        timing = "events around the builds of eagerly launched trees"
        ev = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(depth)] for _ in range(n_hist)]
        with torch.cuda.stream(stream):
            for s in range(n_hist):
                bst.fit_tree(args.warmup + args.steps + s, events=ev[s])
        torch.cuda.synchronize()
        hist_ms[:] = [[ev[s][l][0].elapsed_time(ev[s][l][1]) for l in range(depth)]
                      for s in range(n_hist)]
    sec_per_tree = total_ms / 1e3 / args.steps
    rf_per_tree = n * F * depth
    bytes_lvl = np.array([hist_bytes_per_level(n, F, K, l, rmse, prec, bst.bin_bits)
                          for l in range(depth)])
    hist_s_per_tree = hist_ms.sum(axis=1).mean() / 1e3
    achieved = float(bytes_lvl.sum() / hist_s_per_tree / 1e9)
    # rows each level's build accumulates (the smaller child only, where a
    # level is built by subtraction), from the last tree's leaf sizes
    counts = torch.bincount(bst.leaf.to(torch.int64), minlength=1 << depth).cpu().numpy()
    rows_lvl = executed_rows(counts, depth, bst.subtract_levels())
    lds_issue = None
    if lds_ops_per_level(1, F, K, rmse, prec) is not None:
        ops = {}
        for r in rows_lvl:
            for op, c in lds_ops_per_level(int(r), F, K, rmse, prec).items():
                ops[op] = ops.get(op, 0) + c
        floor = lds_floor_s(ops)
        lds_issue = {"ops_per_tree": ops, "floor_ms_per_tree": round(floor * 1e3, 3),
                     "measured_ms_per_tree": round(hist_s_per_tree * 1e3, 3),
                     "frac": round(floor / hist_s_per_tree, 4),
                     "rates_lane_ops_per_clk_per_cu": {k: LDS_RATE[k] for k in ops},
                     "rates_source": "cbh_probe_lds_rates, this run"}
    snap = snapshot_tree(bst, args.warmup + args.steps + n_hist, np.random.default_rng(1)) \
        if not args.no_cpu else None
    print(f"# {name}: {sec_per_tree * 1e3:.3f} ms/tree, hist {hist_s_per_tree * 1e3:.3f} ms",
          file=sys.stderr, flush=True)
    return {
        "sec_per_tree": round(sec_per_tree, 6),
        "ms_per_step": round(total_ms / args.steps, 4),
        "G_row_features_per_s": round(rf_per_tree / sec_per_tree / 1e9, 3),
        "hist_G_row_features_per_s": round(rf_per_tree / hist_s_per_tree / 1e9, 3),
        "hist_ms_per_level": [round(float(x), 4) for x in hist_ms.mean(axis=0)],
        "hist_subtraction": bool(bst.subtract_levels()),
        "rows_accumulated_per_level": [int(r) for r in rows_lvl],
        "rows_in_leaf_order": bool(bst.use_part),
        "graph_replay": not args.no_graph,
        "hist_timing": timing,
        "ms_per_tree_while_timing_builds": (round(stamped_tree_ms, 4)
                                            if stamped_tree_ms is not None else None),
        "max_norm_err_vs_fp64": None,      # filled by the oracle leg
        "_snapshot": snap,
        "autotune_s": round(t_tune, 2),
        "wall_s_timed": round(t_wall, 3),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4),
                     "traffic": measured_traffic(name, args.workload),
                     "kernel": "cbh_build_histograms / cbh_apply_build_histograms_sub / "
                               "cbh_part_build_histograms (LDS histogram + partial merge)",
                     "algorithmic_bytes_per_launch": int(bytes_lvl.mean()),
                     "avg_launch_ms": round(float(hist_ms.mean()), 5),
                     "lds_issue": lds_issue},
    }


def executed_rows(counts, depth, sub_levels):
    """Rows accumulated by each level's build: all n, or at a level built by
    subtraction the smaller child of every parent (by row count), from the
    final leaf sizes `counts` [2^depth] (leaf bit l = level l's split)."""
    import numpy as np
    n = int(counts.sum())
    out = []
    for lvl in range(depth):
        if lvl == 0 or not sub_levels:
            out.append(n)
            continue
        L = 1 << lvl
        size = np.bincount(np.arange(1 << depth) & (L - 1), weights=counts, minlength=L)
        half = L // 2
        out.append(int(np.minimum(size[:half], size[half:]).sum()))
    return out


def batch_vs_one_by_one(ctx, probs, hists, lvs, prec, lr, l2, side, timed):
    """ms per iteration of the problems batched in one plan (one captured
    graph), and of the same problems each from a one-problem plan and graph
    replayed one after another (the same kernels, P times the launches)."""
    import torch

    from paper_1810_11363_amd import cbhip as cb
    P = len(probs)
    depth = probs[0].depth
    best = torch.zeros((P, depth, 4), dtype=torch.int32, device=hists[0].device)
    plan = cb.cbh_batch_create(ctx, probs, prec, hists, best)
    singles = [cb.cbh_batch_create(ctx, [probs[i]], prec, [hists[i]], best[i])
               for i in range(P)]
    cb.cbh_batch_update(ctx, plan, lr, l2, lvs, True, side.cuda_stream)
    gr = cb.cbh_graph_capture_iteration(ctx, plan, lr, l2, lvs, side.cuda_stream)
    grs = [cb.cbh_graph_capture_iteration(ctx, pl, lr, l2, [lvs[i]], side.cuda_stream)
           for i, pl in enumerate(singles)]

    def one_by_one():
        for g in grs:
            cb.cbh_graph_launch(g, side.cuda_stream)
    with torch.cuda.stream(side):
        ms_b = timed(lambda: cb.cbh_graph_launch(gr, side.cuda_stream), side)
        ms_s = timed(one_by_one, side)
    cb.cbh_sync(ctx, side.cuda_stream)
    for g in [gr] + grs:
        cb.cbh_graph_destroy(g)
    for pl in [plan] + singles:
        cb.cbh_batch_destroy(pl)
    return ms_b, ms_s


def c2_batches(args, ctx, prec, side, timed):
    """The 1M-row RMSE problem as a 5-fold cross-validation batch (each fold
    trains on 4/5 of the rows, numeric borders chosen once on all rows) and
    as an 8-permutation ordered-boosting batch (8 models, each over its own
    permutation's ordered-statistic columns, sharing the numeric bins)."""
    import datagen
    from paper_1810_11363_amd.booster import GpuBooster
    t0 = time.perf_counter()
    base = datagen.make_c2(n=args.c2_rows, s=8)
    full = GpuBooster.from_problem(base, precision=prec, ctx=ctx).prepare()
    # the folds: row weights over one booster's rows (0 on each fold's held-out
    # rows), each fold with its own permutation's statistic columns; the
    # numeric bins are binned once for all folds
    cvq, w = datagen.cv_fold_weights(datagen.make_c2(n=args.c2_rows, s=1), 5)
    cvb = GpuBooster.from_problem(cvq, precision=prec, ctx=ctx).prepare()
    fold_states = [cvb.model_state(j, weight=w[j]) for j in range(5)]
    states = [full.model_state(r) for r in range(8)]
    print(f"# cross-validation and permutation batches prepared in "
          f"{time.perf_counter() - t0:.1f}s", file=sys.stderr, flush=True)
    res = []
    for name, probs, hists, lvs in [
            ("cv", [m.prob for m in fold_states], [m.hist for m in fold_states],
             [m.leaf_values for m in fold_states]),
            ("perm", [m.prob for m in states], [m.hist for m in states],
             [m.leaf_values for m in states])]:
        ms_b, ms_s = batch_vs_one_by_one(ctx, probs, hists, lvs, prec, full.lr, full.l2, side,
                                         timed)
        rows = sum(int(p.n) for p in probs)
        train_rows = int((w > 0).sum()) if name == "cv" else rows
        res.append({
            "problems": len(probs), "rows": rows, "training_rows": train_rows,
            "features": full.F, "depth": full.depth,
            "ms_per_iteration": round(ms_b, 4), "ms_per_tree": round(ms_b / len(probs), 5),
            "g_row_features_per_s": round(rows * full.F * full.depth / (ms_b / 1e3) / 1e9, 3),
            "one_plan_per_problem_ms_per_iteration": round(ms_s, 4),
            "batched_vs_one_plan_per_problem": round(ms_s / ms_b, 3)})
        print(f"# {name} batch: {ms_b:.3f} ms/iteration, one plan per problem {ms_s:.3f}",
              file=sys.stderr, flush=True)
    res[0]["workload"] = (f"5-fold cross-validation of the {args.c2_rows}-row RMSE problem "
                          f"(110 features x 128 bins, depth 6), one model per fold: row "
                          f"weights (0 on the fold's held-out rows) over the shared rows")
    res[1]["workload"] = (f"8 ordered-boosting permutations of the {args.c2_rows}-row RMSE "
                          f"problem, one model per permutation")
    for b in (cvb, full):
        b.close()
    return res[0], res[1]


def run_batch(args):
    """The batching workload: P independent RMSE problems (row counts
    log-uniform in [5e3, 2e6]) trained together, one boosting iteration of
    all of them replayed from the graph cbh_graph_capture_iteration returns;
    beside it the same problems grown one after another, each tree replayed
    from its own graph."""
    import numpy as np
    import torch

    import datagen
    from paper_1810_11363_amd import cbhip as cb
    from paper_1810_11363_amd.booster import GpuBooster
    t_gen = time.perf_counter()
    probs = datagen.make_c4(P=args.batch_p, scale=args.batch_scale)
    t_gen = time.perf_counter() - t_gen
    print(f"# generated {len(probs)} problems in {t_gen:.1f}s", file=sys.stderr, flush=True)
    prec = PRECISIONS[args.precision]
    ctx = cb.cbh_create(0)
    bsts = [GpuBooster.from_problem(p, precision=prec, ctx=ctx).prepare() for p in probs]
    P, depth, F = len(bsts), bsts[0].depth, bsts[0].F
    rows = sum(b.n for b in bsts)
    rf_per_iter = rows * F * depth
    lr, l2 = bsts[0].lr, bsts[0].l2
    dev = bsts[0].device
    side = torch.cuda.Stream(dev)
    # sequential: eager trees first (the shared workspace reaches its largest
    # size before any graph is captured), then one graph per problem
    for b in bsts:
        b.init_gradients()
        b.fit_tree(0)
    torch.cuda.synchronize()
    graphs = [b.capture_tree(1) for b in bsts]

    def seq_iter():
        for g in graphs:
            cb.cbh_graph_launch(g, side)
    # batched
    best = torch.zeros((P, depth, 4), dtype=torch.int32, device=dev)
    plan = cb.cbh_batch_create(ctx, [b.probs[0] for b in bsts], prec, [b.hist for b in bsts],
                               best)
    lvs = [b.leaf_values for b in bsts]
    cb.cbh_batch_update(ctx, plan, lr, l2, lvs, True, side.cuda_stream)
    gr = cb.cbh_graph_capture_iteration(ctx, plan, lr, l2, lvs, side.cuda_stream)
    # the same plan with every level as one persistent launch, for comparison
    cb.cbh_batch_set_fused(plan, True)
    gr_fused = cb.cbh_graph_capture_iteration(ctx, plan, lr, l2, lvs, side.cuda_stream)
    cb.cbh_batch_set_fused(plan, False)

    def batch_iter():
        cb.cbh_graph_launch(gr, side.cuda_stream)

    def batch_iter_fused():
        cb.cbh_graph_launch(gr_fused, side.cuda_stream)

    def timed(fn, stream_obj):
        t_end = time.perf_counter() + args.warmup_s
        while time.perf_counter() < t_end:
            fn()
            torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        with torch.cuda.stream(stream_obj):
            e0.record(stream_obj)
            for _ in range(args.steps):
                fn()
            e1.record(stream_obj)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / args.steps

    with torch.cuda.stream(side):
        ms_batch = timed(batch_iter, side)
        ms_fused = timed(batch_iter_fused, side)
        ms_seq = timed(seq_iter, side)
    cb.cbh_sync(ctx, side.cuda_stream)
    out = {
        "metric": "batched boosting iteration (all problems) and per-tree time",
        "value": round(rf_per_iter / (ms_batch / 1e3) / 1e9, 3),
        "unit": "G row-features/s",
        "n_gpus": 1, "steps": args.steps, "warmup_s": args.warmup_s,
        "ms_per_step": round(ms_batch, 4),
        "ms_per_tree": round(ms_batch / P, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": DTYPES[args.precision], "data": "synthetic",
        "config": {"workload": f"{P} independent RMSE problems, {rows} rows in all "
                               f"(log-uniform 5e3..2e6 x {args.batch_scale}), 50 numeric features "
                               f"at 64 bins + 4 categorical (C=1000) -> {F} columns, depth {depth}",
                   "precision": args.precision, "problems": P, "rows": rows},
        "sequential_ms_per_iteration": round(ms_seq, 4),
        "batched_vs_sequential": round(ms_seq / ms_batch, 3),
        "level_launches": "separate launches per level (cbh_batch_level, the default)",
        "fused_launch_ms_per_iteration": round(ms_fused, 4),
        "fused_vs_separate_launches": round(ms_batch / ms_fused, 3),
    }
    cb.cbh_graph_destroy(gr)
    cb.cbh_graph_destroy(gr_fused)
    for g in graphs:
        cb.cbh_graph_destroy(g)
    cb.cbh_batch_destroy(plan)
    for b in bsts:
        b.close()
    del bsts
    if args.c2_rows > 0:
        cv, perm = c2_batches(args, ctx, prec, side, timed)
        out["cv_batch"], out["perm_batch"] = cv, perm
    cb.cbh_destroy(ctx)
    if not args.no_cpu:
        # the oracle on the smallest problems whose rows add up to ~1e6
        import oracle
        from oracle import boost
        order = np.argsort([p.n for p in probs])
        picked, tot = [], 0
        for i in order:
            if tot + probs[i].n > args.cpu_rows and picked:
                break
            picked.append(i)
            tot += probs[i].n
        ready = []
        for i in picked:
            p = probs[i]
            prep = boost.prepare(p)
            bins, nb = prep.tree_features(0)
            ready.append((p, bins, nb, max(int(prep.nb_num.max()), prep.nb_ts)))
        t0 = time.perf_counter()
        rf = 0
        for p, bins, nb, B in ready:
            approx = np.zeros((p.K, p.n))
            boost.fit_tree(bins, nb, approx, p.label, p.loss, p.K, p.depth, p.lr, p.l2, B)
            rf += p.n * bins.shape[0] * p.depth
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": round(rf / dt / 1e9, 6), "unit": "G row-features/s",
                               "cores": oracle.num_threads(), "kind": "oracle",
                               "sample": f"one tree of each of the {len(picked)} smallest "
                                         f"problems ({tot} rows); borders, bins and statistics "
                                         f"before it are not timed"}
    print(json.dumps(out), flush=True)


def run_apply(args):
    """Model apply, the scorer of Sec. 4 (cbh_apply_model), on a stand-in for
    the paper's scorer comparison: a test set of the shape it scores (10^5
    rows x 2000 features, here at 128 bins, one plain column per feature) and
    a model of 8000 oblivious trees of depth 6 with seeded random splits and
    leaf values. One step applies the whole model to every row."""
    import numpy as np
    import torch

    import oracle
    from paper_1810_11363_amd import cbhip as cb
    n, F, B, T, d = args.n, 2000, 128, 8000, 6
    dev = torch.device("cuda:0")
    stride = (n + 15) // 16 * 16
    gen = torch.Generator(device=dev)
    gen.manual_seed(11363)
    cols = torch.randint(0, B, (F, stride), dtype=torch.uint8, device=dev, generator=gen)
    table = torch.tensor([cols.data_ptr() + stride * f for f in range(F)], dtype=torch.int64,
                         device=dev)
    seg = None
    rng = np.random.default_rng(11364)
    feat = rng.integers(0, F, (T, d)).astype(np.int32)
    border = rng.integers(0, B - 1, (T, d)).astype(np.int32)
    values = rng.normal(size=(T, 1 << d, 1))
    lr = 0.1
    dfeat = torch.from_numpy(feat).to(dev)
    dborder = torch.from_numpy(border).to(dev)
    dvalues = torch.from_numpy(values).to(dev)
    approx = torch.zeros((1, n), dtype=torch.float64, device=dev)
    ctx = cb.cbh_create(0)

    def step():
        cb.cbh_apply_model(ctx, table, seg, n, F, 1, T, d, dfeat, dborder, dvalues, lr, approx)

    for _ in range(2):
        step()
    cb.cbh_sync(ctx)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record()
    for _ in range(args.steps):
        step()
    e1.record()
    cb.cbh_sync(ctx)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / args.steps
    sec = e0.elapsed_time(e1) / 1e3 / args.steps
    # parity on a row sample: one apply from zero, against the oracle
    approx.zero_()
    step()
    cb.cbh_sync(ctx)
    m = min(n, args.cpu_rows)
    sample = cols[:, :m].cpu().numpy()
    got = approx[0, :m].cpu().numpy()
    # the two steps of Sec. 4: binarize the model's (feature, border) pairs
    # once, then the leaves from the bits
    pairs = np.stack([feat.reshape(-1), border.reshape(-1)], 1).astype(np.int64)
    uniq, inv = np.unique(pairs, axis=0, return_inverse=True)
    nb = int(uniq.shape[0])
    dbf = torch.from_numpy(uniq[:, 0].astype(np.int32)).to(dev)
    dbk = torch.from_numpy(uniq[:, 1].astype(np.int32)).to(dev)
    dsb = torch.from_numpy(inv.reshape(T, d).astype(np.int32)).to(dev)
    bits = torch.empty((nb, (n + 31) // 32), dtype=torch.int32, device=dev)
    approx_b = torch.zeros((1, n), dtype=torch.float64, device=dev)

    def step_bin():
        cb.cbh_binarize(ctx, table, seg, n, F, nb, dbf, dbk, bits)
        cb.cbh_apply_model_binarized(ctx, bits, n, nb, 1, T, d, dsb, dvalues, lr, approx_b)

    for _ in range(2):
        step_bin()
    cb.cbh_sync(ctx)
    e2, e3, e4 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    torch.cuda.synchronize()
    e2.record()
    for _ in range(args.steps):
        cb.cbh_binarize(ctx, table, seg, n, F, nb, dbf, dbk, bits)
    e3.record()
    for _ in range(args.steps):
        step_bin()
    e4.record()
    cb.cbh_sync(ctx)
    torch.cuda.synchronize()
    sec_binarize = e2.elapsed_time(e3) / 1e3 / args.steps
    sec_bin = e3.elapsed_time(e4) / 1e3 / args.steps
    approx_b.zero_()
    step_bin()
    cb.cbh_sync(ctx)
    got_b = approx_b[0, :m].cpu().numpy()
    binarized = {"ms_per_step": round(sec_bin * 1e3, 4),
                 "binarize_ms": round(sec_binarize * 1e3, 4),
                 "binary_features": nb,
                 "value": round(n * T / sec_bin / 1e9, 3), "unit": "G row-trees/s",
                 "vs_bins": round(sec / sec_bin, 3)}
    t1 = time.perf_counter()
    want = oracle.apply_model(sample, feat, border, values, lr, np.zeros((1, m)))
    cpu_s = time.perf_counter() - t1
    cb.cbh_destroy(ctx)
    algo_bytes = n * F + 16 * n + feat.nbytes + border.nbytes + values.nbytes
    achieved = algo_bytes / sec / 1e9
    out = {
        "metric": "model apply throughput (rows x trees per second)",
        "value": round(n * T / sec / 1e9, 3),
        "unit": "G row-trees/s",
        "n_gpus": 1,
        "steps": args.steps,
        "ms_per_step": round(sec * 1e3, 4),
        "wall_ms_per_step": round(wall * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"model apply: {n} rows x {F} features at {B} bins (plain "
                               f"columns), {T} oblivious trees of depth {d}, K=1",
                   "rows": n, "features": F, "trees": T, "depth": d},
        "parity": {"rows_checked": m, "bit_exact": bool(np.array_equal(got, want[0])),
                   "binarized_bit_exact": bool(np.array_equal(got_b, want[0]))},
        "binarized": binarized,
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": 8000.0,
                     "unit": "GB/s", "frac": round(achieved / 8000.0, 4), "traffic": None,
                     "kernel": "cbh_apply_model (model_leaves_kernel + model_sum_kernel)",
                     "algorithmic_bytes_per_launch": algo_bytes,
                     "avg_launch_ms": round(sec * 1e3, 4)},
    }
    if not args.no_cpu:
        out["cpu_baseline"] = {"value": round(m * T / cpu_s / 1e9, 4), "unit": "G row-trees/s",
                               "cores": 1, "kind": "oracle",
                               "sample": f"{m} of {n} rows, the whole model; "
                                         f"oracle {cpu_s:.2f} s"}
    print(json.dumps(out), flush=True)


def run_combine(args):
    """Feature combinations (Sec. 2; perfect hashes by radix sort, Sec. 5): the
    dense ids of a pair of categorical features and the ordered statistics of
    the combination for one permutation. Columns of the shape of the large
    workload's categorical features: cardinalities 10^3 and 10^6, Zipf(1.05)
    frequencies. One step = cbh_combine_categories + cbh_compute_ordered_ts
    (one 0/1 target, no bins) + cbh_category_counts."""
    import numpy as np
    import torch

    import datagen
    import oracle
    from paper_1810_11363_amd import cbhip as cb
    n = args.n
    g = np.random.default_rng(1810)
    a = datagen.zipf_ids(g, n, 1000, 1.05).astype(np.int32)
    b = datagen.zipf_ids(g, n, 1_000_000, 1.05).astype(np.int32)
    y = (g.random(n) < 0.3).astype(np.int64)
    perm = g.permutation(n).astype(np.int32)
    dev = torch.device("cuda:0")
    da, db = torch.from_numpy(a).to(dev), torch.from_numpy(b).to(dev)
    dy, dp = torch.from_numpy(y).to(dev), torch.from_numpy(perm).to(dev)
    ids = torch.empty(n, dtype=torch.int32, device=dev)
    m = torch.empty(1, dtype=torch.int64, device=dev)
    num = torch.empty(n, dtype=torch.int64, device=dev)
    den = torch.empty(n, dtype=torch.int32, device=dev)
    ts = torch.empty(n, dtype=torch.float64, device=dev)
    cnt = torch.empty(n, dtype=torch.int32, device=dev)
    ctx = cb.cbh_create(0)

    def step():
        cb.cbh_combine_categories(ctx, da, db, n, ids, m)
        cb.cbh_compute_ordered_ts(ctx, ids, dp, n, dy, 1, 0, 1, 1.0, [0.3], None, 0,
                                  num_out=num, den_out=den, ts_out=ts)
        cb.cbh_category_counts(ctx, ids, n, cnt)

    for _ in range(2):
        step()
    cb.cbh_sync(ctx)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e2 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(args.steps):
        cb.cbh_combine_categories(ctx, da, db, n, ids, m)
    e1.record()
    for _ in range(args.steps):
        step()
    e2.record()
    cb.cbh_sync(ctx)
    torch.cuda.synchronize()
    comb = e0.elapsed_time(e1) / 1e3 / args.steps
    sec = e1.elapsed_time(e2) / 1e3 / args.steps
    got_ids = ids.cpu().numpy()
    got_cnt = cnt.cpu().numpy()
    got_ts = ts.cpu().numpy()
    n_distinct = int(m.item())
    cb.cbh_destroy(ctx)
    rid, rm = oracle.combine_categories(a, b)
    parity_ids = bool(rm == n_distinct and np.array_equal(got_ids, rid))
    parity_cnt = bool(np.array_equal(got_cnt, oracle.category_counts(rid)))
    # the oracle on a row sample: combination ids and the statistics
    k = min(n, args.cpu_rows)
    sp = np.random.default_rng(1811).permutation(k).astype(np.int32)
    t0 = time.perf_counter()
    sid, _ = oracle.combine_categories(a[:k], b[:k])
    _, _, st, _ = oracle.ordered_ts(sid, sp, y[:k], 0, 1.0, 0.3)
    cpu_s = time.perf_counter() - t0
    algo_bytes = 8 * n + 4 * n                     # the two columns in, the ids out
    out = {
        "metric": "feature combination: pair ids + ordered statistics + counts (rows/s)",
        "value": round(n / sec / 1e6, 2),
        "unit": "M rows/s",
        "n_gpus": 1,
        "steps": args.steps,
        "ms_per_step": round(sec * 1e3, 4),
        "combine_ms": round(comb * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32/int64/f64",
        "data": "synthetic",
        "config": {"workload": f"pair of categorical columns, {n} rows, cardinalities 1e3 and "
                               f"1e6, Zipf(1.05); {n_distinct} distinct pairs; one permutation, "
                               f"one 0/1 target",
                   "rows": n, "distinct_pairs": n_distinct},
        "parity": {"ids_bit_exact": parity_ids, "counts_bit_exact": parity_cnt},
        "roofline": {"bound": "hbm", "achieved": round(algo_bytes / comb / 1e9, 1),
                     "peak": 8000.0, "unit": "GB/s",
                     "frac": round(algo_bytes / comb / 1e9 / 8000.0, 4), "traffic": None,
                     "kernel": "cbh_combine_categories (8 radix passes + scan)",
                     "algorithmic_bytes_per_launch": algo_bytes,
                     "avg_launch_ms": round(comb * 1e3, 4)},
    }
    if not args.no_cpu:
        out["cpu_baseline"] = {"value": round(k / cpu_s / 1e6, 3), "unit": "M rows/s",
                               "cores": 1, "kind": "oracle",
                               "sample": f"first {k} of {n} rows; oracle {cpu_s:.2f} s"}
    print(json.dumps(out), flush=True)


def run_combo_trees(args):
    """Trees with greedy feature combinations and three priors per statistic
    (Sec. 2) on the 1M-row RMSE workload: after every split, the split's
    value per row is crossed with each of the 10 categorical features (perfect
    hash, ordered statistics for every prior) and the combinations join the
    candidates of the levels below; every level builds its histograms over
    all candidates directly. Beside it, plain trees on the same columns (the
    three priors, no combinations), grown eagerly as well."""
    import numpy as np
    import torch

    import datagen
    from paper_1810_11363_amd import cbhip as cb
    from paper_1810_11363_amd.booster import GpuBooster

    p = datagen.make_c2(n=args.n)
    p.extra_priors = [p.ts_lo, p.ts_hi]
    prec = PRECISIONS[args.precision]
    out = {"metric": "sec/tree with greedy feature combinations (Sec. 2)", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "higher_is_better": False,
           "scaling": "weak", "vs_baseline": None, "dtype": DTYPES[args.precision],
           "data": "synthetic",
           "config": {"workload": f"1M-row RMSE: n={p.n}, 100 numeric features at 128 bins + "
                                  f"10 categorical with 3 priors each (mean, min and max of "
                                  f"the target) -> 130 columns per tree before combinations, "
                                  f"4 permutations, depth {p.depth}",
                      "rows": p.n, "depth": p.depth, "precision": args.precision}}
    res = {}
    for mode in ("combinations", "plain"):
        bst = GpuBooster.from_problem(p, precision=prec, combinations=mode == "combinations",
                                      partition=False).prepare()
        bst.init_gradients()
        for t in range(args.warmup):
            bst.fit_tree(t)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(bst.stream)
        for t in range(args.warmup, args.warmup + args.steps):
            bst.fit_tree(t)
        e1.record(bst.stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        # the same trees replayed from graphs (one per permutation)
        bst.capture_trees()
        for t in range(args.warmup):
            bst.replay_tree(t)
        torch.cuda.synchronize()
        e0.record(bst.stream)
        for t in range(args.warmup, args.warmup + args.steps):
            bst.replay_tree(t)
        e1.record(bst.stream)
        torch.cuda.synchronize()
        ms_graph = e0.elapsed_time(e1) / args.steps
        bst.drop_graphs()
        # the faster of the two paths is the tree time (a long chain of short
        # kernels can run faster from the stream than from a graph)
        r = {"ms_per_tree_eager": round(ms, 3), "ms_per_tree_graph": round(ms_graph, 3),
             "ms_per_tree": round(min(ms, ms_graph), 3),
             "path": "eager" if ms < ms_graph else "graph",
             "features_per_tree_level0": bst.F}
        ms = min(ms, ms_graph)
        if mode == "combinations":
            # where a tree's time goes: per level, histograms + score, then
            # the leaf bit and the next level's combination columns
            ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)]
                  for _ in range(bst.depth)]
            t = args.warmup + args.steps
            chosen = 0
            for lvl in range(bst.depth):
                ev[lvl][0].record(bst.stream)
                bst.combo_level(t, lvl)
                ev[lvl][1].record(bst.stream)
                bst.combo_advance(t, lvl)
                ev[lvl][2].record(bst.stream)
            torch.cuda.synchronize()
            r["hist_score_ms_per_level"] = [round(e[0].elapsed_time(e[1]), 3) for e in ev]
            r["combination_columns_ms_per_level"] = [round(e[1].elapsed_time(e[2]), 3)
                                                     for e in ev]
            r["candidates_per_level"] = [bst.F + lvl * bst.F_cat * bst.T * bst.Q
                                         for lvl in range(bst.depth)]
            b = bst.best.cpu().numpy()
            chosen = int((b[:, 0] >= bst.F).sum())
            r["combination_splits_in_last_tree"] = chosen
        res[mode] = r
        print(f"# {mode}: {ms:.3f} ms/tree", file=sys.stderr, flush=True)
        bst.close()
    out["modes"] = res
    out["value"] = res["combinations"]["ms_per_tree"] / 1e3
    out["unit"] = "s/tree"
    out["ms_per_step"] = res["combinations"]["ms_per_tree"]
    out["combinations_vs_plain"] = round(res["combinations"]["ms_per_tree"]
                                         / res["plain"]["ms_per_tree"], 2)
    if not args.no_cpu:
        from oracle import boost
        k = args.cpu_rows
        q = datagen.make_c2(n=k)
        q.extra_priors = [q.ts_lo, q.ts_hi]
        prep = boost.prepare(q)
        approx = np.zeros((1, k))
        B = max(int(prep.nb_num.max()), prep.nb_ts)
        t0 = time.perf_counter()
        boost.fit_tree_combinations(prep, q, 0, approx, B)
        cpu_s = time.perf_counter() - t0
        import oracle as orc
        out["cpu_baseline"] = {"value": round(cpu_s * p.n / k, 3), "unit": "s/tree (scaled)",
                               "cores": orc.num_threads(), "kind": "oracle",
                               "sample": f"one combination tree on a {k}-row draw of the same "
                                         f"workload, {cpu_s:.2f} s, scaled by rows"}
    print(json.dumps(out), flush=True)


def copy_bandwidth(mib: int = 1024, reps: int = 5):
    """GB/s (bytes read + written) of a plain device-to-device copy of `mib`
    MiB: the bandwidth a streaming kernel reaches on this GPU."""
    import torch
    x = torch.ones(mib << 18, dtype=torch.float32, device="cuda:0")
    y = torch.empty_like(x)
    y.copy_(x)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        y.copy_(x)
    e1.record()
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) / 1e3 / reps
    del x, y
    return round(2 * (mib << 20) / sec / 1e9, 1)


def cpu_single_thread():
    """The oracle at one thread: all trees of the 10^4-row Logloss workload,
    and 3 trees of the 1M-row RMSE workload (full rows)."""
    import numpy as np

    import datagen
    import oracle
    from oracle import boost
    out = {}
    prev = oracle.num_threads()
    oracle.set_threads(1)
    try:
        for name, p, trees in (("c1_10k_logloss", datagen.make_c1(), None),
                               ("c2_1m_rmse", datagen.make_c2(), 3)):
            prep = boost.prepare(p)
            B = max(int(prep.nb_num.max()), prep.nb_ts)
            approx = np.zeros((p.K, p.n))
            T = p.iterations if trees is None else trees
            t0 = time.perf_counter()
            for t in range(T):
                bins, nb = prep.tree_features(t)
                boost.fit_tree(bins, nb, approx, p.label, p.loss, p.K, p.depth, p.lr, p.l2, B)
            dt = (time.perf_counter() - t0) / T
            F = prep.tree_features(0)[0].shape[0]
            out[name] = {"sec_per_tree": round(dt, 4), "trees": T, "rows": p.n,
                         "G_row_features_per_s": round(p.n * F * p.depth / dt / 1e9, 5),
                         "cores": 1}
    finally:
        oracle.set_threads(prev)
    return out


def resolve(args, workload):
    """Arguments of one tree workload: the user's values where given, else the
    workload's defaults."""
    a = copy.copy(args)
    a.workload = workload
    wl = WORKLOADS[workload]
    for k in ("steps", "n", "cpu_rows", "cpu_trees"):
        if getattr(a, k) is None:
            setattr(a, k, wl[k])
    for k, v in RUN_DEFAULTS.items():
        if getattr(a, k) is None:
            setattr(a, k, wl.get(k, v))
    return a


def run_trees(args):
    """One tree workload (c2, c3, c5): every form timed, the oracle leg; the
    JSON object (not printed)."""
    import torch  # noqa: F401

    import datagen
    from paper_1810_11363_amd.booster import GpuBooster

    rates = measure_lds_rates()
    print(f"# LDS update rates (lane ops per clock per CU): {rates}", file=sys.stderr, flush=True)
    t_gen = time.perf_counter()
    if args.workload == "c5":
        def progress(done, total):
            if done % 8 == 0 or done == total:
                print(f"# generating: {done}/{total} row chunks", file=sys.stderr, flush=True)
        p = datagen.make_c5(n=args.n, progress=progress)
    else:
        p = {"c2": datagen.make_c2, "c3": datagen.make_c3}[args.workload](n=args.n)
    t_gen = time.perf_counter() - t_gen
    print(f"# generated {args.workload} in {t_gen:.1f}s", file=sys.stderr, flush=True)
    part = {"auto": None, "on": True, "off": False}[args.partition]
    bst = GpuBooster.from_problem(p, partition=part).prepare()
    print(f"# prepared: {bst.timings}", file=sys.stderr, flush=True)
    rmse = p.loss == datagen.RMSE
    forms = [args.precision] + [f for f in args.compare.split(",")
                                if f and f not in (args.precision, "none")]
    results = {}
    for f in forms:
        a = args
        if f != args.precision and args.compare_steps:
            # the comparison forms: fewer trees (the float32 compare-and-swap
            # forms take seconds per tree on this workload)
            a = copy.copy(args)
            a.steps, a.warmup, a.hist_trees = args.compare_steps, 1, 1
        results[f] = time_form(bst, f, a, rmse)
        results[f]["timed_trees"] = a.steps
    head = results[args.precision]
    n, F, depth = bst.n, bst.F, bst.depth
    out = {
        "metric": METRIC,
        "value": head["G_row_features_per_s"],
        "unit": "G row-features/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "sec_per_tree": head["sec_per_tree"],
        "hist_G_row_features_per_s": head["hist_G_row_features_per_s"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPES[args.precision],
        "data": "synthetic",
        "config": {"workload": describe(args.workload, p, bst),
                   "precision": args.precision, "features_per_tree": F, "bins": bst.B,
                   "rows": n, "classes": bst.K, "depth": depth},
        "roofline": dict(head["roofline"], copy_gbs=copy_bandwidth()),
        "forms": results,
        "vs_plain_fp32": (round(results["fp32"]["sec_per_tree"] / head["sec_per_tree"], 3)
                          if "fp32" in results else None),
        "preprocess_s": {k: round(v, 4) for k, v in bst.timings.items() if v is not None},
        "lds_rates_lane_ops_per_clk_per_cu": rates,
    }
    if args.workload == "c2":
        out["ordered"] = time_ordered(bst, args, rmse)
        out["ordered"]["vs_plain_tree"] = round(out["ordered"]["ms_per_tree"] /
                                                head["ms_per_step"], 3)
    bst.close()
    # the oracle leg: FP64 error of every form's sampled histograms, then the
    # oracle timed on a row sample of the same workload
    for f, r in results.items():
        snap = r.pop("_snapshot")
        if snap is not None:
            r["max_norm_err_vs_fp64"], q = oracle_error(snap)
            if q is not None:
                r["max_g_err_over_quant_bound"] = q
    if not args.no_cpu:
        print("# cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = dict(cpu_baseline(copy.copy(p), args.cpu_rows, args.cpu_trees),
                                   **cpu_info())
    del p
    return out


def ordered_update_bytes(n, K, s, rmse):
    """Algorithmic HBM bytes of one ordered tree's updates (Sec. 3): the kept
    model once, and per permutation the gather of leaf and label into
    position order, the sums over every model's learning positions, the
    update of every kept entry and the next tree's gradients."""
    import oracle
    M = oracle.ordered_models(n)
    S = int(oracle.ordered_offsets(n)[-1])
    T = (1 << (M - 1)) - 1 if M >= 1 else 0        # learning entries of all models
    gb = 4 * K * (1 if rmse else 2)                # g (and h) written per row
    per_perm = 16 * n + T * (6 + 8 * K) + S * (2 + 16 * K) + n * (8 + gb)
    kept = n * (6 + 8 * K) + n * (2 + 16 * K)
    return kept + s * per_perm, per_perm, S, M


def time_ordered(bst, args, rmse):
    """Ordered boosting (Sec. 3) on the same problem and form: whole trees
    (levels on permutation t mod s's supporting gradients, then the kept
    model and every permutation's supporting models), and the updates alone.
    Eager launches (the tree is a few library calls), CUDA events on the
    booster's stream."""
    import torch
    from paper_1810_11363_amd import cbhip as cb
    torch.cuda.synchronize()
    bst.set_precision(PRECISIONS[args.precision], subtract=args.subtract)
    bst.drop_graphs()
    bst.set_ordered(True)
    bst.init_gradients()
    steps = max(4, min(args.steps, 20))
    for t in range(2):
        bst.fit_tree(t)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(bst.stream)
    for t in range(2, 2 + steps):
        bst.fit_tree(t)
    e1.record(bst.stream)
    torch.cuda.synchronize()
    ms_tree = e0.elapsed_time(e1) / steps
    pr = bst.probs[0]
    e0.record(bst.stream)
    for _ in range(steps):
        for q in range(bst.s):
            cb.cbh_ordered_update(bst.ctx, bst.ords[q], pr, bst.lr, bst.l2,
                                  bst.leaf_values if q == 0 else None, None, bst.stream)
    e1.record(bst.stream)
    torch.cuda.synchronize()
    cb.cbh_sync(bst.ctx)
    ms_upd = e0.elapsed_time(e1) / steps
    total, per_perm, S, M = ordered_update_bytes(bst.n, bst.K, bst.s, rmse)
    bst.set_ordered(False)
    bst.init_gradients()
    gbs = total / (ms_upd * 1e-3) / 1e9
    return {
        "what": "ordered boosting (supporting approximations of every permutation, "
                "cbh_fit_tree_ordered + cbh_ordered_update)",
        "permutations": bst.s, "models_per_permutation": M, "support_doubles_per_class": S,
        "timed_trees": steps, "ms_per_tree": round(ms_tree, 4),
        "update_ms_per_tree": round(ms_upd, 4),
        "update_algorithmic_bytes_per_tree": total,
        "update_roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": 8000.0,
                            "unit": "GB/s", "frac": round(gbs / 8000.0, 4),
                            "note": "update kernels only, eager launches, event-timed "
                                    "(launch gaps included)"},
    }


def run_packed(args):
    """Packed bins (Sec. 5) on the dense numeric workload: the same data
    quantized to 15 bins read as bytes and as 4-bit packed bins, and to 2 bins
    (binary) as bytes and as 1-bit packed bins; the headline form and int16
    on each layout, subtraction on, rows in their original order."""
    import torch  # noqa: F401

    import datagen
    from paper_1810_11363_amd.booster import GpuBooster

    measure_lds_rates()
    p = datagen.make_c3(n=args.n)
    print(f"# generated {p.name}: n={p.label.size}", file=sys.stderr, flush=True)
    forms = [args.precision] + (["int16"] if args.precision != "int16" else [])
    out = {"metric": "sec/tree on packed and byte bins", "n_gpus": 1, "data": "synthetic",
           "config": {"workload": f"10M-row Logloss, {p.x_num.shape[0]} uniform numeric "
                                  f"features quantized to 15 and to 2 bins, depth {p.depth}",
                      "rows": int(p.label.size)},
           "layouts": {}}
    a = copy.copy(args)
    a.no_cpu = True
    for nb, bits in ((15, 4), (2, 1)):
        p.num_bins = nb
        bst = GpuBooster.from_problem(p, partition=False).prepare()
        for b in (8, bits):
            bst.set_bin_bits(b)
            for f in forms:
                r = time_form(bst, f, a, False)
                r.pop("_snapshot", None)
                key = f"{nb}_bins_{'bytes' if b == 8 else f'{b}_bit'}_{f}"
                out["layouts"][key] = {k: r[k] for k in (
                    "sec_per_tree", "hist_ms_per_level", "hist_G_row_features_per_s",
                    "rows_accumulated_per_level", "roofline")}
                print(f"# {key}: {r['sec_per_tree'] * 1e3:.3f} ms/tree", file=sys.stderr,
                      flush=True)
        bst.close()
    L = out["layouts"]
    for nb, bits in ((15, 4), (2, 1)):
        for f in forms:
            k8, kp = f"{nb}_bins_bytes_{f}", f"{nb}_bins_{bits}_bit_{f}"
            L[kp]["speedup_vs_bytes"] = round(L[k8]["sec_per_tree"] / L[kp]["sec_per_tree"], 3)
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", choices=["headline"] + list(WORKLOADS), default="headline")
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=None,
                    help="trees grown before the graphs are captured")
    ap.add_argument("--warmup-s", type=float, default=None,
                    help="seconds of replayed trees before the timed region")
    ap.add_argument("--precision", choices=list(PRECISIONS), default="f64",
                    help="headline histogram form")
    ap.add_argument("--compare", default=None,
                    help="other forms timed in the same run ('' for none)")
    ap.add_argument("--compare-steps", type=int, default=None,
                    help="timed trees of the comparison forms (default: the workload's)")
    ap.add_argument("--n", type=int, default=None)
    ap.add_argument("--batch-p", type=int, default=64, help="problems of the batching workload")
    ap.add_argument("--batch-scale", type=float, default=1.0,
                    help="row-count scale of the batching workload")
    ap.add_argument("--c2-rows", type=int, default=1_000_000,
                    help="rows of the cross-validation and permutation batches of the "
                         "batching workload (0: leave them out)")
    ap.add_argument("--cpu-rows", type=int, default=None)
    ap.add_argument("--cpu-trees", type=int, default=None)
    ap.add_argument("--no-graph", action="store_true",
                    help="launch every call from Python instead of replaying captured trees")
    ap.add_argument("--hist-trees", type=int, default=None,
                    help="trees replayed from graphs with event nodes around every build")
    ap.add_argument("--partition", choices=["auto", "on", "off"], default="auto",
                    help="keep rows in leaf order during a tree (auto: for K > 1, and for depth >= 8 "
                         "in the float forms)")
    ap.add_argument("--subtract", choices=["on", "off", "auto"], default="on",
                    help="histogram subtraction at levels >= 1 for every form (auto: the "
                         "form's default, off for plain float32)")
    ap.add_argument("--no-cpu", action="store_true",
                    help="skip the oracle leg (CPU timing and error vs FP64)")
    ap.add_argument("--autotune", default=None,
                    help="'run' tunes launch plans before each timed region, 'off' keeps "
                         "the defaults, anything else is a cache file to load")
    ap.add_argument("--autotune-save", default=None, metavar="PATH",
                    help="with --autotune run: write the tuned plans of every form to PATH "
                         "(JSON, loadable with --autotune PATH)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a device-to-device copy of MIB MiB five times (reference "
                         "for hardware byte counters) and exit")
    args = ap.parse_args()
    args.subtract = {"on": True, "off": False, "auto": None}[args.subtract]
    if args.copy_calibration:
        import torch
        x = torch.ones(args.copy_calibration << 18, dtype=torch.float32, device="cuda:0")
        y = torch.empty_like(x)
        for _ in range(5):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each": x.numel() * 4, "copies": 5}))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU only; --gpus must be 1 "
                          "(sharding over several GPUs is not implemented)"}))
        sys.exit(2)
    if args.workload in ("c4", "apply", "combine", "packed", "combotrees"):
        a = resolve(args, args.workload)
        {"c4": run_batch, "apply": run_apply, "combine": run_combine,
         "packed": run_packed, "combotrees": run_combo_trees}[args.workload](a)
        return
    if args.workload != "headline":
        print(json.dumps(run_trees(resolve(args, args.workload))), flush=True)
        return
    # headline: the 50M-row MultiClass workload (the largest), then the
    # 1M-row RMSE workload with its own defaults, in one JSON line
    out = run_trees(resolve(args, "c5"))
    c2_args = copy.copy(args)
    for k in ("steps", "warmup", "n", "cpu_rows", "cpu_trees", "compare_steps", "hist_trees",
              "warmup_s", "autotune", "compare"):
        setattr(c2_args, k, None)
    c2 = run_trees(resolve(c2_args, "c2"))
    keep = ("value", "unit", "steps", "warmup", "ms_per_step", "sec_per_tree",
            "hist_G_row_features_per_s", "dtype", "config", "roofline", "forms", "vs_plain_fp32",
            "preprocess_s", "cpu_baseline", "ordered")
    out["c2"] = {k: c2[k] for k in keep if k in c2}
    if not args.no_cpu:
        print("# oracle at one thread ...", file=sys.stderr, flush=True)
        out["cpu_single_thread"] = cpu_single_thread()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
