"""Autotuner for the traversal launch shape: queries per lane (1 / 2 / 4) and
the schedule (plain grid, XCD-contiguous grid, persistent tile queue), and,
for batches too small to fill the GPU, the subtree split of the walks
(dps_set_split: 1 or 2 parts for the query, whose result then does not depend
on the order of the parts, 1 to 8 for the adjoint, cut level 2 to 4).

Times dps_query and the adjoint's stage 1 (after a query with gradients the
walk that forms dL/dx from them, dps_adjoint_accumulate_from_forward;
otherwise dps_adjoint_accumulate) for each shape on a slice of the caller's
own queries (HIP events on the current stream), keeps the fastest
per kernel, and applies it with dps_set_launch.  Results are cached in a JSON file
keyed by the workload shape, so later runs skip the sweep.
"""
from __future__ import annotations

import json
import os
import sys

from . import binding as B

PACKETS = (1, 2, 4)
# subtree-split candidates: tried for dipole trees when the sample holds at
# most SPLIT_MAX_QUERIES queries
SPLIT_MAX_QUERIES = 1 << 21
SPLIT_CUTS = (2, 3, 4)
SPLIT_ADJOINT_PARTS = (2, 4, 8)
# schedule name -> (flag bits for dps_query, flag bits for the adjoint)
SCHEDULES = {"grid": (0, 0), "xcd": (B.LAUNCH_XCD_QUERY, B.LAUNCH_XCD_ADJOINT),
             "persistent": (B.LAUNCH_PERSISTENT_QUERY, B.LAUNCH_PERSISTENT_ADJOINT)}
DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "dps_autotune.json")


def _key(tree, Q, beta, eps, grad):
    kind = getattr(tree, "kernel", "dipole")
    return f"M{tree.M}_C{tree.C}_{tree.storage}_{kind}_Q{Q}_b{beta:g}_e{eps:g}" + ("_fwdgrad" if grad else "_values")


def _time(fn, reps):
    import torch
    fn()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def tune(tree, x, df, beta, eps, sample=1 << 26, reps=2, cache=None, verbose=False, grad=True):
    """Picks and applies the fastest packet sizes; returns
    {"query": k, "adjoint": k, "ms": {...}}.  grad=False times the query
    without spatial gradients (the call the caller will make)."""
    import torch
    cache = cache if cache is not None else os.environ.get("DPS_AUTOTUNE_CACHE", DEFAULT_CACHE)
    key = _key(tree, x.shape[0], beta, eps, grad)
    table = {}
    if cache and os.path.exists(cache):
        try:
            table = json.load(open(cache))
        except (OSError, ValueError):
            table = {}
    if key in table:
        best = table[key]
        B.dps_set_launch(tree, best["query"], best["adjoint"], best["flags"])
        sq, sa, cut = best.get("split", (1, 1, -1))
        B.dps_set_split(tree, sq, sa, cut)
        return best
    if df.shape[0] != x.shape[0] or df.shape[1] != tree.C:
        raise ValueError("df must hold one row of tree.C cotangents per query of x")
    n = min(x.shape[0], sample)
    # a contiguous slice keeps the spatial coherence of the caller's layout
    start = (x.shape[0] - n) // 2 // 256 * 256
    xs = x[start:start + n].contiguous()
    dfs = df[start:start + n].contiguous()
    f = torch.empty((n, tree.C), device=x.device)
    g = torch.empty((n, tree.C, 3), device=x.device) if grad else None
    dx = torch.empty((n, 3), device=x.device)
    ms = {"query": {}, "adjoint": {}}
    B.dps_set_split(tree, 1, 1, -1)
    for mode, (qbit, abit) in SCHEDULES.items():
        for k in PACKETS:
            B.dps_set_launch(tree, k, k, qbit | abit)
            ms["query"][(k, mode)] = _time(
                lambda: B.dps_query(tree, xs, beta, eps, grad=grad, f_out=f, g_out=g), reps)
            B.dps_adjoint_zero(tree)
            if grad and getattr(tree, "kernel", "dipole") == "dipole":
                # the adjoint the caller will run after a query with gradients
                ms["adjoint"][(k, mode)] = _time(
                    lambda: B.dps_adjoint_accumulate_from_forward(tree, xs, beta, eps, dfs, g, dx_out=dx), reps)
            else:
                ms["adjoint"][(k, mode)] = _time(
                    lambda: B.dps_adjoint_accumulate(tree, xs, beta, eps, dfs, dx_out=dx), reps)
            if verbose:
                print(f"[autotune] k={k} {mode}: query {ms['query'][(k, mode)]:.3f} ms, "
                      f"adjoint {ms['adjoint'][(k, mode)]:.3f} ms", file=sys.stderr, flush=True)
    B.dps_adjoint_zero(tree)
    bq = min(ms["query"], key=ms["query"].get)
    ba = min(ms["adjoint"], key=ms["adjoint"].get)
    flags = SCHEDULES[bq[1]][0] | SCHEDULES[ba[1]][1]
    B.dps_set_launch(tree, bq[0], ba[0], flags)
    split = [1, 1, -1]
    if getattr(tree, "kernel", "dipole") == "dipole" and n <= SPLIT_MAX_QUERIES:
        split = _tune_split(tree, xs, dfs, f, g, dx, beta, eps, grad, reps, ms, ms["query"][bq], ms["adjoint"][ba],
                            verbose)
    B.dps_set_split(tree, *split)
    best = {"query": bq[0], "adjoint": ba[0], "query_schedule": bq[1], "adjoint_schedule": ba[1], "flags": flags,
            "split": split,
            "ms": {p: {(f"k{k[0]}_{k[1]}" if isinstance(k, tuple) else k): v for k, v in d.items()}
                   for p, d in ms.items()}}
    if cache:
        try:
            os.makedirs(os.path.dirname(cache), exist_ok=True)
            table[key] = best
            tmp = cache + ".tmp"
            json.dump(table, open(tmp, "w"), indent=1)
            os.replace(tmp, cache)
        except OSError:
            pass
    return best


def _tune_split(tree, xs, dfs, f, g, dx, beta, eps, grad, reps, ms, q_unsplit, a_unsplit, verbose):
    """Times the split walks at each cut level and returns the [query parts,
    adjoint parts, cut] with the smallest query + adjoint time (1 part: the
    unsplit launch already chosen)."""
    best, best_ms = [1, 1, -1], q_unsplit + a_unsplit
    for cut in SPLIT_CUTS:
        B.dps_set_split(tree, 2, 1, cut)
        tq = _time(lambda: B.dps_query(tree, xs, beta, eps, grad=grad, f_out=f, g_out=g), reps)
        ms["query"][f"split2_cut{cut}"] = tq
        times_a = {}
        for pa in SPLIT_ADJOINT_PARTS:
            B.dps_set_split(tree, 1, pa, cut)
            B.dps_adjoint_zero(tree)
            if grad:
                times_a[pa] = _time(
                    lambda: B.dps_adjoint_accumulate_from_forward(tree, xs, beta, eps, dfs, g, dx_out=dx), reps)
            else:  # a split adjoint forms no dL/dx in its walk
                times_a[pa] = _time(
                    lambda: B.dps_adjoint_accumulate(tree, xs, beta, eps, dfs, want_dx=False), reps)
            ms["adjoint"][f"split{pa}_cut{cut}"] = times_a[pa]
        pa = min(times_a, key=times_a.get)
        for pq, t_q in ((1, q_unsplit), (2, tq)):
            for p_a, t_a in ((1, a_unsplit), (pa, times_a[pa])):
                if (pq > 1 or p_a > 1) and t_q + t_a < best_ms:
                    best, best_ms = [pq, p_a, cut], t_q + t_a
        if verbose:
            print(f"[autotune] split cut={cut}: query(2) {tq:.3f} ms, adjoint " +
                  ", ".join(f"({p}) {t:.3f}" for p, t in times_a.items()) + " ms", file=sys.stderr, flush=True)
    B.dps_adjoint_zero(tree)
    return best
