#!/usr/bin/env python3
"""Throughput of Barnes-Hut dipole-sum queries, forward + adjoint, on one GPU.

Workload (sfm-1m): a 1,000,000-point SfM-like cloud (three noisy spheres / tori,
5% outliers, jittered normals, C = 4 attribute channels), queried at the
33,554,432 stratified samples of 512x512 camera rays x 128 samples, beta = 2,
eps = 0.01414, leaf size 16.  All inputs are seeded synthetic arrays resident
in HBM before timing starts.

One step = one training iteration of the hot path: moment refit from the
attributes (dps_set_attributes), primal query with gradients (dps_query), and
the two-stage adjoint (dps_adjoint_zero / _accumulate_from_forward /
_finalize) with dL/df ~ N(0,1): dL/dmu from the adjoint walk, dL/dx =
sum_c dL/df_c grad D_c from the query's gradients.  The adjoint that forms
dL/dx in its own walk (dps_adjoint_accumulate) is timed beside it and
reported in kernel_ms.  The adjoint that also takes cotangents of the gradients
(dps_adjoint_accumulate_grad, N(0,1)) is timed beside it and reported in
kernel_ms.  The tree itself is built once (points are fixed) and its
build time is reported separately.  value = Q / (time per step), FP32-stored
attributes and moments, eager launches.  The same step is also timed with
BF16 storage, eager and captured in one graph.

Grid workload (reported under "grid_512"): the geometry channel at the 512^3
points of the bounding cube (mesh extraction by marching cubes), positions
generated in the kernels.

Appearance workload (reported under "appearance_k32"): the same queries with
the geometry channel on a dipole tree and K = 32 appearance attributes on a
monopole-kernel tree (foreshortening dropped), forward and adjoint of both.

Ray front-end (reported under "ray_frontend"): one 512^2 view of the sfm-1m
cloud with unit geometry attributes: a 1024-sample march for each ray's first
crossing of the 1/2 level, 24/48/8 samples placed around it (80 uniform
without one), and the query of the placed samples.

Batched workload (sfm-8m, reported under "batched"): 8,388,608 points, 8 views
of 256^2 .. 1024^2 rays x 128 samples (438,829,056 primary samples), one shadow
ray of 64 samples and one hit-point query (values and gradients, for the
albedo and normal of the direct shadow term) per primary hit, BF16 storage,
persistent autotuned launches, the whole forward + backward of the render
proxy in one graph.

    python bench.py [--steps K] [--warmup W] [--storage fp32|bf16|both] [--no-batched]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "dipole-sum queries/sec fwd+adjoint at 1M pts, beta=2, FP32 vs BF16-stored"
BETA = 2.0
EPS = math.sqrt(2.0) * 0.01
LEAF = 16
RES = 512
SAMPLES = 128

# Algorithmic FP32 operations per unit of work (FMA = 2, add / mul /
# transcendental = 1), counted from the formulas the kernels evaluate:
#   far test:          d = c - x (3), squares (3), sums (2), beta^2 r^2 (1), compare (1)
#   far source, fwd:   d (3), rsqrt + r^-3 + kappa + lambda (6), per channel:
#                      D.d (5), f += kappa s (2), lambda s (1), g += ... (3 x 4)
#   near point, fwd:   d (3), r^2 (5), radial (6), An.d (5), kappa s, lambda s (2),
#                      G = lambda s d - kappa An (9), per channel: f (2), g (6)
#   far source, adj:   d (3), radial (6), E = sum w D (6C), E.d (5), dx (13),
#                      per channel: w kappa d (4) + wavefront sum (3)
#   near point, adj:   d (3), r^2 (5), radial (6), An.d (5), w.mu (2C), dx (16),
#                      per channel: w kappa s (2) + wavefront sum (1)
def flops_fwd(C):
    return {"test": 10, "far": 9 + 20 * C, "near": 30 + 8 * C}


def flops_adj(C):
    return {"test": 10, "far": 27 + 13 * C, "near": 35 + 5 * C}


# the adjoint walk whose dL/dx comes from the forward's gradients:
#   far source:  d (3), rsqrt + r^-3 + kappa (4), kappa d (3), per channel
#                w kappa d (6) + wavefront sum (3)
#   near point:  d (3), r^2 (5), rsqrt + kappa (4), An.d (5), kappa s (1),
#                per channel w kappa s (2) + wavefront sum (1)
#   per query:   dL/dx = sum_c w_c grad_c (6 C)
def flops_adj_fwdgrad(C):
    return {"test": 10, "far": 10 + 9 * C, "near": 18 + 3 * C, "query": 6 * C}


# monopole kernel (appearance channels, foreshortening dropped), same
# conventions:
#   far source, fwd:   d (3), radial (6), m = kappa (r^2 rsqrt) (2), per channel f += Q m (2)
#   near point, fwd:   d (3), r^2 (5), radial (6), m (2), A m (1), per channel f += mu A m (2)
#   far source, adj:   d (3), radial (6), m (2), gv = (lambda r^2 - kappa) rsqrt (2),
#                      per channel w Q (2), w m (2), wavefront sum (1); gv sum (1), dx (6)
#   near point, adj:   d (3), r^2 (5), radial (6), m (2), gv (2), A m (1), per channel as
#                      above (5); A gv sum (2), dx (6)
def flops_mono_fwd(C):
    return {"test": 10, "far": 11 + 2 * C, "near": 17 + 2 * C}


def flops_mono_adj(C):
    return {"test": 10, "far": 20 + 5 * C, "near": 27 + 5 * C}


# values-only dipole query (the ray march, one channel):
#   far source:  d (3), radial (6), per channel D.d (5), f += kappa s (2)
#   near point:  d (3), r^2 (5), radial (6), An.d (5), kappa s (1), per channel f (2)
def flops_values(C):
    return {"test": 10, "far": 9 + 7 * C, "near": 20 + 2 * C}


MI355X_FP32_VECTOR_TFLOPS = 157.3   # published peak (packed FP32)
MI355X_FP32_VECTOR_NONPACKED_TFLOPS = 78.6   # 256 CU x 4 SIMD x 16 lanes x 2 (FMA) x 2.4 GHz
MI355X_HBM_TBS = 8.0

# sources holding the device code of the point-query traversal kernels (the
# kernels take raw pointers, so the host-side tree header is not among them);
# the HBM byte counters committed under profiles/ are used only while these
# are unchanged
KERNEL_SOURCES = ("paper_2405_16788_amd/csrc/dps_traverse.hip", "paper_2405_16788_amd/csrc/dps_trav_common.h",
                  "paper_2405_16788_amd/csrc/dps_internal.h", "paper_2405_16788_amd/csrc/dps_walk.h")
COUNTER_SUMMARY = "profiles/sfm1m_fp32_hbm_counters.md"


def kernel_source_hash():
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def committed_traffic(kernel, k, persistent, storage):
    """HBM bytes per launch of ``kernel`` (queries per lane k, persistent or
    not) from the committed counter summary (FETCH_SIZE + WRITE_SIZE,
    copy-calibrated), or (None, reason)."""
    path = os.path.join(ROOT, COUNTER_SUMMARY)
    try:
        text = open(path).read()
    except OSError:
        return None, "no committed counter summary"
    m = re.search(r"```json\n(.*?)\n```", text, re.S)
    if not m:
        return None, "counter summary has no data block"
    d = json.loads(m.group(1))
    if d.get("source_sha256") != kernel_source_hash():
        return None, "kernel sources changed since the counters were taken"
    e = d.get("kernels", {}).get(kernel)
    if not e:
        return None, f"no counters for {kernel}"
    if d.get("storage") != storage or e.get("k") != k or e.get("persistent") != persistent:
        return None, (f"counters taken at {d.get('storage')} k={e.get('k')} persistent={e.get('persistent')}, "
                      f"timed run used {storage} k={k} persistent={persistent}")
    return e["read_bytes"] + e["write_bytes"], COUNTER_SUMMARY


# algorithmic bytes per query (fp32 storage s = 4): 32 B node record per
# visit, 12 C s per far-field moment, (32 + C s) per near point, plus I/O;
# the adjoint adds the scatter read-modify-write of 2 x 4 x 3C per far node
# and 2 x 4 x C per near point (before any aggregation)
def bytes_fwd(C, s=4):
    return {"visit": 32, "far": 12 * C * s, "near": 32 + C * s, "io": 12 + 16 * C}


def bytes_adj(C, s=4):
    return {"visit": 32, "far": 12 * C * s + 24 * C, "near": 32 + C * s + 8 * C, "io": 12 + 4 * C + 12}


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--storage", choices=["fp32", "bf16", "both"], default="both")
    ap.add_argument("--res", type=int, default=RES, help="image side (rays = res^2)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="target CPU time of the oracle sample")
    ap.add_argument("--packet", type=str, default="auto",
                    help="launch shape 'query_k,adjoint_k[,flags]' (e.g. 2,4,3) or 'auto' (autotuned)")
    ap.add_argument("--copy-reference", action="store_true",
                    help="only run a 1 GiB device fill + copy (calibrates HBM byte counters)")
    ap.add_argument("--no-graph", action="store_true", help="skip the graph-captured BF16 variant")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched 8M-point workload")
    ap.add_argument("--batched-only", action="store_true", help="only run the batched workload")
    ap.add_argument("--batched-steps", type=int, default=3)
    ap.add_argument("--no-appearance", action="store_true", help="skip the geometry + 32 appearance channel step")
    ap.add_argument("--no-frontend", action="store_true", help="skip the ray front-end (march + resample + query)")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_inputs(res):
    import numpy as np
    import workloads
    t0 = time.time()
    p, n, A, attrs = workloads.sfm_cloud(workloads.SFM_1M_SURFACE, workloads.SFM_1M_OUTLIERS, 10)
    eye = workloads.sfm_camera(11)
    x = workloads.ray_samples(eye, res, res, SAMPLES, 12, order="tile")
    df = workloads.cotangents(x.shape[0], attrs.shape[1], 17)
    log(f"[bench] inputs generated in {time.time() - t0:.1f}s: M={p.shape[0]} Q={x.shape[0]}")
    return p, n, A, attrs, x, df, np


def time_storage(P, dev_in, storage, steps, warmup, packet, graph=False):
    import torch
    p, n, A, attrs, x, df = dev_in
    Q, C = x.shape[0], attrs.shape[1]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tree = P.dps_build(p, n, A, attrs, leaf_size=LEAF, storage=storage)
    torch.cuda.synchronize()
    build_ms = (time.perf_counter() - t0) * 1e3
    if packet == "auto":
        from paper_2405_16788_amd import autotune
        tuned = autotune.tune(tree, x, df, BETA, EPS, cache="", verbose=True)
    else:
        vals = [int(v) for v in packet.split(",")]
        kq, ka = vals[0], vals[1]
        flags = vals[2] if len(vals) > 2 else -1
        P.dps_set_launch(tree, kq, ka, flags)
        tuned = {"query": kq, "adjoint": ka, "flags": P.dps_get_launch(tree)["flags"]}
    f = torch.empty((Q, C), device="cuda")
    g = torch.empty((Q, C, 3), device="cuda")
    dx = torch.empty((Q, 3), device="cuda")
    dattrs = torch.empty((tree.M, C), device="cuda")
    names = ["refit", "query", "adjoint_accumulate", "adjoint_finalize"]
    ev = {k: [] for k in names}

    def step(record):
        e = [torch.cuda.Event(enable_timing=True) for _ in range(5)] if record else None
        if record: e[0].record()
        P.dps_set_attributes(tree, attrs)
        if record: e[1].record()
        P.dps_query(tree, x, BETA, EPS, f_out=f, g_out=g)
        if record: e[2].record()
        P.dps_adjoint_zero(tree)
        # dL/dx from the gradients the query just returned; the walk adds the
        # node and point increments
        P.dps_adjoint_accumulate_from_forward(tree, x, BETA, EPS, df, g, dx_out=dx)
        if record: e[3].record()
        P.dps_adjoint_finalize(tree, dattrs_out=dattrs)
        if record: e[4].record()
        if record:
            for i, k in enumerate(names):
                ev[k].append((e[i], e[i + 1]))

    for _ in range(warmup):
        step(False)
    torch.cuda.synchronize()
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for _ in range(steps):
        step(True)
    end.record()
    torch.cuda.synchronize()
    total_ms = start.elapsed_time(end)
    per = {k: sum(a.elapsed_time(b) for a, b in v) / len(v) for k, v in ev.items()}
    graph_ms = None
    if graph:
        # the same step captured once and replayed
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            step(False)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        cg = torch.cuda.CUDAGraph()
        with torch.cuda.graph(cg):
            step(False)
        for _ in range(max(warmup, 1)):
            cg.replay()
        torch.cuda.synchronize()
        start.record()
        for _ in range(steps):
            cg.replay()
        end.record()
        torch.cuda.synchronize()
        graph_ms = start.elapsed_time(end) / steps
        del cg
    # the adjoint with cotangents of the spatial gradients as well (losses
    # built on grad D, like the paper's surface density): same traversal, the
    # Hessian of each accepted source applied to the cotangents
    gen = torch.Generator(device="cuda").manual_seed(19)
    dg = torch.randn((Q, C, 3), device="cuda", generator=gen)
    P.dps_adjoint_zero(tree)
    P.dps_adjoint_accumulate_grad(tree, x, BETA, EPS, dg, df=df, dx_out=dx)
    torch.cuda.synchronize()
    gms = []
    for _ in range(3):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        P.dps_adjoint_zero(tree)
        a.record()
        P.dps_adjoint_accumulate_grad(tree, x, BETA, EPS, dg, df=df, dx_out=dx)
        b.record()
        torch.cuda.synchronize()
        gms.append(a.elapsed_time(b))
    del dg
    # the adjoint that forms dL/dx in its own walk (no forward gradients at hand)
    wms = []
    for _ in range(3):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        P.dps_adjoint_zero(tree)
        a.record()
        P.dps_adjoint_accumulate(tree, x, BETA, EPS, df, dx_out=dx)
        b.record()
        torch.cuda.synchronize()
        wms.append(a.elapsed_time(b))
    counts = P.dps_query_counts(tree, x, BETA)
    csum = counts.to(torch.int64).sum(0).tolist()
    info = P.dps_tree_info(tree)
    P.dps_destroy(tree)
    per["adjoint_accumulate_with_grad_cotangents"] = sorted(gms)[1]
    per["adjoint_accumulate_dx_in_walk"] = sorted(wms)[1]
    return {"ms_per_step": total_ms / steps, "graph_ms_per_step": graph_ms, "build_ms": build_ms, "kernel_ms": per,
            "counts_total": csum, "tree": info, "packet": {"query": tuned["query"], "adjoint": tuned["adjoint"], "flags": tuned["flags"]}}


def time_batched(P, steps, warmup):
    """The batched multi-view + shadow-ray step (see the module docstring),
    eager once and then as replays of one captured graph."""
    import torch
    import workloads
    from workloads import render as R
    from paper_2405_16788_amd import autotune
    t0 = time.time()
    p, n, A, attrs = workloads.sfm_8m_cloud()
    batch = workloads.make_ray_batch()
    dev = [torch.from_numpy(a).cuda() for a in (p, n, A, attrs)]
    M, C = p.shape[0], attrs.shape[1]
    del p, n, A, attrs
    log(f"[bench] batched inputs generated in {time.time() - t0:.1f}s: M={M} primaries={batch.Q} "
        f"rays={batch.n_rays}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tree = P.dps_build(*dev, leaf_size=LEAF, storage="bf16")
    torch.cuda.synchronize()
    build_ms = (time.perf_counter() - t0) * 1e3
    attrs_d = dev[3]
    del dev
    # a contiguous slice from the middle of the primaries (the larger views,
    # which hold most of the samples), as the autotuner takes by default
    n_tune = min(batch.Q, 1 << 25)
    s0 = (batch.Q - n_tune) // 2 // 256 * 256
    df = torch.ones((n_tune, C), device="cuda")
    tuned = autotune.tune(tree, batch.x[s0:s0 + n_tune], df, BETA, EPS, sample=n_tune, cache="", verbose=True)
    del df

    def step():
        a = attrs_d.detach().requires_grad_(True)
        xl = batch.x.detach().requires_grad_(True)
        loss, aux = R.batched_forward(P.dipole_sum, a, xl, tree, batch, BETA, EPS)
        da, dx = torch.autograd.grad(loss, [a, xl])
        return loss.detach(), aux, da, dx

    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        out = step()  # warm-up (allocator, kernels)
        del out
        torch.cuda.synchronize()
        start.record(side)
        out = step()
        end.record(side)
        torch.cuda.synchronize()
        eager_ms = start.elapsed_time(end)
        n_hits, q_count = int(out[1]["n_hits"]), int(out[1]["q_count"][0])
        del out
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        g_out = step()
    for _ in range(max(warmup, 1)):
        graph.replay()
    torch.cuda.synchronize()
    start.record()
    for _ in range(steps):
        graph.replay()
    end.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(end) / steps
    if int(g_out[1]["n_hits"]) != n_hits:
        raise RuntimeError("graph replay found a different number of hits than the eager step")
    P.dps_check(tree)
    info = P.dps_tree_info(tree)
    del graph, g_out
    P.dps_destroy(tree)
    K = batch.S_shadow
    queries = batch.Q + n_hits * K + n_hits
    return {"value": queries / (ms * 1e-3), "unit": "queries/s", "ms_per_step": ms, "eager_ms_per_step": eager_ms,
            "steps": steps, "queries_per_step": queries, "primary_queries": batch.Q,
            "shadow_rays": n_hits, "shadow_queries": n_hits * K, "hit_point_queries": n_hits,
            "shadow_rows_evaluated": q_count,
            "build_ms": build_ms, "tree_nodes": info["n_nodes"], "tree_depth": info["depth"],
            "storage": "bf16", "packet": {"query": tuned["query"], "adjoint": tuned["adjoint"], "flags": tuned["flags"]},
            "workload": f"sfm-8m: {M} points, views {'/'.join(str(r) for r in batch.res)} squared x "
                        f"{batch.S} samples = {batch.Q} primary samples + {K} per shadow ray + 1 hit-point query per hit, C={C}, "
                        f"beta={BETA}, eps={EPS:.5f}, leaf {LEAF}",
            "step": "refit + primary query (values, gradients) + hit search + shadow query (channel 0, device "
                    "row count) + hit-point query (values, gradients, device row count) + render proxy with the "
                    "direct shadow term + backward (value, gradient-cotangent and shadow adjoints, autograd of the "
                    "proxy), one graph"}


def time_grid(P, dev_in, res, reps=3):
    import torch
    p, n, A, attrs = dev_in[:4]
    tree = P.dps_build(p, n, A, attrs, leaf_size=LEAF)
    dims, origin, spacing = (res,) * 3, (-1.05,) * 3, (2.1 / (res - 1),) * 3
    f = torch.empty((res, res, res, 1), device="cuda")
    P.dps_query_grid(tree, origin, spacing, dims, BETA, EPS, c_begin=0, n_channels=1, f_out=f)
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        P.dps_query_grid(tree, origin, spacing, dims, BETA, EPS, c_begin=0, n_channels=1, f_out=f)
        b.record()
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b))
    P.dps_destroy(tree)
    ms = sorted(ts)[len(ts) // 2]
    return {"value": res ** 3 / (ms * 1e-3), "unit": "points/s", "ms": ms, "points": res ** 3,
            "workload": f"{res}^3 grid over [-1.05, 1.05]^3 on the sfm-1m tree, geometry channel, values only, "
                        f"FP32 storage"}


def time_appearance(P, dev_in, steps, warmup, K=32):
    """Geometry plus appearance channels (C = 1 + K): the geometry channel
    with the dipole kernel (values and gradients), K appearance attributes
    with the monopole kernel (values), forward and adjoint of both, on two
    trees over the same points."""
    import torch
    import workloads
    p, n, A, attrs, x = dev_in[:5]
    Q, M = x.shape[0], p.shape[0]
    app = torch.from_numpy(workloads.appearance_attrs(M, K, 73)).cuda()
    geo = attrs[:, :1].contiguous()
    from paper_2405_16788_amd import autotune
    tg = P.dps_build(p, n, A, geo, leaf_size=LEAF)
    ta = P.dps_build(p, n, A, app, leaf_size=LEAF, kernel="monopole")
    gen = torch.Generator(device="cuda").manual_seed(77)
    dfg = torch.randn((Q, 1), device="cuda", generator=gen)
    dfa = torch.randn((Q, K), device="cuda", generator=gen)
    tuned = {"geometry": autotune.tune(tg, x, dfg, BETA, EPS, cache="", verbose=True),
             "appearance": autotune.tune(ta, x, dfa, BETA, EPS, cache="", verbose=True, grad=False)}
    fg, gg = torch.empty((Q, 1), device="cuda"), torch.empty((Q, 1, 3), device="cuda")
    fa = torch.empty((Q, K), device="cuda")
    dxg, dxa = torch.empty((Q, 3), device="cuda"), torch.empty((Q, 3), device="cuda")
    dag, daa = torch.empty((M, 1), device="cuda"), torch.empty((M, K), device="cuda")
    names = ["refit", "geometry_query", "appearance_query", "geometry_adjoint", "appearance_adjoint_zero",
             "appearance_adjoint_accumulate", "appearance_adjoint_finalize"]
    ev = {k: [] for k in names}

    def step(record):
        e = [torch.cuda.Event(enable_timing=True) for _ in range(len(names) + 1)] if record else None
        if record: e[0].record()
        P.dps_set_attributes(tg, geo)
        P.dps_set_attributes(ta, app)
        if record: e[1].record()
        P.dps_query(tg, x, BETA, EPS, f_out=fg, g_out=gg)
        if record: e[2].record()
        P.dps_query(ta, x, BETA, EPS, grad=False, f_out=fa)
        if record: e[3].record()
        P.dps_adjoint_zero(tg)
        P.dps_adjoint_accumulate(tg, x, BETA, EPS, dfg, dx_out=dxg)
        P.dps_adjoint_finalize(tg, dattrs_out=dag)
        if record: e[4].record()
        P.dps_adjoint_zero(ta)
        if record: e[5].record()
        P.dps_adjoint_accumulate(ta, x, BETA, EPS, dfa, dx_out=dxa)
        if record: e[6].record()
        P.dps_adjoint_finalize(ta, dattrs_out=daa)
        if record: e[7].record()
        if record:
            for i, k in enumerate(names):
                ev[k].append((e[i], e[i + 1]))

    for _ in range(warmup):
        step(False)
    torch.cuda.synchronize()
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(steps):
        step(True)
    end.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(end) / steps
    per = {k: sum(a.elapsed_time(b) for a, b in v) / len(v) for k, v in ev.items()}
    visits, nfar, leaves, near = P.dps_query_counts(ta, x, BETA).to(torch.int64).sum(0).tolist()
    P.dps_check(tg)
    P.dps_check(ta)
    P.dps_destroy(tg)
    P.dps_destroy(ta)
    rl = {}
    for kname, flops, kms in (("appearance_query", flops_mono_fwd(K), per["appearance_query"]),
                              ("appearance_adjoint_accumulate", flops_mono_adj(K),
                               per["appearance_adjoint_accumulate"])):
        fl = flops["test"] * visits + flops["far"] * nfar + flops["near"] * near
        ach = fl / (kms * 1e-3) / 1e12
        rl[kname] = {"bound": "alu", "achieved": ach, "peak": MI355X_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
                     "frac": ach / MI355X_FP32_VECTOR_TFLOPS, "flops_per_launch": fl, "avg_launch_ms": kms,
                     "frac_nonpacked": ach / MI355X_FP32_VECTOR_NONPACKED_TFLOPS}
    return {"value": Q / (ms * 1e-3), "unit": "queries/s", "ms_per_step": ms, "steps": steps, "kernel_ms": per,
            "roofline": rl, "packet": {k: {"query": v["query"], "adjoint": v["adjoint"], "flags": v["flags"]}
                                       for k, v in tuned.items()},
            "workload": f"sfm-1m: {M} points, {Q} queries; geometry channel (dipole kernel, values + gradients) "
                        f"and K={K} appearance attributes N(0,1) (monopole kernel, values), C={1 + K}, FP32 storage",
            "step": "refit both trees + geometry query + appearance query + both adjoints (zero, accumulate with "
                    "dL/dx, finalize)"}


def time_frontend(P, steps, warmup, n_march=1024, counts=(24, 48, 8), n_rays=None):
    """The ray front-end of one view (or of n_rays random pixels of it, a
    training batch, kept in tile order): dense march for each ray's first
    crossing, sample placement around it, and the query (values and
    gradients, all channels) of the placed samples.  The march runs ray-major
    with 2 samples per lane; the placed samples of a whole view are queried in
    the [tile, sample, lane] layout (neighbouring pixels share a wavefront),
    those of a sparse batch ray-major (one ray's window samples share one),
    the faster layout for each."""
    import numpy as np
    import torch
    import workloads
    p, n, A, attrs = workloads.winding_cloud(workloads.SFM_1M_SURFACE, workloads.SFM_1M_OUTLIERS, 10)
    o, d, tn, tf = workloads.tile_camera_rays(workloads.sfm_camera(11), RES)
    if n_rays is not None:
        sel = np.sort(np.random.default_rng(79).choice(o.shape[0], n_rays, replace=False))
        o, d, tn, tf = (np.ascontiguousarray(a[sel]) for a in (o, d, tn, tf))
    dev = [torch.from_numpy(a).cuda() for a in (p, n, A, attrs, o, d, tn, tf)]
    tree = P.dps_build(*dev[:4], leaf_size=LEAF)
    od, dd, tnd, tfd = dev[4:]
    R, C, S = o.shape[0], attrs.shape[1], sum(counts)
    sparse = n_rays is not None
    # measured on this workload: a batch of 4096 rays marches fastest with 1
    # sample per lane (64-sample chunks balance better over few rays), a whole
    # view with 2
    march_k = 1 if sparse else 2
    query_k, tile_layout = (1, False) if sparse else (2, True)
    gen = torch.Generator(device="cuda").manual_seed(78)
    u = torch.rand((R, S), device="cuda", generator=gen)
    hit = torch.empty(R, device="cuda", dtype=torch.int32)
    hv = torch.empty((R, 2), device="cuda")
    t = torch.empty((R, S), device="cuda")
    x = torch.empty((R * S, 3), device="cuda")
    f = torch.empty((R * S, C), device="cuda")
    g = torch.empty((R * S, C, 3), device="cuda")
    # a training batch also runs the backward of its placed samples: the
    # two-stage adjoint with N(0,1) cotangents (seed 80) standing in for the
    # loss gradient, dL/dattrs in caller order and dL/dx per sample
    if sparse:
        df = torch.randn((R * S, C), device="cuda", generator=torch.Generator(device="cuda").manual_seed(80))
        dx = torch.empty((R * S, 3), device="cuda")
        dattrs = torch.empty((p.shape[0], C), device="cuda")
    names = ["march", "resample", "query"] + (["adjoint"] if sparse else [])
    ev = {k: [] for k in names}

    def step(record):
        e = [torch.cuda.Event(enable_timing=True) for _ in range(len(names) + 1)] if record else None
        if record: e[0].record()
        P.dps_set_launch(tree, march_k, 0, 0)
        P.dps_ray_march(tree, od, dd, tnd, tfd, n_march, BETA, EPS, hit_out=hit, values_out=hv)
        if record: e[1].record()
        P.dps_ray_resample(od, dd, tnd, tfd, n_march, hit, hv, u, counts=counts, tile_layout=tile_layout, t_out=t,
                           x_out=x)
        if record: e[2].record()
        P.dps_set_launch(tree, query_k, 0, 0)
        if sparse:
            # measured on this workload: the walks of a batch this small are
            # bound by its heaviest wavefronts; dividing each tile's walk over
            # 2 (query, still order-independent) / 4 (adjoint) wavefronts at
            # tree level 3 shortens them
            P.dps_set_split(tree, 2, 4, 3)
        P.dps_query(tree, x, BETA, EPS, f_out=f, g_out=g)
        if record: e[3].record()
        if sparse:
            # dL/dx from the query's gradients; the walk adds the increments
            P.dps_set_launch(tree, 0, 1, 0)
            P.dps_adjoint_zero(tree)
            P.dps_adjoint_accumulate_from_forward(tree, x, BETA, EPS, df, g, dx_out=dx)
            P.dps_adjoint_finalize(tree, dattrs_out=dattrs)
            if record: e[4].record()
        if record:
            for i, k in enumerate(names):
                ev[k].append((e[i], e[i + 1]))

    for _ in range(warmup):
        step(False)
    torch.cuda.synchronize()
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(steps):
        step(True)
    end.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(end) / steps
    per = {k: sum(a.elapsed_time(b) for a, b in v) / len(v) for k, v in ev.items()}
    # samples the march needs: up to and including j + 1 on a crossing, all n
    # otherwise (the ray-major march also walks chunks past a crossing that
    # were already running when it was found)
    n_eval = torch.where(hit >= 0, hit.to(torch.int64) + 2, torch.full_like(hit, n_march, dtype=torch.int64))
    total = int(n_eval.sum().item())
    hit_frac = float((hit >= 0).float().mean().item())
    # traversal counts per evaluated sample, from dps_query_counts on the evaluated
    # samples of every stride-th ray (the positions of the march formula)
    stride = max(1, R // 2048)
    sel = torch.arange(0, R, stride, device="cuda")
    ks = torch.arange(n_march, device="cuda", dtype=torch.float32)
    h = (tfd[sel] - tnd[sel]) / n_march
    ts = tnd[sel, None] + (ks[None, :] + 0.5) * h[:, None]
    keep = ks[None, :] < n_eval[sel, None].to(torch.float32)
    xs = (od[sel, None, :] + ts[..., None] * dd[sel, None, :])[keep].contiguous()
    c = P.dps_query_counts(tree, xs, BETA).to(torch.int64).sum(0).tolist()
    m = xs.shape[0]
    fv = flops_values(1)
    fl = total * (fv["test"] * c[0] + fv["far"] * c[1] + fv["near"] * c[3]) / m
    ach = fl / (per["march"] * 1e-3) / 1e12
    # the Harnack-accelerated march beside it (same outputs where its bound
    # holds; not part of the step): one warm-up and one timed launch
    P.dps_set_launch(tree, march_k, 0, 0)
    hh = torch.empty_like(hit)
    vh = torch.empty_like(hv)
    evh = torch.empty_like(hit)
    P.dps_ray_march(tree, od, dd, tnd, tfd, n_march, BETA, EPS, hit_out=hit, values_out=hv)
    P.dps_ray_march_harnack(tree, od, dd, tnd, tfd, n_march, BETA, EPS, lower=-0.25, hit_out=hh, values_out=vh,
                            evals_out=evh)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    P.dps_ray_march_harnack(tree, od, dd, tnd, tfd, n_march, BETA, EPS, lower=-0.25, hit_out=hh, values_out=vh,
                            evals_out=evh)
    e1.record()
    torch.cuda.synchronize()
    harnack = {"ms": e0.elapsed_time(e1), "lower": -0.25, "evaluations_per_ray": float(evh.float().mean().item()),
               "dense_samples_per_ray": total / R,
               "same_as_dense_march": bool(torch.equal(hh, hit) and torch.equal(vh, hv))}
    P.dps_check(tree)
    P.dps_destroy(tree)
    return {"value": R / (ms * 1e-3), "unit": "rays/s", "ms_per_step": ms, "steps": steps, "kernel_ms": per,
            "harnack_march": harnack,
            "march": {"samples_evaluated": total, "samples_per_s": total / (per["march"] * 1e-3),
                      "hit_fraction": hit_frac, "per_sample": {"nodes_visited": c[0] / m, "far_nodes": c[1] / m,
                                                                "near_points": c[3] / m},
                      "roofline": {"bound": "alu", "achieved": ach, "peak": MI355X_FP32_VECTOR_TFLOPS,
                                   "unit": "TFLOP/s", "frac": ach / MI355X_FP32_VECTOR_TFLOPS,
                                   "frac_nonpacked": ach / MI355X_FP32_VECTOR_NONPACKED_TFLOPS,
                                   "flops_per_launch": fl,
                                   "counts_from": f"dps_query_counts over the {m} evaluated samples of every "
                                                  f"{stride}th ray"}},
            "workload": f"sfm-1m with unit geometry attributes (winding number), "
                        + (f"{R} random pixels of " if n_rays is not None else "one ")
                        + f"{RES}x{RES} view in 8x8 tiles"
                        + (" (ray order kept)" if n_rays is not None else "")
                        + f": {n_march}-sample march on channel 0 (ray-major, k={march_k}), "
                        + f"{'/'.join(map(str, counts))} samples placed "
                        f"(or {S} uniform), query of the {R * S} placed samples (values + gradients, C={C}, "
                        f"k={query_k}, {'[tile, sample, lane]' if tile_layout else 'ray-major'} order)"
                        + (", adjoint of the placed samples (N(0,1) cotangents, k=1, dL/dx from the query's "
                           "gradients); query and adjoint walks split over 2 / 4 wavefronts per tile at tree "
                           "level 3" if sparse else "")
                        + ", FP32 storage",
            "step": "ray march + resample + query of the placed samples"
                    + (" + their adjoint (zero, accumulate, finalize)" if sparse else "")}


def host_cpu():
    """CPU model, logical CPUs, the CPUs this process may run on, and the
    threads the oracle legs use: the affinity set, capped by OMP_NUM_THREADS
    when that is set (the share of the host that goes with one GPU)."""
    model = "unknown"
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                model = ln.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        aff = len(os.sched_getaffinity(0))
    except AttributeError:
        aff = os.cpu_count() or 1
    threads = aff
    omp = os.environ.get("OMP_NUM_THREADS", "")
    if omp.isdigit() and int(omp) > 0:
        threads = min(threads, int(omp))
    return {"model": model, "nproc": os.cpu_count(), "affinity": aff, "threads": threads,
            "omp_num_threads": omp or None}


def cpu_baseline(np, p, n, A, attrs, x, df, seconds):
    """The FP64 oracle on the host's cores: Barnes-Hut forward + adjoint on a
    bounded sample of the workload's queries (all threads, and one thread),
    and the direct O(Q M) sum + its adjoint on 512 of the queries."""
    import oracle
    oracle.build(force=False)
    host = host_cpu()
    cores = host["threads"]
    T = oracle.Tree(p, n, A, attrs, LEAF)
    rng = np.random.default_rng(18)

    def run(k, nt):
        idx = np.sort(rng.choice(x.shape[0], size=k, replace=False))
        xs, dfs = x[idx], df[idx]
        t0 = time.perf_counter()
        T.query(xs, BETA, EPS, nthreads=nt)
        T.adjoint(xs, BETA, EPS, dfs, nthreads=nt)
        return time.perf_counter() - t0

    # the oracle adjoint has a fixed cost (thread-private accumulators over all
    # nodes and points), so calibrate time = a + b k on two sample sizes
    k1, k2 = 8192, 32768
    t1, t2 = run(k1, cores), run(k2, cores)
    b = max((t2 - t1) / (k2 - k1), 1e-9)
    a = max(t1 - b * k1, 0.0)
    k = int(min(x.shape[0], max(k2, (seconds - a) / b)))
    dt = run(k, cores)
    k_one = 65536
    dt_one = run(k_one, 1)
    # direct sum (eq. dipole_sum, no tree) and its exact adjoint on a fixed
    # 4096-query subset (seed 18), the O(Q M) reference cost
    n_dir = min(4096, x.shape[0])
    idx = np.sort(np.random.default_rng(18).choice(x.shape[0], size=n_dir, replace=False))
    t0 = time.perf_counter()
    oracle.direct(p, n, A, attrs, x[idx], EPS, nthreads=cores)
    oracle.direct_adjoint(p, n, A, attrs, x[idx], EPS, df[idx], nthreads=cores)
    dt_dir = time.perf_counter() - t0
    return {"value": k / dt, "unit": "queries/s", "cores": cores, "kind": "oracle",
            "sample": f"{k} queries drawn (seed 18) from the {x.shape[0]}-query set; FP64 Barnes-Hut "
                      f"forward (values+gradients) + adjoint on the full {p.shape[0]}-point tree, "
                      f"{dt:.1f} s wall on {cores} threads; tree build excluded",
            "host": host,
            "one_thread": {"value": k_one / dt_one, "unit": "queries/s", "sample": f"{k_one} queries, {dt_one:.1f} s"},
            "direct_sum": {"value": n_dir / dt_dir, "unit": "queries/s", "cores": cores,
                           "sample": f"{n_dir} queries (seed 18), FP64 direct sum over all {p.shape[0]} points "
                                     f"(values + gradients) + its adjoint, {dt_dir:.1f} s wall",
                           "extrapolated_s_for_all_queries": x.shape[0] / n_dir * dt_dir}}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (--gpus {args.gpus} requested); the multi-GPU design "
              "(replicated tree, query sharding, one all-reduce of dL/dattrs) is not built.", file=sys.stderr)
        sys.exit(2)
    import torch
    if args.copy_reference:
        a = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
        a.fill_(1.0)
        torch.cuda.synchronize()
        b = a.clone()
        torch.cuda.synchronize()
        print(json.dumps({"copy_reference_bytes": a.numel() * 4, "ok": bool(b[-1].item() == 1.0)}))
        return
    import paper_2405_16788_amd as P
    P.load()
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.batched_only:
        b = time_batched(P, args.batched_steps, args.warmup)
        print(json.dumps({"metric": "batched dipole-sum queries/sec fwd+adjoint, 8M pts, 8 views + shadow rays, "
                                    "BF16-stored, one graph", "value": b["value"], "unit": "queries/s", "n_gpus": 1,
                          "steps": args.batched_steps, "warmup": args.warmup, "ms_per_step": b["ms_per_step"],
                          "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
                          "data": "synthetic", "config": {"workload": b["workload"]}, "batched": b}), flush=True)
        return
    p, n, A, attrs, x, df, np = make_inputs(args.res)
    dev_in = [torch.from_numpy(a).cuda() for a in (p, n, A, attrs, x, df)]
    Q, C = x.shape[0], attrs.shape[1]
    storages = ["fp32", "bf16"] if args.storage == "both" else [args.storage]
    res = {}
    for st in storages:
        log(f"[bench] timing storage={st}")
        res[st] = time_storage(P, dev_in, st, args.steps, args.warmup, args.packet,
                               graph=(st == "bf16" and not args.no_graph))
        log(f"[bench] {st}: {res[st]['ms_per_step']:.2f} ms/step (graph {res[st]['graph_ms_per_step']}), "
            f"kernels {res[st]['kernel_ms']}")
    main_st = "fp32" if "fp32" in res else storages[0]
    r = res[main_st]
    visits, nfar, leaves, near = r["counts_total"]
    ffw, fad = flops_fwd(C), flops_adj_fwdgrad(C)
    fl_q = ffw["test"] * visits + ffw["far"] * nfar + ffw["near"] * near
    fl_a = fad["test"] * visits + fad["far"] * nfar + fad["near"] * near + fad["query"] * Q
    bfw, bad = bytes_fwd(C), bytes_adj(C)
    by_q = bfw["visit"] * visits + bfw["far"] * nfar + bfw["near"] * near + bfw["io"] * Q
    by_a = bad["visit"] * visits + bad["far"] * nfar + bad["near"] * near + bad["io"] * Q
    kq, ka = r["kernel_ms"]["query"], r["kernel_ms"]["adjoint_accumulate"]
    dom, fl, by, ms = ("adjoint_accumulate", fl_a, by_a, ka) if ka >= kq else ("query", fl_q, by_q, kq)
    achieved = fl / (ms * 1e-3) / 1e12
    pk = r["packet"]
    adj = dom == "adjoint_accumulate"
    persistent = bool(pk["flags"] & (8 if adj else 4))
    kname = ("k_adjoint" if adj else "k_query") + ("_persistent" if persistent else "")
    # queries per lane the kernel ran with: the query with gradients over 4
    # channels runs packets of 4 as 2
    k_run = pk["adjoint"] if adj else min(pk["query"], 2)
    traffic, traffic_src = committed_traffic(kname, k_run, persistent, main_st)
    out = {
        "metric": METRIC,
        "value": Q / (r["ms_per_step"] * 1e-3),
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"sfm-1m: {p.shape[0]} points, {args.res}x{args.res} rays x {SAMPLES} samples "
                               f"= {Q} queries, C={C}, beta={BETA}, eps={EPS:.5f}, leaf {LEAF}",
                   "storage": main_st, "step": "refit + query(values, gradients) + adjoint(zero, accumulate "
                                               "with dL/dx from the query's gradients, finalize)"},
        "roofline": {"bound": "alu", "kernel": dom, "achieved": achieved, "peak": MI355X_FP32_VECTOR_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / MI355X_FP32_VECTOR_TFLOPS, "traffic": traffic,
                     "traffic_source": traffic_src, "flops_per_launch": fl, "avg_launch_ms": ms,
                     "peak_nonpacked": MI355X_FP32_VECTOR_NONPACKED_TFLOPS,
                     "frac_nonpacked": achieved / MI355X_FP32_VECTOR_NONPACKED_TFLOPS,
                     "hbm_achieved_GBps": (traffic / (ms * 1e-3) / 1e9) if traffic else None},
        "roofline_hbm_algorithmic": {
            "kernel": dom, "bytes_per_launch": by, "achieved": by / (ms * 1e-3) / 1e9, "peak": MI355X_HBM_TBS * 1e3,
            "unit": "GB/s", "frac": by / (ms * 1e-3) / 1e9 / (MI355X_HBM_TBS * 1e3),
            "note": "bytes the method touches if nothing were shared; coherent wavefronts share node and moment "
                    "loads through the caches, so this exceeds HBM peak"},
        "per_query": {"nodes_visited": visits / Q, "far_nodes": nfar / Q, "leaves_opened": leaves / Q,
                      "near_points": near / Q},
        "paper_timings": {
            "hardware": "1x NVIDIA RTX 4090 (Sec. 7.1)",
            "figures": "training 1000 iterations in 3 min, 3000 in 8 min, 20000 in 1 h, 4096 rays per iteration, "
                       "1024 march + 80 samples per ray (whole training step: MLP, renderer, optimiser)",
            "note": "the paper gives no kernel-level query rate, so there is no number for this metric to compare "
                    "against (vs_baseline null)"},
    }
    fw = flops_adj(C)
    fl_w = fw["test"] * visits + fw["far"] * nfar + fw["near"] * near
    out["roofline"]["adjoint_dx_in_walk"] = {
        "note": "dps_adjoint_accumulate forming dL/dx in its own walk (no forward gradients at hand)",
        "avg_launch_ms": r["kernel_ms"]["adjoint_accumulate_dx_in_walk"], "flops_per_launch": fl_w,
        "achieved": fl_w / (r["kernel_ms"]["adjoint_accumulate_dx_in_walk"] * 1e-3) / 1e12}
    for st, rr in res.items():
        out[f"{st}_stored"] = {"value": Q / (rr["ms_per_step"] * 1e-3), "ms_per_step": rr["ms_per_step"],
                               "kernel_ms": rr["kernel_ms"], "build_ms": rr["build_ms"],
                               "tree_nodes": rr["tree"]["n_nodes"], "tree_bytes": rr["tree"]["bytes"],
                               "packet": rr["packet"]}
        if rr["graph_ms_per_step"]:
            out[f"{st}_stored_graph"] = {"value": Q / (rr["graph_ms_per_step"] * 1e-3),
                                         "ms_per_step": rr["graph_ms_per_step"],
                                         "step": "the same step captured in one graph and replayed"}
    # marching-cubes grid on the same tree: 512^3 points over the bounding
    # cube, geometry channel only, positions generated in the kernels
    log("[bench] 512^3 grid query")
    out["grid_512"] = time_grid(P, dev_in, 512)
    if not args.no_appearance:
        log("[bench] geometry + 32 appearance channels")
        out["appearance_k32"] = time_appearance(P, dev_in, max(1, min(args.steps, 5)), 1)
        log(f"[bench] appearance: {out['appearance_k32']['ms_per_step']:.1f} ms/step, "
            f"kernels {out['appearance_k32']['kernel_ms']}")
    if not args.no_frontend:
        log("[bench] ray front-end (march + resample + query)")
        out["ray_frontend"] = time_frontend(P, max(1, min(args.steps, 3)), 1)
        out["ray_frontend_batch"] = time_frontend(P, max(1, min(args.steps, 5)), 1, n_rays=4096)
        log(f"[bench] ray front-end: {out['ray_frontend']['ms_per_step']:.1f} ms/view, "
            f"kernels {out['ray_frontend']['kernel_ms']}")
        log(f"[bench] ray front-end, 4096-ray batch: {out['ray_frontend_batch']['ms_per_step']:.2f} ms, "
            f"kernels {out['ray_frontend_batch']['kernel_ms']}")
        for key in ("ray_frontend", "ray_frontend_batch"):
            hm = out[key]["harnack_march"]
            log(f"[bench] {key}: Harnack-accelerated march {hm['ms']:.1f} ms, {hm['evaluations_per_ray']:.0f} "
                f"evaluations per ray (dense {hm['dense_samples_per_ray']:.0f}), same as the dense march: "
                f"{hm['same_as_dense_march']}")
    if not args.no_cpu_baseline:
        log("[bench] CPU oracle baseline")
        out["cpu_baseline"] = cpu_baseline(np, p, n, A, attrs, x, df, args.cpu_seconds)
    del p, n, A, attrs, x, df, dev_in
    if not args.no_batched:
        import gc
        gc.collect()
        torch.cuda.empty_cache()
        log("[bench] batched workload")
        out["batched"] = time_batched(P, args.batched_steps, args.warmup)
        log(f"[bench] batched: {out['batched']['ms_per_step']:.1f} ms/step, "
            f"{out['batched']['value'] / 1e6:.1f} M queries/s")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
