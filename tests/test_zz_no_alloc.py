"""dps_adjoint_noalloc -- the adjoint of dps_adjoint with its working buffers
(node and point accumulators, tile counters) in a static per-device
workspace -- called through the C ABI and checked against dps_adjoint and the
FP64 oracle, on consecutive calls of decreasing size (the workspace keeps the
previous call's contents), under graph capture, and for a tree too large for
the workspace."""
import ctypes as ct

import numpy as np
import pytest

import workloads
from parity import TOL_FP32, norm_err, to_dev, to_host

pytestmark = pytest.mark.gpu

BETA, EPS = 2.0, 0.02


@pytest.fixture(scope="module")
def P():
    import torch
    import paper_2405_16788_amd as lib
    lib.load()
    assert torch.cuda.is_available()
    return lib


def _vp(t):
    return None if t is None else ct.c_void_p(t.data_ptr())


def _noalloc(P, tree, xd, dfd, da, dx):
    import torch
    stream = ct.c_void_p(torch.cuda.current_stream().cuda_stream)
    return P.load().dps_adjoint_noalloc(tree.handle, _vp(xd), xd.shape[0], BETA, EPS, _vp(dfd), _vp(da), _vp(dx),
                                        stream)


def _case(P, orc, cloud, Q, seed, flags):
    import torch
    p, n, A, mu = cloud
    tree = P.dps_build(*to_dev(p, n, A, mu), leaf_size=16)
    P.dps_set_launch(tree, 4, 4, flags)
    x = workloads.sphere_queries(Q, seed)
    df = workloads.cotangents(Q, mu.shape[1], seed + 1)
    xd, dfd = to_dev(x, df)
    ref = orc.Tree(p, n, A, mu, 16).adjoint(x, BETA, EPS, df)
    return tree, x, df, xd, dfd, ref


def _check(P, tree, xd, dfd, ref, tag):
    import torch
    da = torch.full((tree.M, tree.C), float("nan"), device="cuda")
    dx = torch.full((xd.shape[0], 3), float("nan"), device="cuda")
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    rc = _noalloc(P, tree, xd, dfd, da, dx)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    assert rc == 0, P.dps_last_error()
    d_ref, dx_ref = P.dps_adjoint(tree, xd, BETA, EPS, dfd)
    e = {"dattrs vs dps_adjoint": norm_err(to_host(da), to_host(d_ref), ref["sdmu"]),
         "dx vs dps_adjoint": norm_err(to_host(dx), to_host(dx_ref), ref["sdx"]),
         "dattrs vs oracle": norm_err(to_host(da), ref["dmu"], ref["sdmu"]),
         "dx vs oracle": norm_err(to_host(dx), ref["dx"], ref["sdx"])}
    print(f"[noalloc] {tag}: " + ", ".join(f"{k} {v:.3g}" for k, v in e.items()) + f"; free memory change {free1 - free0}",
          flush=True)
    assert all(v <= TOL_FP32 for v in e.values()), e
    P.dps_check(tree)
    return free1 - free0


def test_noalloc_adjoint_matches_dps_adjoint(P, orc):
    """Two calls in a row on one tree, the second with fewer queries, then a
    call on a smaller tree; the workspace is cleared by each call."""
    big = workloads.sfm_cloud(60000, 3000, 61)
    tree, x, df, xd, dfd, ref = _case(P, orc, big, 20000, 5, 12)
    _check(P, tree, xd, dfd, ref, "sfm-63k, 20000 queries, persistent")
    xs, dfs = x[:3000], df[:3000]
    xsd, dfsd = to_dev(xs, dfs)
    ref_s = orc.Tree(*big, 16).adjoint(xs, BETA, EPS, dfs)
    change = _check(P, tree, xsd, dfsd, ref_s, "same tree, 3000 queries")
    assert change >= 0  # nothing allocated by the call
    small = workloads.sphere_cloud(8192, 1)
    tree2, _, _, xd2, dfd2, ref2 = _case(P, orc, small, 2500, 7, 0)
    change = _check(P, tree2, xd2, dfd2, ref2, "sphere-8k, 2500 queries, grid launch")
    assert change >= 0
    # no queries: dL/dmu is zero
    import torch
    da = torch.full((tree2.M, tree2.C), float("nan"), device="cuda")
    assert _noalloc(P, tree2, xd2[:0], dfd2[:0], da, None) == 0
    torch.cuda.synchronize()
    assert float(da.abs().max()) == 0.0


def test_noalloc_adjoint_in_a_captured_graph(P, orc):
    import torch
    tree, x, df, xd, dfd, ref = _case(P, orc, workloads.sphere_cloud(8192, 1), 4096, 11, 12)
    da = torch.empty((tree.M, tree.C), device="cuda")
    dx = torch.empty((xd.shape[0], 3), device="cuda")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        assert _noalloc(P, tree, xd, dfd, da, dx) == 0  # warm-up outside the capture
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=side):
            rc = _noalloc(P, tree, xd, dfd, da, dx)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    assert rc == 0
    for rep, scale in enumerate((1.0, -2.5, 1.0)):
        dfd.copy_(torch.from_numpy(df * np.float32(scale)).cuda())
        graph.replay()
        torch.cuda.synchronize()
        d_ref, dx_ref = P.dps_adjoint(tree, xd, BETA, EPS, dfd)
        e1 = norm_err(to_host(da), to_host(d_ref), abs(scale) * ref["sdmu"])
        e2 = norm_err(to_host(dx), to_host(dx_ref), abs(scale) * ref["sdx"])
        print(f"[noalloc] graph replay {rep}: dattrs {e1:.3g} dx {e2:.3g}", flush=True)
        assert e1 <= TOL_FP32 and e2 <= TOL_FP32


def test_noalloc_rejects_a_tree_beyond_the_workspace(P):
    import torch
    rng = np.random.default_rng(3)
    M, C = 270000, 32
    p = rng.uniform(-1, 1, (M, 3)).astype(np.float32)
    n = rng.standard_normal((M, 3)).astype(np.float32)
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    A = np.full(M, 4.0 / M, np.float32)
    mu = rng.standard_normal((M, C)).astype(np.float32)
    tree = P.dps_build(*to_dev(p, n, A, mu), leaf_size=16)
    x = torch.zeros((64, 3), device="cuda")
    df = torch.ones((64, C), device="cuda")
    da = torch.full((M, C), 7.0, device="cuda")
    rc = _noalloc(P, tree, x, df, da, None)
    assert rc == 1
    msg = P.dps_last_error()
    print(f"[noalloc] {msg}", flush=True)
    assert "workspace" in msg
    torch.cuda.synchronize()
    assert float(da.min()) == 7.0 and float(da.max()) == 7.0  # untouched
