"""Failure paths, forced from the host so that every kernel exits normally:
the traversal step guard (a lowered step limit makes every traversal stop
early and record the tree's sticky device error, which dps_check reports),
and an allocation failure during a build (a memory cap below what the build
needs returns DPS_ERR_OOM, no handle, nothing left allocated)."""
import numpy as np
import pytest

import workloads
from parity import to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    import paper_2405_16788_amd as lib
    lib.load()
    assert torch.cuda.is_available()
    return lib


@pytest.mark.parametrize("persistent", [False, True])
def test_step_guard_reports_device_error(P, persistent):
    import torch
    p, n, A, mu = workloads.sphere_cloud(8192, 1)
    dev = to_dev(p, n, A, mu)
    tree = P.dps_build(*dev, leaf_size=16)
    good = P.dps_build(*dev, leaf_size=16)
    mono = P.dps_build(*dev, leaf_size=16, kernel="monopole")
    x = workloads.sphere_queries(5000, 2)
    df = workloads.cotangents(5000, 4, 17)
    xd, dfd = to_dev(x, df)
    flags = (P.LAUNCH_PERSISTENT_QUERY | P.LAUNCH_PERSISTENT_ADJOINT) if persistent else 0
    for t in (tree, mono):
        P.dps_set_launch(t, 0, 0, flags)
        P.dps_set_step_limit(t, 7)
    with pytest.raises(P.DpsError):
        P.dps_set_step_limit(tree, -1)
    with pytest.raises(P.DpsError):
        P.dps_set_step_limit(tree, P.dps_tree_info(tree)["n_nodes"] + 1)
    print(f"[failure] step limit 7, persistent={persistent}", flush=True)
    # every traversal kind runs to completion on the host side and returns OK
    f, g = P.dps_query(tree, xd, 2.0, 0.05)
    P.dps_query_counts(tree, xd, 2.0)
    P.dps_adjoint(tree, xd, 2.0, 0.05, dfd)
    P.dps_adjoint_zero(tree)
    P.dps_adjoint_accumulate_grad(tree, xd, 2.0, 0.05, torch.ones((5000, 4, 3), device="cuda"))
    P.dps_query_grid(tree, (-1.0, -1.0, -1.0), (0.1, 0.1, 0.1), (20, 20, 20), 2.0, 0.05, 0, 1)
    o = torch.zeros((64, 3), device="cuda")
    o[:, 2] = -3.0
    d = torch.zeros((64, 3), device="cuda")
    d[:, 2] = 1.0
    tn = torch.full((64,), 1.0, device="cuda")
    tf = torch.full((64,), 5.0, device="cuda")
    P.dps_ray_march(tree, o, d, tn, tf, 256, 2.0, 0.05, 0, 0.5)
    P.dps_query(mono, xd, 2.0, 0.05)
    P.dps_adjoint(mono, xd, 2.0, 0.05, dfd)
    torch.cuda.synchronize()
    # the guard fired: sticky device error on the limited trees only
    for t in (tree, mono):
        with pytest.raises(P.DpsError) as e:
            P.dps_check(t)
        assert e.value.status == 3
    P.dps_check(good)
    # sticky: restoring the limit does not clear it; the tree still runs
    P.dps_set_step_limit(tree, 0)
    f2, _ = P.dps_query(tree, xd, 2.0, 0.05)
    fg, _ = P.dps_query(good, xd, 2.0, 0.05)
    assert torch.equal(f2, fg)
    with pytest.raises(P.DpsError):
        P.dps_check(tree)
    for t in (tree, good, mono):
        P.dps_destroy(t)


def test_memory_cap_gives_oom_and_frees_everything(P):
    import torch
    p, n, A, mu = workloads.sfm_cloud(60000, 3000, 61)
    dev = to_dev(p, n, A, mu)
    torch.cuda.synchronize()
    ref = P.dps_build(*dev, leaf_size=16)
    need = P.dps_tree_info(ref)["bytes"]
    P.dps_destroy(ref)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    try:
        for cap in (1 << 10, need // 2, need - 1):
            P.dps_set_memory_limit(cap)
            with pytest.raises(P.DpsError) as e:
                P.dps_build(*dev, leaf_size=16)
            assert e.value.status == 2, e.value
            print(f"[failure] cap {cap} bytes (tree needs {need}): {e.value}", flush=True)
            torch.cuda.synchronize()
            # nothing of the failed build stays allocated (allocator granularity aside)
            assert torch.cuda.mem_get_info()[0] >= free0 - (4 << 20)
        # a cap the build fits under: its temporary buffers are freed before
        # the last tree arrays are allocated, so tree bytes plus the largest
        # scratch set suffice
        P.dps_set_memory_limit(64 * need)
        t = P.dps_build(*dev, leaf_size=16)
        assert P.dps_tree_info(t)["bytes"] == need
        P.dps_destroy(t)
    finally:
        P.dps_set_memory_limit(0)
    t = P.dps_build(*dev, leaf_size=16)
    P.dps_check(t)
    P.dps_destroy(t)
