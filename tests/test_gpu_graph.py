"""Batching pattern: a whole training step (moment refit, primal query with
gradients, adjoint zero / accumulate / finalize) captured once in a hipGraph
and replayed.  Every replay is compared with the eager result of the same
step, with eager work and synchronisations between the replays; the forward
outputs are deterministic (bit-identical), the atomically accumulated
attribute gradients agree to FP64 summation-order rounding."""
import numpy as np
import pytest

import workloads
from parity import to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("flags", [3, 12])
def test_step_graph_replays_match_eager(flags):
    import torch
    import paper_2405_16788_amd as P
    P.load()
    p, n, A, mu = workloads.sfm_cloud(200_000, 10_000, 10)
    x = workloads.ray_samples(workloads.sfm_camera(11), 64, 64, 128, 12, order="tile")
    Q, C = x.shape[0], mu.shape[1]
    df = workloads.cotangents(Q, C, 17)
    pd, nd, Ad, mud, xd, dfd = to_dev(p, n, A, mu, x, df)
    tree = P.dps_build(pd, nd, Ad, mud, leaf_size=16)
    P.dps_set_launch(tree, 2, 4, flags)
    beta, eps = 2.0, 0.01414
    f = torch.empty((Q, C), device="cuda")
    g = torch.empty((Q, C, 3), device="cuda")
    dx = torch.empty((Q, 3), device="cuda")
    da = torch.empty((tree.M, C), device="cuda")

    def step():
        P.dps_set_attributes(tree, mud)
        P.dps_query(tree, xd, beta, eps, f_out=f, g_out=g)
        P.dps_adjoint_zero(tree)
        P.dps_adjoint_accumulate(tree, xd, beta, eps, dfd, dx_out=dx)
        P.dps_adjoint_finalize(tree, dattrs_out=da)

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    ref = {k: to_host(v).copy() for k, v in (("f", f), ("g", g), ("dx", dx), ("da", da))}

    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step()
    for r in range(4):
        for v in (f, g, dx, da):
            v.fill_(float("nan"))  # eager work between replays
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert np.array_equal(to_host(f), ref["f"]), f"replay {r}: f differs"
        assert np.array_equal(to_host(g), ref["g"]), f"replay {r}: grad differs"
        assert np.array_equal(to_host(dx), ref["dx"]), f"replay {r}: dx differs"
        got = to_host(da).astype(np.float64)
        scale = np.abs(ref["da"]).max()
        assert np.max(np.abs(got - ref["da"])) <= 1e-6 * scale, f"replay {r}: dattrs differs"
        # eager calls between replays keep working on the same tree
        P.dps_query(tree, xd[:1000].contiguous(), beta, eps)
    P.dps_check(tree)
