"""Ray front-end on the GPU (Sec. 7.1, ray sampling): the dense march
(``dps_ray_march``) against the oracle's march on the same FP32 sample
positions, and the sample placement (``dps_ray_resample``) bit for bit against
the oracle's FP32 placement on the same synthetic inputs, plus argument
checks and the march at the benchmark's 512 x 512 view of sfm-1m."""
import math

import numpy as np
import pytest

import workloads
from parity import TOL_BF16, TOL_FP32, to_dev, to_host

pytestmark = pytest.mark.gpu

BETA = 2.0
EPS = math.sqrt(2.0) * 0.01
N_MARCH = 1024


@pytest.fixture(scope="module")
def P():
    import torch
    import paper_2405_16788_amd as lib
    lib.load()
    assert torch.cuda.is_available()
    return lib


@pytest.fixture(scope="module")
def scene(orc):
    """A 21,000-point cloud with unit geometry attributes (channel 0 is the
    regularized winding number), 32 x 32 tile-ordered camera rays."""
    from oracle import rays
    p, n, A, mu = workloads.winding_cloud(20000, 1000, 90)
    o, d, tn, tf = workloads.tile_camera_rays(workloads.sfm_camera(91), 32)
    T = orc.Tree(p, n, A, mu, 16)
    ref = rays.march(T, o, d, tn, tf, N_MARCH, BETA, EPS)
    return (p, n, A, mu), (o, d, tn, tf), ref


def _check_march(hit, hv, ref, tol, level=0.5):
    """The GPU's crossing index equals the oracle's, except where a sample
    between the two lies within the tolerance band of the level (its side is
    then not fixed by the precision); the GPU's values at its own index match
    the oracle's there, and straddle the level."""
    j_o, v, sv = ref["j"], ref["v"], ref["sv"]
    n = v.shape[1]
    same = hit == j_o
    for r in np.nonzero(~same)[0]:
        a = n - 1 if hit[r] < 0 else hit[r]
        b = n - 1 if j_o[r] < 0 else j_o[r]
        lo, hi = min(a, b), min(max(a, b) + 1, n - 1)
        band = np.abs(v[r, lo:hi + 1] - level) <= tol * sv[r, lo:hi + 1]
        assert np.any(band), (r, hit[r], j_o[r])
    assert np.mean(same) >= 0.98
    h = hit >= 0
    assert np.all((hv[h, 0] >= level) != (hv[h, 1] >= level))
    rr = np.nonzero(h)[0]
    jj = hit[h]
    assert np.all(np.abs(hv[h, 0] - v[rr, jj]) <= tol * sv[rr, jj])
    assert np.all(np.abs(hv[h, 1] - v[rr, jj + 1]) <= tol * sv[rr, jj + 1])
    assert np.all(hv[~h] == 0.0)
    return int(np.sum(h))


@pytest.mark.parametrize("storage", ["fp32", "bf16"])
@pytest.mark.parametrize("k", [1, 2, 4])
def test_march_matches_oracle(P, scene, storage, k):
    (p, n, A, mu), (o, d, tn, tf), ref = scene
    print(f"[rays] march storage={storage} k={k} R={o.shape[0]} n={N_MARCH}", flush=True)
    tree = P.dps_build(*to_dev(p, n, A, mu), leaf_size=16, storage=storage)
    P.dps_set_launch(tree, k, 0, -1)
    od, dd, tnd, tfd = to_dev(o, d, tn, tf)
    hit, hv = P.dps_ray_march(tree, od, dd, tnd, tfd, N_MARCH, BETA, EPS)
    P.dps_check(tree)
    hits = _check_march(to_host(hit), to_host(hv), ref, TOL_BF16 if storage == "bf16" else TOL_FP32)
    print(f"[rays] {hits} of {o.shape[0]} rays cross the level set", flush=True)
    assert 0 < hits < o.shape[0]


def test_march_values_are_the_point_query_values(P, scene):
    """At the sample positions around each crossing (computed by the oracle's
    FP32 position formula) the point query gives the march's values."""
    from oracle import rays
    (p, n, A, mu), (o, d, tn, tf), ref = scene
    tree = P.dps_build(*to_dev(p, n, A, mu), leaf_size=16)
    od, dd, tnd, tfd = to_dev(o, d, tn, tf)
    hit, hv = P.dps_ray_march(tree, od, dd, tnd, tfd, N_MARCH, BETA, EPS)
    hit, hv = to_host(hit), to_host(hv)
    rr = np.nonzero(hit >= 0)[0]
    t, _ = rays.march_t(tn[rr], tf[rr], N_MARCH)
    x = rays.positions(o[rr], d[rr], t)
    xs = np.concatenate([x[np.arange(len(rr)), hit[rr]], x[np.arange(len(rr)), hit[rr] + 1]]).astype(np.float32)
    f, _ = P.dps_query_channels(tree, to_dev(xs)[0], BETA, EPS, 0, 1, grad=False)
    f = to_host(f)[:, 0]
    want = np.concatenate([hv[rr, 0], hv[rr, 1]])
    print(f"[rays] march vs point query: bitwise equal {np.array_equal(f, want)}, "
          f"max |diff| {np.max(np.abs(f - want)):.3g}", flush=True)
    sv = np.concatenate([ref["sv"][rr, hit[rr]], ref["sv"][rr, hit[rr] + 1]])
    assert np.all(np.abs(f - want) <= 2 * TOL_FP32 * sv)


@pytest.mark.parametrize("layout", [0, 1])
@pytest.mark.parametrize("counts,window", [((24, 48, 8), 8.0), ((3, 5, 2), 2.5)])
def test_resample_bitwise(P, orc, layout, counts, window):
    import torch
    from oracle import rays
    o, d, tn, tf = workloads.tile_camera_rays(workloads.sfm_camera(92), 32)
    R = o.shape[0] if layout else 1000
    o, d, tn, tf = o[:R], d[:R], tn[:R], tf[:R]
    S = sum(counts)
    j, vj, vj1, u = workloads.synthetic_crossings(R, N_MARCH, 93, S)
    hv = np.stack([vj, vj1], axis=1)
    dev = to_dev(o, d, tn, tf, j, hv, u)
    t, x = P.dps_ray_resample(*dev[:4], N_MARCH, dev[4], dev[5], dev[6], counts=counts, window=window,
                              tile_layout=bool(layout))
    torch.cuda.synchronize()
    tr, xr, _ = rays.resample(o, d, tn, tf, N_MARCH, j, vj, vj1, u, counts=counts, window=window)
    t, x = to_host(t), to_host(x)
    assert np.array_equal(t, tr)
    if layout:
        rows = ((np.arange(R)[:, None] // 64) * S + np.arange(S)[None, :]) * 64 + (np.arange(R)[:, None] % 64)
        xr_rows = np.empty((R * S, 3), np.float32)
        xr_rows[rows.reshape(-1)] = xr.reshape(-1, 3)
        assert np.array_equal(x, xr_rows)
    else:
        assert np.array_equal(x, xr.reshape(-1, 3))


def test_ray_arguments(P):
    import torch
    p, n, A, mu = workloads.winding_cloud(4000, 100, 94)
    tree = P.dps_build(*to_dev(p, n, A, mu), leaf_size=16)
    mono = P.dps_build(*to_dev(p, n, A, mu), leaf_size=16, kernel="monopole")
    o, d, tn, tf = to_dev(*workloads.tile_camera_rays(workloads.sfm_camera(95), 8))
    with pytest.raises(P.DpsError):
        P.dps_ray_march(mono, o, d, tn, tf, 64, BETA, EPS)
    with pytest.raises(P.DpsError):
        P.dps_ray_march(tree, o, d, tn, tf, 1, BETA, EPS)
    with pytest.raises(P.DpsError):
        P.dps_ray_march(tree, o, d, tn, tf, 64, BETA, EPS, channel=4)
    with pytest.raises(P.DpsError):
        P.dps_ray_march(tree, o, d, tn, tf, 64, -1.0, EPS)
    e = torch.empty((0, 3), device="cuda")
    z = torch.empty(0, device="cuda")
    hit, hv = P.dps_ray_march(tree, e, e, z, z, 64, BETA, EPS)
    assert hit.numel() == 0
    R = 60
    j, vj, vj1, u = (torch.from_numpy(a).cuda() for a in workloads.synthetic_crossings(R, 64, 96))
    hv = torch.stack([vj, vj1], dim=1).contiguous()
    with pytest.raises(P.DpsError):  # the tile layout needs whole tiles of 64 rays
        P.dps_ray_resample(o[:R], d[:R], tn[:R], tf[:R], 64, j, hv, u, tile_layout=True)
    with pytest.raises(P.DpsError):
        P.dps_ray_resample(o[:R], d[:R], tn[:R], tf[:R], 0, j, hv, u)
    with pytest.raises(P.DpsError):
        P.dps_ray_resample(o[:R], d[:R], tn[:R], tf[:R], 64, j, hv, u, window=-1.0)
    P.dps_check(tree)


def test_march_sfm_1m_512(P, orc):
    """The march at the benchmark's size: the 1M-point cloud with unit
    geometry attributes and the 512 x 512 view (262,144 rays x 1024 samples),
    sampled rays against the oracle's march, then the 80-sample placement in
    the tile layout and the query of the placed samples."""
    import torch
    from oracle import rays
    p, n, A, mu = workloads.winding_cloud(workloads.SFM_1M_SURFACE, workloads.SFM_1M_OUTLIERS, 10)
    o, d, tn, tf = workloads.tile_camera_rays(workloads.sfm_camera(11), 512)
    R = o.shape[0]
    print(f"[rays] sfm-1m march R={R} n={N_MARCH}", flush=True)
    tree = P.dps_build(*to_dev(p, n, A, mu), leaf_size=16)
    od, dd, tnd, tfd = to_dev(o, d, tn, tf)
    hit, hv = P.dps_ray_march(tree, od, dd, tnd, tfd, N_MARCH, BETA, EPS)
    P.dps_check(tree)
    hit_h, hv_h = to_host(hit), to_host(hv)
    frac = float(np.mean(hit_h >= 0))
    print(f"[rays] hit fraction {frac:.4f}", flush=True)
    assert 0.02 < frac < 0.9
    idx = np.sort(np.random.default_rng(97).choice(R, 160, replace=False))
    idx = np.union1d(idx, np.nonzero(hit_h >= 0)[0][:96])
    T = orc.Tree(p, n, A, mu, 16)
    ref = rays.march(T, o[idx], d[idx], tn[idx], tf[idx], N_MARCH, BETA, EPS)
    _check_march(hit_h[idx], hv_h[idx], ref, TOL_FP32)
    u = torch.rand((R, 80), device="cuda", generator=torch.Generator(device="cuda").manual_seed(98))
    t, x = P.dps_ray_resample(od, dd, tnd, tfd, N_MARCH, hit, hv, u, tile_layout=True)
    f, g = P.dps_query(tree, x, BETA, EPS)
    P.dps_check(tree)
    assert torch.isfinite(f).all() and torch.isfinite(g).all()
    assert bool((t[:, 1:] >= t[:, :-1]).all())
    # rays with a crossing: the dense window holds the level set, so placed
    # samples of the ray lie on both sides of it (a ray that only grazes the
    # level may miss one side)
    hits = torch.nonzero(hit >= 0).squeeze(1)[:256]
    rows = ((hits[:, None] // 64) * 80 + torch.arange(80, device="cuda")[None, :]) * 64 + (hits[:, None] % 64)
    fv = f[rows.reshape(-1), 0].reshape(-1, 80)
    both = ((fv >= 0.5).any(dim=1) & (fv < 0.5).any(dim=1)).float().mean().item()
    print(f"[rays] hit rays with placed samples on both sides of the level: {both:.3f}", flush=True)
    assert both >= 0.9


def test_front_end_graph_replays(P):
    """March, placement and the query of the placed samples captured in one
    graph: every replay equals the eager result, with eager work between the
    replays, and rays moved in place between replays reach the captured
    kernels."""
    import torch
    p, n, A, mu = workloads.winding_cloud(40000, 2000, 99)
    o, d, tn, tf = workloads.tile_camera_rays(workloads.sfm_camera(100), 64)
    tree = P.dps_build(*to_dev(p, n, A, mu), leaf_size=16)
    P.dps_set_launch(tree, 2, 2, P.LAUNCH_PERSISTENT_QUERY | P.LAUNCH_PERSISTENT_ADJOINT)
    od, dd, tnd, tfd = to_dev(o, d, tn, tf)
    R = o.shape[0]
    u = torch.rand((R, 80), device="cuda", generator=torch.Generator(device="cuda").manual_seed(101))
    hit = torch.empty(R, device="cuda", dtype=torch.int32)
    hv = torch.empty((R, 2), device="cuda")
    t = torch.empty((R, 80), device="cuda")
    x = torch.empty((R * 80, 3), device="cuda")
    f = torch.empty((R * 80, mu.shape[1]), device="cuda")
    g = torch.empty((R * 80, mu.shape[1], 3), device="cuda")

    def step():
        P.dps_ray_march(tree, od, dd, tnd, tfd, N_MARCH, BETA, EPS, hit_out=hit, values_out=hv)
        P.dps_ray_resample(od, dd, tnd, tfd, N_MARCH, hit, hv, u, tile_layout=True, t_out=t, x_out=x)
        P.dps_query(tree, x, BETA, EPS, f_out=f, g_out=g)

    def snapshot():
        torch.cuda.synchronize()
        return [to_host(v).copy() for v in (hit, hv, t, x, f, g)]

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step()
        ref = snapshot()
    torch.cuda.current_stream().wait_stream(side)
    assert 0 < int((ref[0] >= 0).sum()) < R
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step()
    for r in range(3):
        for v in (hv, t, x, f, g):
            v.fill_(float("nan"))
        hit.fill_(-7)
        torch.cuda.synchronize()
        graph.replay()
        got = snapshot()
        for a, b in zip(got, ref):
            assert np.array_equal(a, b), f"replay {r}"
        P.dps_query(tree, x[:4096], BETA, EPS)  # eager work between replays
    # the rays move (in place): the captured march follows them
    od.mul_(1.05)
    step()
    ref2 = snapshot()
    graph.replay()
    got = snapshot()
    for a, b in zip(got, ref2):
        assert np.array_equal(a, b), "replay after the rays moved"
    assert not np.array_equal(ref2[3], ref[3])
    P.dps_check(tree)


def test_march_edge_cases(P, orc):
    """Two march samples, zero-length rays (t_near = t_far: every sample at
    one point, no crossing) and a ray count that is not a multiple of 64,
    against the oracle's march."""
    from oracle import rays
    p, n, A, mu = workloads.winding_cloud(20000, 1000, 90)
    o, d, tn, tf = workloads.tile_camera_rays(workloads.sfm_camera(91), 16)
    R = 200
    o, d, tn, tf = o[:R].copy(), d[:R].copy(), tn[:R].copy(), tf[:R].copy()
    tf[::7] = tn[::7]
    tree = P.dps_build(*to_dev(p, n, A, mu), leaf_size=16)
    T = orc.Tree(p, n, A, mu, 16)
    od, dd, tnd, tfd = to_dev(o, d, tn, tf)
    for n_s in (2, 3, 97):
        print(f"[rays] edge cases: R={R} n={n_s}", flush=True)
        hit, hv = P.dps_ray_march(tree, od, dd, tnd, tfd, n_s, BETA, EPS)
        ref = rays.march(T, o, d, tn, tf, n_s, BETA, EPS)
        _check_march(to_host(hit), to_host(hv), ref, TOL_FP32)
        assert np.all(to_host(hit)[::7] == -1)
    P.dps_check(tree)


@pytest.mark.parametrize("storage", ["fp32", "bf16"])
@pytest.mark.parametrize("R,n_s", [(1024, 1024), (200, 97), (64, 40), (4096, 1024), (1, 2), (37, 128), (37, 129), (300, 255)])
def test_march_ray_major_equals_ray_per_lane(P, storage, R, n_s):
    """The ray-major march (a wavefront per chunk of one ray's samples) and
    the ray-per-lane march give the same crossing index and values bit for
    bit, for packets 1, 2 and 4."""
    import torch
    p, n, A, mu = workloads.winding_cloud(20000, 1000, 90)
    o, d, tn, tf = workloads.tile_camera_rays(workloads.sfm_camera(91), 64)
    sel = np.linspace(0, o.shape[0] - 1, R).astype(np.int64)  # spread over the view
    o, d, tn, tf = o[sel].copy(), d[sel].copy(), tn[sel].copy(), tf[sel].copy()
    tree = P.dps_build(*to_dev(p, n, A, mu), leaf_size=16, storage=storage)
    od, dd, tnd, tfd = to_dev(o, d, tn, tf)
    for k in (1, 2, 4):
        print(f"[rays] ray-major vs ray per lane: {storage} R={R} n={n_s} k={k}", flush=True)
        P.dps_set_launch(tree, k, 0, P.LAUNCH_PERSISTENT_QUERY)
        hs, vs = P.dps_ray_march(tree, od, dd, tnd, tfd, n_s, BETA, EPS)
        P.dps_set_launch(tree, k, 0, P.LAUNCH_PERSISTENT_QUERY | P.LAUNCH_MARCH_WHOLE)
        hw, vw = P.dps_ray_march(tree, od, dd, tnd, tfd, n_s, BETA, EPS)
        torch.cuda.synchronize()
        assert np.array_equal(to_host(hs), to_host(hw))
        assert np.array_equal(to_host(vs), to_host(vw))
        if R >= 200:
            assert int((hs >= 0).sum()) > 0
    P.dps_check(tree)


def test_march_crossing_values_without_workspace(P):
    """The march's crossing values come from the chunk that found the crossing
    when the tree's workspace is there; captured into a graph before any
    workspace exists, or under a memory limit that refuses it, the march
    evaluates them in a second pass: the same bits every way."""
    import torch
    p, n, A, mu = workloads.winding_cloud(20000, 1000, 90)
    o, d, tn, tf = workloads.tile_camera_rays(workloads.sfm_camera(91), 64)
    R = 1000
    o, d, tn, tf = o[:R].copy(), d[:R].copy(), tn[:R].copy(), tf[:R].copy()
    od, dd, tnd, tfd = to_dev(o, d, tn, tf)
    results = {}
    for k in (1, 2):
        # a fresh tree: the captured march has no workspace and takes the second pass
        tree = P.dps_build(*to_dev(p, n, A, mu), leaf_size=16)
        P.dps_set_launch(tree, k, 0, 0)
        bytes0 = P.dps_tree_info(tree)["bytes"]
        hit = torch.empty(R, device="cuda", dtype=torch.int32)
        hv = torch.empty((R, 2), device="cuda")
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            torch.cuda.synchronize()
            graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(graph):
                P.dps_ray_march(tree, od, dd, tnd, tfd, 300, BETA, EPS, hit_out=hit, values_out=hv)
        torch.cuda.current_stream().wait_stream(side)
        assert P.dps_tree_info(tree)["bytes"] == bytes0  # nothing allocated under capture
        hit.fill_(-7)
        hv.fill_(float("nan"))
        graph.replay()
        torch.cuda.synchronize()
        captured = (to_host(hit).copy(), to_host(hv).copy())
        # eager: allocates the workspace and gathers the values from it
        he, ve = P.dps_ray_march(tree, od, dd, tnd, tfd, 300, BETA, EPS)
        chunks = -(-(300 - 1) // (64 * k - 1))
        assert P.dps_tree_info(tree)["bytes"] == bytes0 + R * chunks * 8
        eager = (to_host(he).copy(), to_host(ve).copy())
        # captured with the workspace in place: the graph gathers from it
        with torch.cuda.stream(side):
            torch.cuda.synchronize()
            graph2 = torch.cuda.CUDAGraph()
            with torch.cuda.graph(graph2):
                P.dps_ray_march(tree, od, dd, tnd, tfd, 300, BETA, EPS, hit_out=hit, values_out=hv)
        torch.cuda.current_stream().wait_stream(side)
        # a larger march outgrows the workspace; both graphs keep working
        P.dps_ray_march(tree, od, dd, tnd, tfd, 1024, BETA, EPS)
        for gr in (graph, graph2):
            hit.fill_(-7)
            hv.fill_(float("nan"))
            gr.replay()
            torch.cuda.synchronize()
            assert np.array_equal(to_host(hit), eager[0]) and np.array_equal(to_host(hv), eager[1])
        assert np.array_equal(captured[0], eager[0]) and np.array_equal(captured[1], eager[1])
        assert 0 < int((eager[0] >= 0).sum()) < R
        P.dps_check(tree)
        P.dps_destroy(tree)
        # a memory limit that leaves no room for the workspace
        tree = P.dps_build(*to_dev(p, n, A, mu), leaf_size=16)
        P.dps_set_launch(tree, k, 0, 0)
        b = P.dps_tree_info(tree)["bytes"]
        P.dps_set_memory_limit(b + 64)
        try:
            hl, vl = P.dps_ray_march(tree, od, dd, tnd, tfd, 300, BETA, EPS)
            torch.cuda.synchronize()
            assert P.dps_tree_info(tree)["bytes"] == b
        finally:
            P.dps_set_memory_limit(0)
        assert np.array_equal(to_host(hl), eager[0]) and np.array_equal(to_host(vl), eager[1])
        P.dps_destroy(tree)
        results[k] = eager
    assert np.array_equal(results[1][0], results[2][0]) and np.array_equal(results[1][1], results[2][1])


@pytest.mark.parametrize("storage", ["fp32", "bf16"])
@pytest.mark.parametrize("cloud", ["winding", "sphere"])
def test_harnack_march_equals_the_dense_march(P, orc, storage, cloud):
    """The Harnack-accelerated march returns the dense march's crossing index
    and values bit for bit (same walk at the same FP32 positions) on every
    ray, matches the oracle's Harnack march (whose index equals the oracle's
    dense march) to the precision of the field, and evaluates the field far
    fewer times than the dense march needs."""
    from oracle import rays
    if cloud == "winding":
        p, n, A, mu = workloads.winding_cloud(20000, 1000, 90)
        o, d, tn, tf = workloads.tile_camera_rays(workloads.sfm_camera(91), 64)
        eps = EPS
    else:
        p, n, A = workloads.fibonacci_sphere(40000)
        mu = np.ones((p.shape[0], 1), np.float32)
        o, d, tn, tf = workloads.tile_camera_rays(workloads.sfm_camera(92), 32)
        eps = 0.05
    tree = P.dps_build(*to_dev(p, n, A, mu), leaf_size=16, storage=storage)
    od, dd, tnd, tfd = to_dev(o, d, tn, tf)
    R = o.shape[0]
    print(f"[rays] Harnack march {cloud} {storage} R={R}", flush=True)
    hit, hv = P.dps_ray_march(tree, od, dd, tnd, tfd, N_MARCH, BETA, eps)
    hh, vh, ev = P.dps_ray_march_harnack(tree, od, dd, tnd, tfd, N_MARCH, BETA, eps, lower=-0.25, want_evals=True)
    P.dps_check(tree)
    hit, hv, hh, vh, ev = (to_host(a) for a in (hit, hv, hh, vh, ev))
    assert np.array_equal(hh, hit), np.nonzero(hh != hit)
    assert np.array_equal(vh.view(np.int32), hv.view(np.int32))
    crossing = hit >= 0
    assert 0 < crossing.sum() < R
    needed = np.where(crossing, hit + 2, N_MARCH)
    print(f"[rays] {crossing.sum()} of {R} cross; evaluations {ev.mean():.1f} per ray (dense {needed.mean():.1f}), "
          f"max {ev.max()}", flush=True)
    assert np.all(ev >= 1) and ev.mean() < 0.5 * needed.mean()
    # the oracle's Harnack march on a subset of the rays
    sel = np.arange(0, R, max(1, R // 256))
    T = orc.Tree(p, n, A, mu, 16)
    ho = rays.harnack_march(T, p, o[sel], d[sel], tn[sel], tf[sel], N_MARCH, BETA, eps, level=0.5, lower=-0.25)
    ref = rays.march(T, o[sel], d[sel], tn[sel], tf[sel], N_MARCH, BETA, eps)
    assert np.array_equal(ho["j"], ref["j"])
    _check_march(hh[sel], vh[sel], ref, TOL_BF16 if storage == "bf16" else TOL_FP32)


def test_march_non_finite_rays(P, scene):
    """Rays with a NaN or infinite origin, direction or interval are not
    checked: they find no crossing (index -1, values 0), every other ray gets
    the same bits as in a batch without them, in the dense march (packets 1
    and 2) and in the Harnack march, and no device error is raised."""
    (p, n, A, mu), (o, d, tn, tf), _ = scene
    R = 256
    o, d, tn, tf = (np.ascontiguousarray(a[:R]).copy() for a in (o, d, tn, tf))
    ob, db, tnb, tfb = o.copy(), d.copy(), tn.copy(), tf.copy()
    ob[3] = np.nan
    db[70, 1] = np.inf
    tfb[129] = np.inf
    tnb[200] = np.nan
    bad = np.array([3, 70, 129, 200])
    good = np.setdiff1d(np.arange(R), bad)
    tree = P.dps_build(*to_dev(p, n, A, mu), leaf_size=16)
    clean = to_dev(*(np.ascontiguousarray(a[good]) for a in (o, d, tn, tf)))
    dirty = to_dev(ob, db, tnb, tfb)
    for k in (1, 2):
        P.dps_set_launch(tree, k, 0, -1)
        hit0, hv0 = (to_host(a) for a in P.dps_ray_march(tree, *clean, N_MARCH, BETA, EPS))
        hit, hv = (to_host(a) for a in P.dps_ray_march(tree, *dirty, N_MARCH, BETA, EPS))
        assert np.array_equal(hit[good], hit0), k
        assert np.array_equal(hv[good].view(np.int32), hv0.view(np.int32)), k
        assert np.all(hit[bad] == -1) and np.all(hv[bad] == 0.0), k
        assert 0 < np.sum(hit0 >= 0) < good.size
    hh, vh, _ = P.dps_ray_march_harnack(tree, *dirty, N_MARCH, BETA, EPS, lower=-0.25)
    assert np.array_equal(to_host(hh), hit)
    assert np.array_equal(to_host(vh).view(np.int32), hv.view(np.int32))
    P.dps_check(tree)


def _deep_scene(R=256, seed=5):
    """The deep-cluster cloud (a tree of 21 levels) with every normal pointing
    away from the cluster centre and unit geometry attributes, and R rays
    aimed at the centre with offsets of 2^-2 .. 2^-21, so that their samples
    walk the deepest levels and most of them cross the level set."""
    p, n, A, mu = workloads.deep_cluster_cloud(10, C=2)
    c = workloads.scenes.DEEP_CENTRE
    v = p - c
    n = (v / np.linalg.norm(v, axis=1, keepdims=True)).astype(np.float32)
    mu[:, 0] = 1.0
    rng = np.random.default_rng(seed)
    u = rng.standard_normal((R, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    off = rng.standard_normal((R, 3)) * (2.0 ** -rng.integers(2, 22, R))[:, None]
    o = (c - 1.5 * u).astype(np.float32)
    d = (c + off) - o
    d = (d / np.linalg.norm(d, axis=1, keepdims=True)).astype(np.float32)
    tn = np.full(R, 1.0, np.float32)
    tf = np.full(R, 2.0, np.float32)
    return (p, n, A, mu), (o, d, tn, tf)


def test_march_on_a_tree_of_21_levels(P, orc):
    """The dense march (packets 1, 2, 4) against the oracle's, and the
    Harnack-accelerated march against the dense one bit for bit, on rays
    through a cluster whose tree reaches its last level."""
    from oracle import rays
    (p, n, A, mu), (o, d, tn, tf) = _deep_scene()
    tree = P.dps_build(*to_dev(p, n, A, mu), leaf_size=16)
    assert P.dps_tree_info(tree)["depth"] == 21
    T = orc.Tree(p, n, A, mu, 16)
    ref = rays.march(T, o, d, tn, tf, 256, BETA, 0.05)
    od, dd, tnd, tfd = to_dev(o, d, tn, tf)
    for k in (1, 2, 4):
        P.dps_set_launch(tree, k, 0, -1)
        hit, hv = P.dps_ray_march(tree, od, dd, tnd, tfd, 256, BETA, 0.05)
        hits = _check_march(to_host(hit), to_host(hv), ref, TOL_FP32)
        assert hits > o.shape[0] // 2, (k, hits)
    hh, vh, _ = P.dps_ray_march_harnack(tree, od, dd, tnd, tfd, 256, BETA, 0.05, lower=-0.25)
    assert np.array_equal(to_host(hh), to_host(hit))
    assert np.array_equal(to_host(vh).view(np.int32), to_host(hv).view(np.int32))
    P.dps_check(tree)


def test_harnack_march_edge_cases(P):
    """Two samples, zero-length rays, a ray count that is not a multiple of
    64, a bound that is no bound at all (the march then falls back to single
    steps and still returns the dense march's crossing), no evaluation
    counts, and argument errors."""
    import torch
    p, n, A, mu = workloads.winding_cloud(20000, 1000, 90)
    o, d, tn, tf = workloads.tile_camera_rays(workloads.sfm_camera(91), 16)
    R = 200
    o, d, tn, tf = o[:R].copy(), d[:R].copy(), tn[:R].copy(), tf[:R].copy()
    tf[::7] = tn[::7]
    tree = P.dps_build(*to_dev(p, n, A, mu), leaf_size=16)
    od, dd, tnd, tfd = to_dev(o, d, tn, tf)
    for n_s, lower in ((2, -0.25), (3, -0.25), (97, -0.25), (300, -0.25), (300, 0.49), (300, -5.0)):
        print(f"[rays] Harnack edge case n={n_s} lower={lower}", flush=True)
        hit, hv = P.dps_ray_march(tree, od, dd, tnd, tfd, n_s, BETA, EPS)
        hh, vh, ev = P.dps_ray_march_harnack(tree, od, dd, tnd, tfd, n_s, BETA, EPS, lower=lower)
        assert ev is None
        hit, hv, hh, vh = (to_host(a) for a in (hit, hv, hh, vh))
        assert np.array_equal(hh, hit) and np.array_equal(vh.view(np.int32), hv.view(np.int32))
        assert np.all(hh[::7] == -1)
    P.dps_check(tree)
    x0 = torch.empty((0, 3), device="cuda")
    t0 = torch.empty(0, device="cuda")
    h0, v0, _ = P.dps_ray_march_harnack(tree, x0, x0, t0, t0, 64, BETA, EPS)
    assert h0.shape == (0,)
    for bad in (dict(lower=0.5), dict(lower=0.7), dict(lower=float("nan")), dict(n_samples=1), dict(channel=4)):
        kw = dict(n_samples=64, lower=-0.25)
        kw.update(bad)
        with pytest.raises(P.DpsError):
            P.dps_ray_march_harnack(tree, od, dd, tnd, tfd, kw["n_samples"], BETA, EPS, lower=kw["lower"],
                                    channel=kw.get("channel", 0))
