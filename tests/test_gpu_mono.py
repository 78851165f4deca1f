"""Monopole-kernel trees (appearance attributes summed with the foreshortening
factor of the kernel dropped, Sec. 7.1): queries, adjoints, channel subsets,
device row counts and the moment export against the FP64 oracle's monopole
tree (same far decisions, FP64 arithmetic), the transpose identity at full
size, and the entry points a monopole tree rejects."""
import math

import numpy as np
import pytest

import workloads
from parity import TOL_BF16, TOL_FP32, norm_err, to_dev, to_host

pytestmark = pytest.mark.gpu

BETA = 2.0


@pytest.fixture(scope="module")
def P():
    import torch
    import paper_2405_16788_amd as lib
    lib.load()
    assert torch.cuda.is_available()
    return lib


def _dup_cloud(M, C, seed):
    """Random cloud in [-1,1]^3 in which every 7th point repeats an earlier
    one (coincident sources), with appearance attributes."""
    rng = np.random.default_rng(seed)
    p = rng.uniform(-1.0, 1.0, size=(M, 3)).astype(np.float32)
    p[7::7] = p[: len(p[7::7])]
    n = rng.standard_normal((M, 3))
    n = (n / np.linalg.norm(n, axis=1, keepdims=True)).astype(np.float32)
    A = rng.uniform(0.5, 2.0, size=M).astype(np.float32) * np.float32(4.0 / M)
    return p, n, A, workloads.appearance_attrs(M, C, seed + 1)


CLOUDS = {
    "sphere-8k-c5": lambda: (*workloads.sphere_cloud(8192, 1)[:3], workloads.appearance_attrs(8192, 5, 60)),
    "sfm-20k-c32": lambda: (*workloads.sfm_cloud(20000, 1000, 10)[:3], workloads.appearance_attrs(21000, 32, 61)),
    "dup-3001-c3": lambda: _dup_cloud(3001, 3, 62),
}


def _queries(p, Q, seed):
    """Queries in the cloud's box, the first 64 of them exactly at source
    points (coincident query and source: no contribution)."""
    x = workloads.sphere_queries(Q, seed, half=1.2)
    x[:64] = p[np.random.default_rng(seed + 1).choice(p.shape[0], 64, replace=False)]
    return x


def _tol(storage):
    return TOL_BF16 if storage == "bf16" else TOL_FP32


@pytest.mark.parametrize("storage", ["fp32", "bf16"])
@pytest.mark.parametrize("name", list(CLOUDS))
def test_mono_query_parity(P, orc, name, storage):
    p, n, A, mu = CLOUDS[name]()
    x = _queries(p, 2500, 63)
    tree = P.dps_build(*to_dev(p, n, A, mu), leaf_size=16, storage=storage, kernel="monopole")
    assert P.dps_get_kernel(tree) == "monopole"
    T = orc.Tree(p, n, A, mu, 16, kind="monopole")
    (xd,) = to_dev(x)
    for eps in (0.05, 0.0):
        ref = T.query(x, BETA, eps)
        assert np.all(np.isfinite(ref["f"]))
        for k, flags in ((1, 0), (2, P.LAUNCH_XCD_QUERY), (4, P.LAUNCH_PERSISTENT_QUERY)):
            print(f"[mono] query {name} {storage} eps={eps} k={k} flags={flags}", flush=True)
            P.dps_set_launch(tree, k, 0, flags)
            f, g = P.dps_query(tree, xd, BETA, eps)
            f0, _ = P.dps_query(tree, xd, BETA, eps, grad=False)
            assert norm_err(to_host(f), ref["f"], ref["sf"]) <= _tol(storage)
            assert norm_err(to_host(g), ref["g"], ref["sg"]) <= _tol(storage)
            assert norm_err(to_host(f0), ref["f"], ref["sf"]) <= _tol(storage)
    # the traversal decisions are those of the dipole tree
    c = to_host(P.dps_query_counts(tree, xd, BETA))
    assert np.array_equal(c, T.query(x, BETA, 0.05)["counts"])
    P.dps_check(tree)


def test_mono_coincident_sources_contribute_nothing(P, orc):
    """Queries at the position of every source of a small cloud with repeated
    points, at eps = 0 (the kernel is singular there): with beta so large that
    only zero-radius nodes (single or coincident points, exact as monopoles)
    are far, the sums are the oracle's direct sums, which skip every source
    at the query point."""
    p, n, A, mu = _dup_cloud(257, 4, 64)
    tree = P.dps_build(*to_dev(p, n, A, mu), leaf_size=8, kernel="monopole")
    (xd,) = to_dev(p)
    f, g = P.dps_query(tree, xd, 1e6, 0.0)
    ref = orc.direct_mono(p, A, mu, p, 0.0)
    fh, gh = to_host(f), to_host(g)
    assert np.all(np.isfinite(fh)) and np.all(np.isfinite(gh))
    assert norm_err(fh, ref["f"], ref["sf"]) <= TOL_FP32
    assert norm_err(gh, ref["g"], ref["sg"]) <= TOL_FP32


@pytest.mark.parametrize("storage", ["fp32", "bf16"])
@pytest.mark.parametrize("name", list(CLOUDS))
def test_mono_adjoint_parity(P, orc, name, storage):
    p, n, A, mu = CLOUDS[name]()
    C = mu.shape[1]
    x = _queries(p, 2500, 65)
    df = workloads.cotangents(x.shape[0], C, 66)
    tree = P.dps_build(*to_dev(p, n, A, mu), leaf_size=16, storage=storage, kernel="monopole")
    T = orc.Tree(p, n, A, mu, 16, kind="monopole")
    xd, dfd = to_dev(x, df)
    for eps in (0.05, 0.0):
        ref = T.adjoint(x, BETA, eps, df)
        for k, flags in ((1, 0), (2, P.LAUNCH_XCD_ADJOINT), (4, P.LAUNCH_PERSISTENT_ADJOINT)):
            print(f"[mono] adjoint {name} {storage} eps={eps} k={k} flags={flags}", flush=True)
            P.dps_set_launch(tree, 0, k, flags)
            da, dx = P.dps_adjoint(tree, xd, BETA, eps, dfd)
            # dL/dmu involves only geometry and df: FP32 bound for both storages
            assert norm_err(to_host(da), ref["dmu"], ref["sdmu"] + 1e-30) <= TOL_FP32
            assert norm_err(to_host(dx), ref["dx"], ref["sdx"][:, None] + 1e-30) <= _tol(storage)
    P.dps_check(tree)


def test_mono_tree_of_21_levels(P, orc):
    """Monopole query and adjoint on a tree that reaches its last level, with
    queries at every scale around the deep cluster and at its points (FP32
    storage), in each packet size."""
    p, n, A, mu = workloads.deep_cluster_cloud(10, C=5)
    x = np.concatenate([workloads.sphere_queries(1000, 67, half=1.2), workloads.deep_cluster_probes(p, 68)])
    df = workloads.cotangents(x.shape[0], mu.shape[1], 69)
    tree = P.dps_build(*to_dev(p, n, A, mu), leaf_size=16, kernel="monopole")
    assert P.dps_tree_info(tree)["depth"] == 21
    T = orc.Tree(p, n, A, mu, 16, kind="monopole")
    xd, dfd = to_dev(x, df)
    for eps in (0.05, 0.0):
        ref = T.query(x, BETA, eps)
        adj = T.adjoint(x, BETA, eps, df)
        for k in (1, 2, 4):
            P.dps_set_launch(tree, k, k, P.LAUNCH_PERSISTENT_QUERY | P.LAUNCH_PERSISTENT_ADJOINT)
            f, g = P.dps_query(tree, xd, BETA, eps)
            assert norm_err(to_host(f), ref["f"], ref["sf"]) <= TOL_FP32, (eps, k)
            assert norm_err(to_host(g), ref["g"], ref["sg"]) <= TOL_FP32, (eps, k)
            da, dx = P.dps_adjoint(tree, xd, BETA, eps, dfd)
            assert norm_err(to_host(da), adj["dmu"], adj["sdmu"] + 1e-30) <= TOL_FP32, (eps, k)
            assert norm_err(to_host(dx), adj["dx"], adj["sdx"][:, None] + 1e-30) <= TOL_FP32, (eps, k)
    assert np.array_equal(to_host(P.dps_query_counts(tree, xd, BETA)), T.query(x, BETA, 0.05)["counts"])
    P.dps_check(tree)


@pytest.mark.parametrize("storage", ["fp32", "bf16"])
def test_mono_channel_subsets_and_row_counts(P, orc, storage):
    p, n, A, mu = CLOUDS["sfm-20k-c32"]()
    x = _queries(p, 3001, 67)
    Q, C = x.shape[0], mu.shape[1]
    df = workloads.cotangents(Q, C, 68)
    tree = P.dps_build(*to_dev(p, n, A, mu), leaf_size=16, storage=storage, kernel="monopole")
    T = orc.Tree(p, n, A, mu, 16, kind="monopole")
    ref = T.query(x, BETA, 0.03)
    xd, dfd = to_dev(x, df)
    import torch
    for c0, nc in ((0, 32), (2, 7), (16, 16), (30, 2), (4, 1)):
        print(f"[mono] channels [{c0}, {c0 + nc}) {storage}", flush=True)
        sl = slice(c0, c0 + nc)
        f, g = P.dps_query_channels(tree, xd, BETA, 0.03, c0, nc)
        assert norm_err(to_host(f), ref["f"][:, sl], ref["sf"][:, sl]) <= _tol(storage)
        assert norm_err(to_host(g), ref["g"][:, sl], ref["sg"][:, sl]) <= _tol(storage)
        # a device row count: rows past it stay untouched
        qc = torch.tensor([1234], dtype=torch.int64, device="cuda")
        fo = torch.full((Q, nc), 7.0, device="cuda")
        P.dps_query_channels(tree, xd, BETA, 0.03, c0, nc, grad=False, f_out=fo, q_count=qc)
        fo = to_host(fo)
        assert np.all(fo[1234:] == 7.0)
        assert norm_err(fo[:1234], ref["f"][:1234, sl], ref["sf"][:1234, sl]) <= _tol(storage)
        # adjoint of the subset: equal to the full adjoint with df zero elsewhere
        dfs = np.zeros_like(df)
        dfs[:1234, sl] = df[:1234, sl]
        a = T.adjoint(x, BETA, 0.03, dfs)
        P.dps_adjoint_zero(tree)
        dx = torch.full((Q, 3), 5.0, device="cuda")
        P.dps_adjoint_accumulate_channels(tree, xd, BETA, 0.03, c0, nc, dfd[:, sl].contiguous(), dx_out=dx,
                                          q_count=qc)
        da = to_host(P.dps_adjoint_finalize(tree))
        dx = to_host(dx)
        assert np.all(dx[1234:] == 5.0)
        assert norm_err(da, a["dmu"], a["sdmu"] + 1e-30) <= TOL_FP32
        assert norm_err(dx[:1234], a["dx"][:1234], a["sdx"][:1234, None] + 1e-30) <= _tol(storage)
    with pytest.raises(P.DpsError):
        P.dps_query_channels(tree, xd, BETA, 0.03, 30, 3)
    P.dps_check(tree)


def test_mono_export_refit_and_rejections(P, orc):
    import torch
    p, n, A, mu = CLOUDS["sphere-8k-c5"]()
    pd, nd, Ad, mud = to_dev(p, n, A, mu)
    tree = P.dps_build(pd, nd, Ad, mud, leaf_size=16, kernel="monopole")
    T = orc.Tree(p, n, A, mu, 16, kind="monopole")
    oe = T.export()
    ex = P.dps_export_tree(tree)
    assert np.array_equal(to_host(ex["nodes"]), oe["nodes"])
    assert np.array_equal(to_host(ex["geom"]).view(np.int32), oe["geom"].view(np.int32))
    mom = to_host(ex["moments"]).astype(np.float64)
    assert np.all(mom[:, :, 1:] == 0.0) and np.all(oe["D"][:, :, 1:] == 0.0)
    # charge scale: sum over the node's points of A |mu|
    perm, nodes = oe["perm"].astype(np.int64), oe["nodes"]
    w = A.astype(np.float64)[perm][:, None] * np.abs(mu.astype(np.float64)[perm])
    cs = np.concatenate([np.zeros((1, w.shape[1])), np.cumsum(w, axis=0)])
    b = nodes[:, 4].astype(np.int64)
    sc = cs[b + nodes[:, 5]] - cs[b]
    assert np.max(np.abs(mom[:, :, 0] - oe["D"][:, :, 0]) / (sc + 1e-30)) <= 1e-5
    # a refit with new attributes follows the oracle's refit
    mu2 = workloads.appearance_attrs(mu.shape[0], mu.shape[1], 69)
    P.dps_set_attributes(tree, to_dev(mu2)[0])
    T.set_attrs(mu2)
    x = _queries(p, 1000, 70)
    (xd,) = to_dev(x)
    ref = T.query(x, BETA, 0.05)
    f, _ = P.dps_query(tree, xd, BETA, 0.05)
    assert norm_err(to_host(f), ref["f"], ref["sf"]) <= TOL_FP32
    # entry points defined for the dipole kernel only
    Q = x.shape[0]
    dg = torch.zeros((Q, 5, 3), device="cuda")
    df = torch.zeros((Q, 5), device="cuda")
    with pytest.raises(P.DpsError):
        P.dps_adjoint_accumulate_grad(tree, xd, BETA, 0.05, dg)
    with pytest.raises(P.DpsError):
        P.dps_adjoint_accumulate_ext(tree, xd, BETA, 0.05, df=df)
    with pytest.raises(P.DpsError):
        P.dps_set_normals(tree, nd)
    with pytest.raises(P.DpsError):
        P.dps_query_grid(tree, (0, 0, 0), (0.1, 0.1, 0.1), (4, 4, 4), BETA, 0.05)
    with pytest.raises(P.DpsError):
        P.dps_adjoint_finalize_ext(tree, attrs=True, normals=True)
    da, _, _ = P.dps_adjoint_finalize_ext(tree, attrs=True)
    assert da.shape == (p.shape[0], 5)
    with pytest.raises(ValueError):
        P.dps_build(pd, nd, Ad, mud, kernel="quadrupole")
    P.dps_check(tree)


def test_mono_autograd(P, orc):
    """dipole_sum on a monopole tree: dL/dattrs and dL/dx of L = sum w . f
    against the oracle adjoint with df = w; the gradient output is returned
    but cannot carry cotangents."""
    import torch
    p, n, A, mu = CLOUDS["sfm-20k-c32"]()
    x = _queries(p, 2000, 71)
    w = workloads.cotangents(x.shape[0], mu.shape[1], 72)
    tree = P.dps_build(*to_dev(p, n, A, mu), leaf_size=16, kernel="monopole")
    attrs = to_dev(mu)[0].requires_grad_(True)
    xt = to_dev(x)[0].requires_grad_(True)
    (wt,) = to_dev(w)
    f, g = P.dipole_sum(attrs, xt, tree, BETA, 0.02)
    torch.sum(wt * f).backward()
    ref = orc.Tree(p, n, A, mu, 16, kind="monopole").adjoint(x, BETA, 0.02, w)
    assert norm_err(to_host(attrs.grad), ref["dmu"], ref["sdmu"] + 1e-30) <= TOL_FP32
    assert norm_err(to_host(xt.grad), ref["dx"], ref["sdx"][:, None] + 1e-30) <= TOL_FP32
    f, g = P.dipole_sum(attrs, xt, tree, BETA, 0.02)
    with pytest.raises(RuntimeError):
        torch.sum(g).backward()
    eps_t = torch.tensor(0.02, dtype=torch.float64, requires_grad=True)
    with pytest.raises(ValueError):
        P.dipole_sum(attrs, xt, tree, BETA, eps_t)
    P.dps_check(tree)


def test_mono_sfm_1m_c32_full_size(P, orc):
    """The appearance sums at the benchmark's full size: sfm-1m (1,000,000
    points) with K = 32 appearance attributes, 512 x 512 rays x 128 samples
    (33,554,432 queries) in one call, values on a seeded sample against the
    oracle, and the full-size adjoint through the transpose identity
    sum df . f = sum dattrs . mu (f is linear in the attributes) and dL/dx on
    sampled queries."""
    import torch
    eps = math.sqrt(2.0) * 0.01
    p, n, A, _ = workloads.sfm_cloud(workloads.SFM_1M_SURFACE, workloads.SFM_1M_OUTLIERS, 10)
    mu = workloads.appearance_attrs(p.shape[0], 32, 73)
    x = workloads.ray_samples(workloads.sfm_camera(11), 512, 512, 128, 12, order="tile")
    Q = x.shape[0]
    pd, nd, Ad, mud, xd = to_dev(p, n, A, mu, x)
    print(f"[mono] build sfm-1m C=32, Q={Q}", flush=True)
    tree = P.dps_build(pd, nd, Ad, mud, leaf_size=16, kernel="monopole")
    T = orc.Tree(p, n, A, mu, 16, kind="monopole")
    f, _ = P.dps_query(tree, xd, BETA, eps, grad=False)
    P.dps_check(tree)
    idx = np.sort(np.random.default_rng(74).choice(Q, 3000, replace=False))
    it = torch.from_numpy(idx).cuda()
    ref = T.query(x[idx], BETA, eps)
    e = norm_err(to_host(f[it]), ref["f"], ref["sf"])
    print(f"[mono] sampled value error {e:.3g}", flush=True)
    assert e <= TOL_FP32
    assert torch.isfinite(f).all()
    del x
    print("[mono] full-size adjoint", flush=True)
    dfd = torch.empty((Q, 32), device="cuda")
    gen = torch.Generator(device="cuda")
    gen.manual_seed(75)
    dfd.normal_(generator=gen)
    da, dx = P.dps_adjoint(tree, xd, BETA, eps, dfd)
    P.dps_check(tree)
    lhs = torch.sum(dfd.double() * f.double(), dim=0)
    rhs = torch.sum(da.double() * mud.double(), dim=0)
    scale = torch.sum((dfd.double() * f.double()).abs(), dim=0)
    rel = ((lhs - rhs).abs() / scale).max().item()
    print(f"[mono] transpose identity, relative to sum |df f|: {rel:.3g}", flush=True)
    assert rel < 1e-4
    dfs = to_host(dfd[it]).astype(np.float32)
    a = T.adjoint(to_host(xd[it]), BETA, eps, dfs)
    e = norm_err(to_host(dx[it]), a["dx"], a["sdx"][:, None] + 1e-30)
    print(f"[mono] sampled dx error {e:.3g}", flush=True)
    assert e <= TOL_FP32
    P.dps_destroy(tree)
