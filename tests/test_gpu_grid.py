"""Grid queries for mesh extraction (marching cubes on the geometry field):
``dps_query_grid`` against the FP64 oracle at the same FP32 grid points, and
bit-identical to ``dps_query`` at those points (the per-query arithmetic does
not depend on how queries are packed into wavefronts)."""
import numpy as np
import pytest

import workloads
from parity import TOL_BF16, TOL_FP32, norm_err, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    import paper_2405_16788_amd as lib
    lib.load()
    assert torch.cuda.is_available()
    return lib


def grid_points(origin, spacing, dims):
    """FP32 coordinates o + (float)i * h (one rounding per operation), [nz,ny,nx,3]."""
    o = np.asarray(origin, np.float32)
    h = np.asarray(spacing, np.float32)
    axes = [o[a] + np.arange(dims[a], dtype=np.float32) * h[a] for a in range(3)]
    z, y, x = np.meshgrid(axes[2], axes[1], axes[0], indexing="ij")
    return np.stack([x, y, z], axis=-1).astype(np.float32)


@pytest.mark.parametrize("storage", ["fp32", "bf16"])
@pytest.mark.parametrize("k,dims", [(1, (37, 23, 19)), (2, (16, 16, 16)), (4, (5, 41, 7)), (2, (1, 1, 1))])
def test_grid_matches_oracle_and_point_queries(P, orc, storage, k, dims):
    p, n, A, mu = workloads.sfm_cloud(30000, 1500, 10)
    origin, spacing = (-1.2, -1.1, -1.0), (2.4 / 36, 2.2 / 22, 2.0 / 18)
    tree = P.dps_build(*to_dev(p, n, A, mu), leaf_size=16, storage=storage)
    P.dps_set_launch(tree, k, 0, -1)
    f, g = P.dps_query_grid(tree, origin, spacing, dims, 2.0, 0.02, grad=True)
    pts = grid_points(origin, spacing, dims)
    xs = pts.reshape(-1, 3)
    ref = orc.Tree(p, n, A, mu, 16).query(xs, 2.0, 0.02)
    tol = TOL_BF16 if storage == "bf16" else TOL_FP32
    fh, gh = to_host(f).reshape(-1, mu.shape[1]), to_host(g).reshape(-1, mu.shape[1], 3)
    assert norm_err(fh, ref["f"], ref["sf"]) <= tol
    assert norm_err(gh, ref["g"], ref["sg"]) <= tol
    xd = to_dev(xs)[0]
    fq, gq = P.dps_query(tree, xd, 2.0, 0.02)
    assert np.array_equal(fh, to_host(fq)) and np.array_equal(gh, to_host(gq))
    # a channel subset without gradients (the marching-cubes call): bitwise
    # equal to the point query of the same kernel variant
    f0, g0 = P.dps_query_grid(tree, origin, spacing, dims, 2.0, 0.02, c_begin=0, n_channels=1)
    assert g0 is None
    fq0, _ = P.dps_query_channels(tree, xd, 2.0, 0.02, 0, 1, grad=False)
    assert np.array_equal(to_host(f0).reshape(-1), to_host(fq0)[:, 0])
    assert norm_err(to_host(f0).reshape(-1), ref["f"][:, 0], ref["sf"][:, 0]) <= tol
    P.dps_check(tree)


def test_grid_rejects_bad_arguments(P):
    # the C entry point validates before any device work (a small output
    # buffer stands in; it is never written)
    import ctypes as ct
    import torch
    p, n, A, mu = workloads.sphere_cloud(512, 1)
    tree = P.dps_build(*to_dev(p, n, A, mu), leaf_size=16)
    buf = torch.zeros(64, device="cuda")
    lib = P.load()

    def call(origin, spacing, dims):
        o = (ct.c_float * 3)(*origin)
        h = (ct.c_float * 3)(*spacing)
        d = (ct.c_int64 * 3)(*dims)
        return lib.dps_query_grid(tree.handle, ct.cast(o, ct.c_void_p), ct.cast(h, ct.c_void_p),
                                  ct.cast(d, ct.c_void_p), 2.0, 0.05, 0, 1, ct.c_void_p(buf.data_ptr()), None, None)

    for dims in ((0, 4, 4), (4, -1, 4), (1 << 25, 1, 1), (1 << 14, 1 << 14, 1 << 14)):
        assert call((0, 0, 0), (0.1, 0.1, 0.1), dims) == 1
    assert call((0, float("nan"), 0), (0.1, 0.1, 0.1), (4, 4, 4)) == 1
    assert call((0, 0, 0), (0.1, float("inf"), 0.1), (4, 4, 4)) == 1
    torch.cuda.synchronize()
    assert not torch.any(buf != 0)
    P.dps_check(tree)


def test_grid_256_sfm_1m_sampled(P, orc):
    """A 256^3 grid over the sfm-1m cloud's bounding cube (16.8M points, the
    geometry channel only), sampled points against the oracle and bitwise
    against point queries."""
    import torch
    p, n, A, mu = workloads.sfm_cloud(workloads.SFM_1M_SURFACE, workloads.SFM_1M_OUTLIERS, 10)
    mu[:, 0] = 1.0
    tree = P.dps_build(*to_dev(p, n, A, mu), leaf_size=16)
    dims = (256, 256, 256)
    origin, spacing = (-1.05, -1.05, -1.05), (2.1 / 255,) * 3
    f, _ = P.dps_query_grid(tree, origin, spacing, dims, 2.0, 0.01414, c_begin=0, n_channels=1)
    torch.cuda.synchronize()
    rng = np.random.default_rng(90)
    idx = rng.integers(0, 256, size=(4096, 3))
    o, h = np.asarray(origin, np.float32), np.asarray(spacing, np.float32)
    xs = (o[None, :] + idx.astype(np.float32) * h[None, :]).astype(np.float32)
    got = to_host(f)[idx[:, 2], idx[:, 1], idx[:, 0], 0]
    ref = orc.Tree(p, n, A, mu, 16).query(xs, 2.0, 0.01414)
    assert norm_err(got, ref["f"][:, 0], ref["sf"][:, 0]) <= TOL_FP32
    fq, _ = P.dps_query_channels(tree, to_dev(xs)[0], 2.0, 0.01414, 0, 1, grad=False)
    assert np.array_equal(got, to_host(fq)[:, 0])
    # the field is a winding number: ~1 inside the shapes, ~0 far outside
    fh = to_host(f)[..., 0]
    assert 0.01 < np.mean(fh > 0.5) < 0.5 and abs(float(fh[0, 0, 0])) < 0.05
    P.dps_check(tree)
