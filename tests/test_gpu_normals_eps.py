"""Derivatives in the point normals and in eps (both optimised by the
paper's inverse rendering, Sec. 5.2): ``dps_adjoint_accumulate_ext`` /
``dps_adjoint_finalize_ext`` and ``dps_set_normals`` against the FP64
oracle, and the autograd path against central differences of an oracle-
evaluated loss built from the values and gradients."""
import math

import numpy as np
import pytest

import workloads
from parity import TOL_BF16, TOL_FP32, norm_err, to_dev, to_host
from test_gpu_gradcot import _density_loss_numpy, _density_loss_torch, _random_cloud

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    import paper_2405_16788_amd as lib
    lib.load()
    assert torch.cuda.is_available()
    return lib


CLOUDS = {
    "sphere-8k": lambda: workloads.sphere_cloud(8192, 1),
    "random-3001-c5": lambda: _random_cloud(3001, 8, C=5),
    "sfm-20k": lambda: workloads.sfm_cloud(20000, 1000, 10),
}


@pytest.mark.parametrize("storage", ["fp32", "bf16"])
@pytest.mark.parametrize("name", list(CLOUDS))
def test_normals_eps_parity(P, orc, name, storage):
    p, n, A, mu = CLOUDS[name]()
    Q, C = 3000, mu.shape[1]
    x = workloads.sphere_queries(Q, 51, half=1.2)
    df = workloads.cotangents(Q, C, 52)
    dg = np.random.default_rng(53).standard_normal((Q, C, 3)).astype(np.float32)
    tree = P.dps_build(*to_dev(p, n, A, mu), leaf_size=16, storage=storage)
    T = orc.Tree(p, n, A, mu, 16)
    xd, dfd, dgd = to_dev(x, df, dg)
    tol = TOL_BF16 if storage == "bf16" else TOL_FP32
    for eps in (0.05, 0.0):
        for use_df, use_dg in ((True, True), (True, False), (False, True)):
            print(f"[normals-eps] {name} {storage} eps={eps} df={use_df} dg={use_dg}", flush=True)
            P.dps_adjoint_zero(tree)
            dx = P.dps_adjoint_accumulate_ext(tree, xd, 2.0, eps, df=dfd if use_df else None,
                                              dg=dgd if use_dg else None, want=P.WANT_NORMALS | P.WANT_EPS)
            da, dn, de = P.dps_adjoint_finalize_ext(tree, attrs=True, normals=True, eps=True)
            ref = T.adjoint(x, 2.0, eps, df if use_df else None, dg=dg if use_dg else None, extra=True)
            assert norm_err(to_host(da), ref["dmu"], ref["sdmu"] + 1e-30) <= TOL_FP32
            assert norm_err(to_host(dx), ref["dx"], ref["sdx"][:, None] + 1e-30) <= tol
            # dL/dn uses the stored attributes: the storage bound
            assert norm_err(to_host(dn), ref["dn"], ref["sdn"][:, None] + 1e-30) <= tol
            got = float(to_host(de)[0])
            assert abs(got - ref["deps"]) <= tol * ref["sdeps"] + 1e-30, (got, ref["deps"], ref["sdeps"])
            if eps == 0.0:
                assert got == 0.0
    P.dps_check(tree)


def test_set_normals(P, orc):
    p, n, A, mu = workloads.sfm_cloud(20000, 1000, 11)
    rng = np.random.default_rng(54)
    n2 = n + 0.3 * rng.standard_normal(n.shape).astype(np.float32)
    n2 = (n2 / np.linalg.norm(n2, axis=1, keepdims=True)).astype(np.float32)
    x = workloads.sphere_queries(4000, 55, half=1.2)
    df = workloads.cotangents(4000, mu.shape[1], 56)
    pd, nd, Ad, mud, n2d, xd, dfd = to_dev(p, n, A, mu, n2, x, df)
    tree = P.dps_build(pd, nd, Ad, mud, leaf_size=16)
    before = {k: to_host(v).copy() for k, v in P.dps_export_tree(tree).items()}
    P.dps_set_normals(tree, n2d)
    P.dps_set_attributes(tree, mud)
    after = {k: to_host(v) for k, v in P.dps_export_tree(tree).items()}
    # normals do not enter the tree geometry
    for k in ("codes", "perm", "nodes", "geom"):
        assert np.array_equal(before[k], after[k]), k
    T2 = orc.Tree(p, n2, A, mu, 16)
    oe = T2.export()
    assert np.array_equal(after["nodes"], oe["nodes"])
    f, g = P.dps_query(tree, xd, 2.0, 0.05)
    ref = T2.query(x, 2.0, 0.05)
    assert norm_err(to_host(f), ref["f"], ref["sf"]) <= TOL_FP32
    assert norm_err(to_host(g), ref["g"], ref["sg"]) <= TOL_FP32
    P.dps_adjoint_zero(tree)
    P.dps_adjoint_accumulate_ext(tree, xd, 2.0, 0.05, df=dfd, want=P.WANT_NORMALS, want_dx=False)
    da, dn, _ = P.dps_adjoint_finalize_ext(tree, attrs=True, normals=True)
    a = T2.adjoint(x, 2.0, 0.05, df, extra=True)
    assert norm_err(to_host(da), a["dmu"], a["sdmu"] + 1e-30) <= TOL_FP32
    assert norm_err(to_host(dn), a["dn"], a["sdn"][:, None] + 1e-30) <= TOL_FP32
    with pytest.raises(P.DpsError):
        P.dps_adjoint_accumulate_ext(tree, xd, 2.0, 0.05, df=dfd, want=4)
    with pytest.raises(P.DpsError):
        P.dps_adjoint_accumulate_ext(tree, xd, 2.0, 0.05)
    P.dps_check(tree)


def test_autograd_normals_and_eps_match_fd(P, orc):
    """The density loss of the gradient-cotangent test, differentiated w.r.t.
    the normals (a random direction field; the sums are linear in the
    normals, so the oracle's response to the direction field gives exact
    perturbed values) and w.r.t. eps (Richardson differences with the
    oracle at eps +- h; the far decisions do not depend on eps)."""
    import torch
    p, n, A, mu = workloads.winding_cloud(40000, 2000, 80)
    eye = workloads.sfm_camera(81)
    n_rays, S = 128, 64
    o, d, t0, t1 = workloads.camera_rays(eye, 64, 64)
    pix, x = workloads.pixel_ray_samples(eye, 64, 64, S, 82, n_rays, 83)
    omega = d.reshape(-1, 3)[pix]
    dt = ((t1 - t0) / S).reshape(-1)[pix]
    target = np.random.default_rng(84).uniform(size=(n_rays, 3))
    beta, eps0 = 2.0, 0.02
    tree = P.dps_build(*to_dev(p, n, A, mu), leaf_size=16)
    attrs = to_dev(mu)[0]
    normals = to_dev(n)[0].requires_grad_(True)
    eps_t = torch.tensor(eps0, dtype=torch.float64, requires_grad=True)
    xt = to_dev(x)[0]
    om_t, dt_t, tg_t = (torch.tensor(a, dtype=torch.float32, device="cuda") for a in (omega, dt, target))
    f, g = P.dipole_sum(attrs, xt, tree, beta, eps_t, normals=normals)
    loss = torch.sum(_density_loss_torch(f, g, om_t, dt_t, tg_t, n_rays, S))
    dn, de = torch.autograd.grad(loss, [normals, eps_t])
    dn, de = to_host(dn).astype(np.float64), float(de)

    def L(ff, gg):
        return _density_loss_numpy(ff, gg, omega, dt, target, n_rays, S)

    base = orc.Tree(p, n, A, mu, 16).query(x, beta, eps0)
    # normals: the response to a direction field e is the sum with normals e
    e = np.random.default_rng(85).standard_normal(n.shape).astype(np.float32)
    re_ = orc.Tree(p, e, A, mu, 16).query(x, beta, eps0)
    h = 1e-4 / max(np.abs(re_["f"]).max(), 1e-30)
    cd = {s: (L(base["f"] + s * re_["f"], base["g"] + s * re_["g"]) -
              L(base["f"] - s * re_["f"], base["g"] - s * re_["g"])) / (2 * s) for s in (h, h / 2)}
    per_ray = (4 * cd[h / 2] - cd[h]) / 3
    got = float(np.sum(dn * e))
    print(f"[normals-eps] dL/dn . e: gpu {got:.9g} fd {np.sum(per_ray):.9g}", flush=True)
    assert abs(got - np.sum(per_ray)) <= 2e-4 * np.sum(np.abs(per_ray)) + 1e-9
    # eps
    T = orc.Tree(p, n, A, mu, 16)
    hs = {}
    for s in (2e-4, 1e-4):
        rp, rm = T.query(x, beta, eps0 + s), T.query(x, beta, eps0 - s)
        hs[s] = (L(rp["f"], rp["g"]) - L(rm["f"], rm["g"])) / (2 * s)
    per_ray = (4 * hs[1e-4] - hs[2e-4]) / 3
    print(f"[normals-eps] dL/deps: gpu {de:.9g} fd {np.sum(per_ray):.9g}", flush=True)
    assert abs(de - np.sum(per_ray)) <= 1e-3 * np.sum(np.abs(per_ray)) + 1e-9
    P.dps_check(tree)
