"""Cotangents of the spatial gradient (dL/d grad D): the Hessian adjoint
``dps_adjoint_accumulate_grad`` against the FP64 oracle, and the autograd
path of a loss built from grad D -- a volume-rendering proxy with the paper's
surface density |w . grad v| / v (Sec. 3.1, eq. surface_density) -- against
central differences of the same loss evaluated with the oracle."""
import math

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


def _random_cloud(M, seed, C=4):
    rng = np.random.default_rng(seed)
    p = rng.uniform(-1, 1, size=(M, 3))
    n = rng.standard_normal((M, 3))
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    A = rng.uniform(0.5, 1.5, size=M) * (4.0 / max(M, 1))
    mu = rng.standard_normal((M, C))
    return p.astype(np.float32), n.astype(np.float32), A.astype(np.float32), mu.astype(np.float32)


CLOUDS = {
    "sphere-8k": lambda: workloads.sphere_cloud(8192, 1),
    "random-3001-c5": lambda: _random_cloud(3001, 8, C=5),
    "random-2000-c1": lambda: _random_cloud(2000, 9, C=1),
}


def _tol(storage):
    return TOL_BF16 if storage == "bf16" else TOL_FP32


@pytest.mark.parametrize("storage", ["fp32", "bf16"])
@pytest.mark.parametrize("eps", [0.05, 0.0])
@pytest.mark.parametrize("name", list(CLOUDS))
def test_grad_cotangent_parity(P, orc, name, eps, storage):
    import torch
    p, n, A, mu = CLOUDS[name]()
    Q, C = 3000, mu.shape[1]
    x = workloads.sphere_queries(Q, 31)
    df = workloads.cotangents(Q, C, 17)
    dg = np.random.default_rng(18).standard_normal((Q, C, 3)).astype(np.float32)
    tree = P.dps_build(*to_dev(p, n, A, mu), leaf_size=16, storage=storage)
    T = orc.Tree(p, n, A, mu, 16)
    xd, dfd, dgd = to_dev(x, df, dg)
    tol = _tol(storage)
    for with_df in (True, False):
        print(f"[gradcot] {name} eps={eps} {storage} df={with_df}", flush=True)
        P.dps_adjoint_zero(tree)
        dx = P.dps_adjoint_accumulate_grad(tree, xd, 2.0, eps, dgd, df=dfd if with_df else None)
        da = P.dps_adjoint_finalize(tree)
        ref = T.adjoint(x, 2.0, eps, df if with_df else None, dg=dg)
        # d grad / d mu depends on geometry only: the FP32 bound in both storages
        assert norm_err(to_host(da), ref["dmu"], ref["sdmu"] + 1e-30) <= TOL_FP32
        assert norm_err(to_host(dx), ref["dx"], ref["sdx"][:, None] + 1e-30) <= tol
    P.dps_check(tree)


@pytest.mark.parametrize("flags", [0, 3, 12])
@pytest.mark.parametrize("k", [1, 2, 4])
def test_grad_cotangent_launch_shapes(P, orc, k, flags):
    p, n, A, mu = _random_cloud(3001, 7, C=2)
    Q = 4099
    x = workloads.sphere_queries(Q, 33)
    dg = np.random.default_rng(19).standard_normal((Q, 2, 3)).astype(np.float32)
    df = workloads.cotangents(Q, 2, 20)
    tree = P.dps_build(*to_dev(p, n, A, mu), leaf_size=16)
    P.dps_set_launch(tree, k, k, flags)
    T = orc.Tree(p, n, A, mu, 16)
    xd, dgd, dfd = to_dev(x, dg, df)
    P.dps_adjoint_zero(tree)
    dx = P.dps_adjoint_accumulate_grad(tree, xd, 2.0, 0.05, dgd, df=dfd)
    da = P.dps_adjoint_finalize(tree)
    ref = T.adjoint(x, 2.0, 0.05, df, dg=dg)
    assert norm_err(to_host(da), ref["dmu"], ref["sdmu"] + 1e-30) <= TOL_FP32
    assert norm_err(to_host(dx), ref["dx"], ref["sdx"][:, None] + 1e-30) <= TOL_FP32
    P.dps_check(tree)


@pytest.mark.parametrize("k", [1, 2, 4])
def test_grad_cotangent_on_a_tree_of_21_levels(P, orc, k):
    """The Hessian adjoint on a tree that reaches its last level, with queries
    at every scale around the deep cluster and at its points (eps = 0.05:
    without regularisation the Hessian factor 1/r^7 leaves the FP32 range
    10^-7 from a point)."""
    p, n, A, mu = workloads.deep_cluster_cloud(10, C=2)
    x = np.concatenate([workloads.sphere_queries(1000, 35), workloads.deep_cluster_probes(p, 36)])
    Q = x.shape[0]
    dg = np.random.default_rng(37).standard_normal((Q, 2, 3)).astype(np.float32)
    df = workloads.cotangents(Q, 2, 38)
    tree = P.dps_build(*to_dev(p, n, A, mu), leaf_size=16)
    assert P.dps_tree_info(tree)["depth"] == 21
    P.dps_set_launch(tree, k, k, P.LAUNCH_PERSISTENT_ADJOINT)
    T = orc.Tree(p, n, A, mu, 16)
    xd, dgd, dfd = to_dev(x, dg, df)
    P.dps_adjoint_zero(tree)
    dx = P.dps_adjoint_accumulate_grad(tree, xd, 2.0, 0.05, dgd, df=dfd)
    da = P.dps_adjoint_finalize(tree)
    ref = T.adjoint(x, 2.0, 0.05, df, dg=dg)
    assert norm_err(to_host(da), ref["dmu"], ref["sdmu"] + 1e-30) <= TOL_FP32
    assert norm_err(to_host(dx), ref["dx"], ref["sdx"][:, None] + 1e-30) <= TOL_FP32
    P.dps_check(tree)


def test_grad_cotangent_subsets_counts_and_accumulation(P, orc):
    import torch
    p, n, A, mu = _random_cloud(3001, 8, C=5)
    Q, C = 2000, 5
    x = workloads.sphere_queries(Q, 34)
    rng = np.random.default_rng(21)
    dg = rng.standard_normal((Q, C, 3)).astype(np.float32)
    df = workloads.cotangents(Q, C, 22)
    tree = P.dps_build(*to_dev(p, n, A, mu), leaf_size=16)
    T = orc.Tree(p, n, A, mu, 16)
    xd = to_dev(x)[0]
    # channels [2, 4) with a device row count: rows past it untouched
    k = 1234
    dgs = np.ascontiguousarray(dg[:, 2:4])
    dgsd = to_dev(dgs)[0]
    qc = torch.tensor([k], dtype=torch.int64, device="cuda")
    dx = torch.full((Q, 3), float("nan"), device="cuda")
    P.dps_adjoint_zero(tree)
    P.dps_adjoint_accumulate_grad(tree, xd, 2.0, 0.05, dgsd, c_begin=2, n_channels=2, dx_out=dx, q_count=qc)
    da = to_host(P.dps_adjoint_finalize(tree))
    dgf = np.zeros_like(dg)
    dgf[:, 2:4] = dg[:, 2:4]
    ref = T.adjoint(x[:k], 2.0, 0.05, None, dg=dgf[:k])
    dxh = to_host(dx)
    assert np.isnan(dxh[k:]).all()
    assert norm_err(da, ref["dmu"], ref["sdmu"] + 1e-30) <= TOL_FP32
    assert norm_err(dxh[:k], ref["dx"], ref["sdx"][:, None] + 1e-30) <= TOL_FP32
    # gradient and value cotangents from separate calls accumulate into one
    # push-down
    xd, dgd, dfd = to_dev(x, dg, df)
    P.dps_adjoint_zero(tree)
    P.dps_adjoint_accumulate(tree, xd, 2.0, 0.05, dfd, want_dx=False)
    P.dps_adjoint_accumulate_grad(tree, xd, 2.0, 0.05, dgd, want_dx=False)
    da = to_host(P.dps_adjoint_finalize(tree))
    ref = T.adjoint(x, 2.0, 0.05, df, dg=dg)
    assert norm_err(da, ref["dmu"], ref["sdmu"] + 1e-30) <= TOL_FP32
    # invalid arguments
    with pytest.raises(P.DpsError):
        P.dps_adjoint_accumulate_grad(tree, xd, 2.0, 0.05, dgsd, c_begin=4, n_channels=2)
    P.dps_check(tree)


# ----------------------------------------------------------------------------
# autograd through the surface density of the paper
# ----------------------------------------------------------------------------
S_VAC, DELTA_ABS = 10.0, 1e-2


def _density_loss_torch(f, g, omega, dt, target, n_rays, S):
    """sigma_j = s phi(s gv) sqrt((w . grad gv)^2 + delta^2) / Phi(s gv),
    gv = 1/2 - D_0 (so grad gv = -grad D_0), alpha = 1 - exp(-sigma dt),
    colour = sum_j T_j alpha_j D_{1:3}(x_j), loss = sum |colour - target|^2."""
    import torch
    f = f.reshape(n_rays, S, -1)
    g = g.reshape(n_rays, S, -1, 3)
    z = S_VAC * (0.5 - f[..., 0])
    wg = -torch.sum(omega[:, None, :] * g[..., 0, :], dim=-1)
    ratio = torch.exp(-0.5 * z * z - 0.5 * math.log(2 * math.pi) - torch.special.log_ndtr(z))
    sig = S_VAC * ratio * torch.sqrt(wg * wg + DELTA_ABS ** 2)
    tau = sig * dt[:, None]
    trans = torch.exp(-(torch.cumsum(tau, dim=1) - tau))
    alpha = -torch.expm1(-tau)
    col = torch.sum((trans * alpha)[..., None] * f[..., 1:4], dim=1)
    return torch.sum((col - target) ** 2, dim=1)


def _density_loss_numpy(f, g, omega, dt, target, n_rays, S):
    from scipy.special import log_ndtr
    f = f.reshape(n_rays, S, -1)
    g = g.reshape(n_rays, S, -1, 3)
    z = S_VAC * (0.5 - f[..., 0])
    wg = -np.sum(omega[:, None, :] * g[..., 0, :], axis=-1)
    ratio = np.exp(-0.5 * z * z - 0.5 * math.log(2 * math.pi) - log_ndtr(z))
    sig = S_VAC * ratio * np.sqrt(wg * wg + DELTA_ABS ** 2)
    tau = sig * dt[:, None]
    trans = np.exp(-(np.cumsum(tau, axis=1) - tau))
    alpha = -np.expm1(-tau)
    col = np.sum((trans * alpha)[..., None] * f[..., 1:4], axis=1)
    return np.sum((col - target) ** 2, axis=1)


def test_autograd_surface_density_matches_fd(P, orc):
    import torch
    p, n, A, mu = workloads.winding_cloud(60000, 3000, 70)
    eye = workloads.sfm_camera(71)
    n_rays, S = 160, 64
    o, d, t0, t1 = workloads.camera_rays(eye, 64, 64)
    pix, x = workloads.pixel_ray_samples(eye, 64, 64, S, 72, n_rays, 73)
    omega = d.reshape(-1, 3)[pix]
    dt = ((t1 - t0) / S).reshape(-1)[pix]
    target = np.random.default_rng(74).uniform(size=(n_rays, 3))
    beta, eps = 2.0, 0.01414
    tree = P.dps_build(*to_dev(p, n, A, mu), leaf_size=16)
    attrs = to_dev(mu)[0].requires_grad_(True)
    xt = to_dev(x)[0].requires_grad_(True)
    om_t, dt_t, tg_t = (torch.tensor(a, dtype=torch.float32, device="cuda") for a in (omega, dt, target))
    f, g = P.dipole_sum(attrs, xt, tree, beta, eps)
    loss = torch.sum(_density_loss_torch(f, g, om_t, dt_t, tg_t, n_rays, S))
    da, dx = torch.autograd.grad(loss, [attrs, xt])
    da, dx = to_host(da).astype(np.float64), to_host(dx).astype(np.float64)

    Ta = orc.Tree(p, n, A, mu, 16)
    base = Ta.query(x, beta, eps)
    print(f"[density] loss gpu {float(loss.detach()):.6g} oracle "
          f"{np.sum(_density_loss_numpy(base['f'], base['g'], omega, dt, target, n_rays, S)):.6g}", flush=True)
    # attributes: the field and its gradient are linear in mu, so a step along
    # dmu moves them by the oracle's response to dmu
    dmu = np.random.default_rng(75).standard_normal(mu.shape).astype(np.float32)
    Td = orc.Tree(p, n, A, dmu, 16)
    rd = Td.query(x, beta, eps)
    scale = max(np.abs(rd["f"]).max(), np.abs(rd["g"]).max() * 1e-2)
    h = 1e-4 / scale

    def L(a):
        return _density_loss_numpy(base["f"] + a * rd["f"], base["g"] + a * rd["g"], omega, dt, target, n_rays, S)

    cd = {s: (L(s) - L(-s)) / (2 * s) for s in (h, h / 2)}
    per_ray = (4 * cd[h / 2] - cd[h]) / 3
    fd = float(np.sum(per_ray))
    got = float(np.sum(da * dmu))
    print(f"[density] d loss / d attrs . dmu: gpu {got:.9g} fd {fd:.9g}", flush=True)
    assert abs(got - fd) <= 2e-4 * float(np.sum(np.abs(per_ray))) + 1e-9
    # positions: single coordinates of samples near the surface, re-evaluated
    # with the oracle (values and gradients change), skipped where the
    # traversal changes inside the step
    rng = np.random.default_rng(76)
    cand = np.nonzero(np.abs(base["f"][:, 0] - 0.5) < 0.45)[0]
    assert cand.size > 20
    checked = 0
    for q in rng.choice(cand, size=min(40, cand.size), replace=False):
        r = q // S
        k = int(rng.integers(3))
        blk_f, blk_g = base["f"][r * S:(r + 1) * S].copy(), base["g"][r * S:(r + 1) * S].copy()

        def term(step):
            xp = x[q:q + 1].astype(np.float64).copy()
            xp[0, k] += step
            xp32 = xp.astype(np.float32)
            rr = Ta.query(xp32, beta, eps)
            if not np.array_equal(rr["counts"][0], base["counts"][q]):
                return None
            bf, bg = blk_f.copy(), blk_g.copy()
            bf[q - r * S], bg[q - r * S] = rr["f"][0], rr["g"][0]
            val = _density_loss_numpy(bf, bg, omega[r:r + 1], dt[r:r + 1], target[r:r + 1], 1, S)[0]
            return val, float(xp32[0, k])

        hs = 2.0 ** -16
        vals = {s: term(s) for s in (hs, -hs, hs / 2, -hs / 2)}
        if any(v is None for v in vals.values()):
            continue
        c1 = (vals[hs][0] - vals[-hs][0]) / (vals[hs][1] - vals[-hs][1])
        c2 = (vals[hs / 2][0] - vals[-hs / 2][0]) / (vals[hs / 2][1] - vals[-hs / 2][1])
        fdq = (4 * c2 - c1) / 3
        assert abs(dx[q, k] - fdq) <= 2e-3 * (abs(fdq) + 1e-3 * np.abs(dx[r * S:(r + 1) * S]).max()) + 1e-7, \
            f"sample {q} axis {k}: gpu {dx[q, k]} fd {fdq}"
        checked += 1
    print(f"[density] position derivatives checked on {checked} samples", flush=True)
    assert checked >= 20
    P.dps_check(tree)


def test_grad_cotangent_graph_replays(P):
    import torch
    p, n, A, mu = _random_cloud(3001, 7)
    Q = 20000
    x = workloads.sphere_queries(Q, 35)
    dg = np.random.default_rng(23).standard_normal((Q, 4, 3)).astype(np.float32)
    df = workloads.cotangents(Q, 4, 24)
    tree = P.dps_build(*to_dev(p, n, A, mu), leaf_size=16)
    P.dps_set_launch(tree, 2, 2, 12)
    xd, dgd, dfd = to_dev(x, dg, df)
    dx = torch.empty((Q, 3), device="cuda")
    da = torch.empty((tree.M, 4), device="cuda")

    def step():
        P.dps_adjoint_zero(tree)
        P.dps_adjoint_accumulate_grad(tree, xd, 2.0, 0.05, dgd, df=dfd, dx_out=dx)
        P.dps_adjoint_finalize(tree, dattrs_out=da)

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    ref_dx, ref_da = to_host(dx).copy(), to_host(da).astype(np.float64)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step()
    for r in range(3):
        dx.fill_(float("nan"))
        da.fill_(float("nan"))
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert np.array_equal(to_host(dx), ref_dx), f"replay {r}"
        assert np.max(np.abs(to_host(da) - ref_da)) <= 1e-6 * np.abs(ref_da).max(), f"replay {r}"
    P.dps_check(tree)
