"""Batching pattern: several views of uneven resolution plus one shadow ray per
primary hit, evaluated as one primary launch and one shadow launch whose
size is decided on the device (``q_count``), the whole forward + backward
captured in one graph.

* q_count semantics of the channel entry points (rows past the device count
  untouched, clamping, graph replays with a count changed in between);
* a small batch end to end against the FP64 oracle: primary values, hit
  decisions, shadow values at oracle-placed samples, and the gradients of the
  batched loss w.r.t. attributes and sample positions against central
  differences of the same loss evaluated with the oracle;
* graph replays against eager steps, including attributes updated in place
  between replays;
* the full 8,388,608-point, 8-view, 438,829,056-sample batch (BF16 storage,
  persistent launches, autotuned launch shape) on sampled outputs.
"""
import numpy as np
import pytest

import workloads
from parity import TOL_BF16, TOL_FP32, norm_err, norm_err_all, to_dev, to_host
from workloads import render as R

pytestmark = pytest.mark.gpu

BETA, EPS = 2.0, 0.01414


@pytest.fixture(scope="module")
def P():
    import torch
    import paper_2405_16788_amd as lib
    lib.load()
    assert torch.cuda.is_available()
    return lib


def _tol(storage):
    return TOL_BF16 if storage == "bf16" else TOL_FP32


def _ray_major(a, S, last):
    """[T*S*64, last] batch layout -> [T*64, S, last] (ray-major)."""
    T = a.shape[0] // (S * 64)
    return a.reshape(T, S, 64, last).transpose(0, 2, 1, 3).reshape(T * 64, S, last)


# ----------------------------------------------------------------------------
# device row counts
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("storage", ["fp32", "bf16"])
def test_q_count_rows(P, orc, storage):
    import torch
    p, n, A, mu = workloads.winding_cloud(20000, 1000, 50)
    x = workloads.sphere_queries(5000, 51)
    Q, C = x.shape[0], mu.shape[1]
    df = workloads.cotangents(Q, C, 52)
    T = orc.Tree(p, n, A, mu, 16)
    ref = T.query(x, BETA, 0.05)
    tree = P.dps_build(*to_dev(p, n, A, mu), leaf_size=16, storage=storage)
    xd, dfd = to_dev(x, df)
    qc = torch.zeros(1, dtype=torch.int64, device="cuda")
    tol = _tol(storage)
    nan = float("nan")
    for k in (0, 1, 2999, Q, Q + 2000, -5):
        kk = min(max(k, 0), Q)
        print(f"[q_count] storage={storage} count={k}", flush=True)
        qc.fill_(k)
        f = torch.full((Q, C), nan, device="cuda")
        g = torch.full((Q, C, 3), nan, device="cuda")
        P.dps_query_channels(tree, xd, BETA, 0.05, 0, C, f_out=f, g_out=g, q_count=qc)
        fh, gh = to_host(f), to_host(g)
        assert np.isnan(fh[kk:]).all() and np.isnan(gh[kk:]).all()
        assert norm_err(fh[:kk], ref["f"][:kk], ref["sf"][:kk]) <= tol
        assert norm_err(gh[:kk], ref["g"][:kk], ref["sg"][:kk]) <= tol
        dx = torch.full((Q, 3), nan, device="cuda")
        P.dps_adjoint_zero(tree)
        P.dps_adjoint_accumulate_channels(tree, xd, BETA, 0.05, 0, C, dfd, dx_out=dx, q_count=qc)
        da = to_host(P.dps_adjoint_finalize(tree))
        dxh = to_host(dx)
        assert np.isnan(dxh[kk:]).all()
        if kk == 0:
            assert not np.any(da)
        else:
            adj = T.adjoint(x[:kk], BETA, 0.05, df[:kk])
            assert norm_err(da, adj["dmu"], adj["sdmu"] + 1e-30) <= TOL_FP32
            assert norm_err(dxh[:kk], adj["dx"], adj["sdx"]) <= tol
    # the count is read when the kernels run: replays of one captured launch
    # follow a count written between them
    f = torch.full((Q, C), nan, device="cuda")
    qc.fill_(Q)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        P.dps_query_channels(tree, xd, BETA, 0.05, 0, C, grad=False, f_out=f, q_count=qc)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        P.dps_query_channels(tree, xd, BETA, 0.05, 0, C, grad=False, f_out=f, q_count=qc)
    for k in (3000, 1234, Q, 0):
        f.fill_(nan)
        qc.fill_(k)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        fh = to_host(f)
        assert np.isnan(fh[k:]).all(), f"replay with count {k}: rows past the count written"
        assert norm_err(fh[:k], ref["f"][:k], ref["sf"][:k]) <= tol
    P.dps_check(tree)


# ----------------------------------------------------------------------------
# small batch end to end against the oracle
# ----------------------------------------------------------------------------
class OracleBatch:
    """The batched proxy evaluated with the FP64 oracle (values from two
    oracle trees: attributes a and a direction d, combined linearly)."""

    def __init__(self, orc, p, n, A, mu, dmu, xb, batch_host):
        self.Ta = orc.Tree(p, n, A, mu, 16)
        self.Td = orc.Tree(p, n, A, dmu, 16)
        self.x = xb
        self.b = batch_host
        S = batch_host["S"]
        ra = self.Ta.query(xb, BETA, EPS, want_grad=False)
        rd = self.Td.query(xb, BETA, EPS, want_grad=False)
        self.fa = _ray_major(ra["f"], S, mu.shape[1])
        self.fd = _ray_major(rd["f"], S, mu.shape[1])
        self.sfa = _ray_major(ra["sf"], S, mu.shape[1])
        self.xr = _ray_major(xb.astype(np.float64), S, 3)

    def shadow_values(self, xs, has, alpha):
        """Channel-0 values at the shadow samples of the hit rays (FP32
        positions, as the GPU reads them) and the traversal counts."""
        n, K = xs.shape[:2]
        fs = np.zeros((n, K))
        cnt = np.zeros((n, K, 4), dtype=np.int64)
        if has.any():
            q = xs[has].reshape(-1, 3).astype(np.float32)
            ra = self.Ta.query(q, BETA, EPS, want_grad=False)
            val = ra["f"][:, 0]
            if alpha != 0.0:
                val = val + alpha * self.Td.query(q, BETA, EPS, want_grad=False)["f"][:, 0]
            fs[has] = val.reshape(-1, K)
            cnt[has] = ra["counts"].reshape(-1, K, 4)
        return fs, cnt

    def hit_values(self, hit, has, alpha):
        """Values and gradients of all channels at the hits (FP32 positions)
        and the traversal counts of those queries."""
        n, C = hit.shape[0], self.fa.shape[2]
        fh, gh = np.zeros((n, C)), np.zeros((n, C, 3))
        cnt = np.zeros((n, 4), dtype=np.int64)
        if has.any():
            q = hit[has].astype(np.float32)
            ra = self.Ta.query(q, BETA, EPS)
            fv, gv = ra["f"], ra["g"]
            if alpha != 0.0:
                rd = self.Td.query(q, BETA, EPS)
                fv, gv = fv + alpha * rd["f"], gv + alpha * rd["g"]
            fh[has], gh[has], cnt[has] = fv, gv, ra["counts"]
        return fh, gh, cnt

    def terms(self, alpha):
        f = self.fa + alpha * self.fd
        has, j, hit = R.primary_hits_numpy(f[..., 0], self.xr)
        xs = R.shadow_samples_numpy(hit, has, self.b["light"], self.b["u"])
        fs, cnt = self.shadow_values(xs, has, alpha)
        fh, gh, hcnt = self.hit_values(hit, has, alpha)
        t = R.batched_ray_terms_numpy(f, fs, has, self.b["target"], fh, gh, hit, self.b["light"])
        return t, has, j, (cnt, hcnt), xs


def _small_batch(P, orc, storage):
    import torch
    p, n, A, mu = workloads.winding_cloud(30000, 1500, 53)
    batch = workloads.make_ray_batch(res=(16, 24, 32), S=32, S_shadow=16, seeds=(54, 55))
    rng = np.random.default_rng(56)
    dmu = rng.standard_normal(mu.shape).astype(np.float32)
    bh = {"S": batch.S, "light": to_host(batch.ray_light).astype(np.float64),
          "u": to_host(batch.shadow_u).astype(np.float64), "target": to_host(batch.target).astype(np.float64)}
    ob = OracleBatch(orc, p, n, A, mu, dmu, to_host(batch.x), bh)
    pd, nd, Ad, mud = to_dev(p, n, A, mu)
    tree = P.dps_build(pd, nd, Ad, mud, leaf_size=16, storage=storage)
    return tree, batch, ob, mu, dmu, mud


def _gpu_step(P, tree, batch, mud, ray_weight=None):
    import torch
    attrs = mud.clone().requires_grad_(True)
    x = batch.x.clone().requires_grad_(True)
    loss, aux = R.batched_forward(P.dipole_sum, attrs, x, tree, batch, BETA, EPS, ray_weight=ray_weight)
    da, dx = torch.autograd.grad(loss, [attrs, x])
    return loss, aux, da, dx


def test_batched_small_against_oracle(P, orc):
    import torch
    tree, batch, ob, mu, dmu, mud = _small_batch(P, orc, "fp32")
    S, K, C = batch.S, batch.S_shadow, mu.shape[1]
    terms0, has_o, j_o, cnt0, xs_o = ob.terms(0.0)
    n_rays = has_o.size
    print(f"[batched-small] rays={n_rays} hits={int(has_o.sum())} Q={batch.Q}", flush=True)
    assert 20 <= has_o.sum() < n_rays
    # forward parity of every primary sample
    loss, aux, _, _ = _gpu_step(P, tree, batch, mud)
    fg = _ray_major(to_host(aux["f"]), S, C)
    assert norm_err(fg, ob.fa, ob.sfa) <= TOL_FP32
    # hit decisions agree wherever no sample sits within the FP32 error of 1/2
    margin = np.min(np.abs(ob.fa[..., 0] - 0.5) / np.maximum(ob.sfa[..., 0], 1e-30), axis=1)
    robust = margin > 1e-4
    has_g = to_host(aux["has"])
    assert robust.mean() > 0.9
    assert np.array_equal(has_g[robust], has_o[robust])
    assert int(aux["n_hits"]) == int(has_g.sum())
    assert int(aux["q_count"][0]) == -(-int(has_g.sum()) // 64) * 64 * K
    # the compacted shadow launch evaluated at oracle-placed samples
    xs32 = xs_o[has_o].reshape(-1, 3).astype(np.float32)
    nh = int(has_o.sum())
    rows = np.arange(nh)
    grp, lane = rows // 64, rows % 64
    qrow = ((grp * K)[:, None] + np.arange(K)[None, :]) * 64 + lane[:, None]
    cap = -(-nh // 64) * 64 * K
    xq = np.zeros((cap + 64 * K, 3), np.float32)
    xq[qrow.reshape(-1)] = xs32
    (xqd,) = to_dev(xq)
    qc = torch.tensor([cap], dtype=torch.int64, device="cuda")
    fs = torch.full((xq.shape[0], 1), float("nan"), device="cuda")
    P.dps_query_channels(tree, xqd, BETA, EPS, 0, 1, grad=False, f_out=fs, q_count=qc)
    fsh = to_host(fs)
    assert np.isnan(fsh[cap:]).all()
    ref = ob.Ta.query(xs32, BETA, EPS, want_grad=False)
    assert norm_err(fsh[qrow.reshape(-1), 0], ref["f"][:, 0], ref["sf"][:, 0]) <= TOL_FP32

    # gradients of the batched loss against central differences of the
    # oracle-evaluated loss.  Rays whose hit index or shadow traversal
    # changes inside the step are left out of the loss (weight 0), decided
    # from the oracle alone.
    # a field step of 2e-3 moves the hits by ~1e-4, far above the FP32
    # rounding of the shadow sample positions the oracle reads
    step = 2e-3 / max(float(np.abs(ob.fd[..., 0]).max()), 1e-30)
    runs = {a: ob.terms(a) for a in (step, -step, step / 2, -step / 2)}
    keep = robust.copy()
    for a, (_, has_a, j_a, cnt_a, _) in runs.items():
        keep &= (has_a == has_o) & ((j_a == j_o) | ~has_o)
        keep &= np.all(cnt_a[0] == cnt0[0], axis=(1, 2)) & np.all(cnt_a[1] == cnt0[1], axis=1)
    assert keep.sum() > 0.8 * n_rays and (keep & has_o).sum() >= 10
    w = keep.astype(np.float64)
    cd = {h: (np.sum(w * runs[h][0]) - np.sum(w * runs[-h][0])) / (2 * h) for h in (step, step / 2)}
    fd_attr = (4.0 * cd[step / 2] - cd[step]) / 3.0
    per_ray = np.abs((runs[step / 2][0] - runs[-step / 2][0]) / step) * w
    (wd,) = to_dev(w.astype(np.float32))
    _, aux, da, dx = _gpu_step(P, tree, batch, mud, ray_weight=wd)
    got = float(np.sum(to_host(da).astype(np.float64) * dmu))
    print(f"[batched-small] d loss / d attrs . dmu: gpu {got:.9g} fd {fd_attr:.9g}", flush=True)
    assert abs(got - fd_attr) <= 1e-3 * float(per_ray.sum()) + 1e-9
    # positions: per ray, the two samples around the hit of kept hit rays moved
    # along a random direction; this moves the hit and so the whole shadow ray
    # (each ray's loss term depends on its own samples only).  Step 3e-4, or
    # 1e-4 where a traversal changes inside the larger step; the FP32
    # rounding of the moved shadow samples leaves ~1e-3 relative noise.
    rng = np.random.default_rng(57)
    cand = np.nonzero(keep & has_o)[0]
    pick = rng.choice(cand, size=min(40, cand.size), replace=False)
    dxh = _ray_major(to_host(dx), S, 3)
    checked = 0
    for r in pick:
        dirx = np.zeros((S, 3))
        dirx[j_o[r]:j_o[r] + 2] = rng.standard_normal((2, 3))
        res = _fd_position_ray(ob, r, dirx, 3e-4) or _fd_position_ray(ob, r, dirx, 1e-4)
        if res is None:
            continue
        fd, eff = res
        got = float(np.sum(dxh[r].astype(np.float64) * eff))
        scale = abs(fd) + 1e-3 * float(np.abs(dxh[r]).sum() * np.abs(dirx).max())
        assert abs(got - fd) <= 5e-3 * scale + 1e-6, f"ray {r}: gpu {got} fd {fd}"
        checked += 1
    print(f"[batched-small] position derivatives checked on {checked} rays", flush=True)
    assert checked >= 16
    P.dps_check(tree)


def _fd_position_ray(ob, r, dirx, h):
    """Central difference (Richardson over h, h/2) of ray r's loss term when
    its S samples move by h * dirx, with the moved positions rounded to FP32
    (as the GPU would read them) and values from the oracle.  Returns
    (derivative, effective direction): the rounding is folded into the
    direction the difference quotient actually measures.  None if the hit
    index or any traversal changes inside the step."""
    b = ob.b
    x0 = ob.xr[r]
    base = ob.Ta.query(x0.astype(np.float32), BETA, EPS, want_grad=False)

    def term(step):
        xp = (x0 + step * dirx).astype(np.float32)
        ra = ob.Ta.query(xp, BETA, EPS, want_grad=False)
        if not np.array_equal(ra["counts"], base["counts"]):
            return None
        f = ra["f"][None]
        has, j, hit = R.primary_hits_numpy(f[..., 0], xp.astype(np.float64)[None])
        xs = R.shadow_samples_numpy(hit, has, b["light"][r:r + 1], b["u"][r:r + 1])
        fs, cnt = ob.shadow_values(xs, has, 0.0)
        fh, gh, hcnt = ob.hit_values(hit, has, 0.0)
        val = R.batched_ray_terms_numpy(f, fs, has, b["target"][r:r + 1], fh, gh, hit, b["light"][r:r + 1])[0]
        return val, bool(has[0]), int(j[0]), (cnt, hcnt), xp.astype(np.float64) - x0

    vals = {s: term(s) for s in (h, -h, h / 2, -h / 2)}
    if any(v is None for v in vals.values()):
        return None
    if len({(v[1], v[2]) for v in vals.values()}) != 1:
        return None
    c0 = vals[h][3]
    if not all(np.array_equal(v[3][0], c0[0]) and np.array_equal(v[3][1], c0[1]) for v in vals.values()):
        return None
    cd = {s: (vals[s][0] - vals[-s][0]) / (2 * s) for s in (h, h / 2)}
    dd = {s: (vals[s][4] - vals[-s][4]) / (2 * s) for s in (h, h / 2)}
    return (4.0 * cd[h / 2] - cd[h]) / 3.0, (4.0 * dd[h / 2] - dd[h]) / 3.0


def _clone_state(aux, loss, da, dx):
    return {"loss": to_host(loss).copy(), "f": to_host(aux["f"]).copy(), "fs": to_host(aux["fs"]).copy(),
            "q_count": int(aux["q_count"][0]), "da": to_host(da).astype(np.float64), "dx": to_host(dx).copy()}


def _compare(st, ref, what):
    assert st["q_count"] == ref["q_count"], f"{what}: shadow count differs"
    assert np.array_equal(st["f"], ref["f"]), f"{what}: primary values differ"
    qc = ref["q_count"]
    assert np.array_equal(st["fs"][:qc], ref["fs"][:qc]), f"{what}: shadow values differ"
    assert np.array_equal(st["loss"], ref["loss"]), f"{what}: loss differs"
    assert np.array_equal(st["dx"], ref["dx"]), f"{what}: position gradient differs"
    scale = np.abs(ref["da"]).max()
    assert np.max(np.abs(st["da"] - ref["da"])) <= 1e-5 * scale, f"{what}: attribute gradient differs"


@pytest.mark.parametrize("flags", [3, 12])
def test_batched_graph_replays(P, orc, flags):
    """The whole batched step in one graph: every replay equals an eager step
    on the same attributes, also after the attributes change in place."""
    import torch
    p, n, A, mu = workloads.winding_cloud(60000, 3000, 58)
    batch = workloads.make_ray_batch(res=(32, 48, 64, 40), S=64, S_shadow=32, seeds=(59, 60))
    pd, nd, Ad, mud = to_dev(p, n, A, mu)
    tree = P.dps_build(pd, nd, Ad, mud, leaf_size=16, storage="bf16")
    P.dps_set_launch(tree, 2, 4, flags)
    attrs = mud.clone()
    x = batch.x.clone()

    def step():
        # fresh leaves over the same storage: in-place updates of attrs reach
        # every call, and no autograd node outlives its step
        a = attrs.detach().requires_grad_(True)
        xl = x.detach().requires_grad_(True)
        loss, aux = R.batched_forward(P.dipole_sum, a, xl, tree, batch, BETA, EPS)
        da, dx = torch.autograd.grad(loss, [a, xl])
        return loss.detach(), aux, da, dx

    def eager():
        out = step()
        torch.cuda.synchronize()
        return _clone_state(out[1], *((out[0],) + out[2:]))

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        ref = eager()
    torch.cuda.current_stream().wait_stream(side)
    assert 0 < ref["q_count"] < batch.n_rays * batch.S_shadow
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        g_loss, g_aux, g_da, g_dx = step()
    for r in range(3):
        for v in (g_loss, g_aux["f"], g_aux["fs"], g_da, g_dx):
            v.fill_(float("nan"))
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        _compare(_clone_state(g_aux, g_loss, g_da, g_dx), ref, f"replay {r}")
        P.dps_query(tree, batch.x[:4096].contiguous(), BETA, EPS)  # eager work between replays
    # attributes updated in place (as an optimiser would) reach the captured
    # refit: geometry scaled (moves the hits, changes the shadow count) and
    # colours halved
    attrs[:, 0].mul_(1.3)
    attrs[:, 1:].mul_(0.5)
    ref2 = eager()
    assert ref2["q_count"] != ref["q_count"]
    graph.replay()
    torch.cuda.synchronize()
    _compare(_clone_state(g_aux, g_loss, g_da, g_dx), ref2, "replay after update")
    P.dps_check(tree)


# ----------------------------------------------------------------------------
# the full batch: 8,388,608 points, 8 views 256^2..1024^2, 128 + 64 samples
# ----------------------------------------------------------------------------
def test_sfm_8m_batched(P, orc):
    import torch
    print("[sfm-8m] generating the scene", flush=True)
    p, n, A, mu = workloads.sfm_8m_cloud()
    batch = workloads.make_ray_batch()
    S, K, C = batch.S, batch.S_shadow, mu.shape[1]
    assert batch.Q == 438_829_056 and batch.n_rays == 3_428_352
    pd, nd, Ad, mud = to_dev(p, n, A, mu)
    tree = P.dps_build(pd, nd, Ad, mud, leaf_size=16, storage="bf16")
    info = P.dps_tree_info(tree)
    print(f"[sfm-8m] tree nodes={info['n_nodes']} depth={info['depth']}", flush=True)
    from paper_2405_16788_amd import autotune
    df = torch.randn(1 << 22, C, device="cuda")
    best = autotune.tune(tree, batch.x[: 1 << 22], df, BETA, EPS, sample=1 << 22, reps=1, cache="")
    del df
    print(f"[sfm-8m] launch {best['query']},{best['adjoint']},{best['flags']}", flush=True)
    def step():
        a = mud.detach().requires_grad_(True)
        xl = batch.x.detach().requires_grad_(True)
        loss, aux = R.batched_forward(P.dipole_sum, a, xl, tree, batch, BETA, EPS)
        da, dx = torch.autograd.grad(loss, [a, xl])
        return loss.detach(), aux, da, dx

    rng = np.random.default_rng(61)
    qs = np.sort(rng.choice(batch.Q, size=2048, replace=False))
    rays = np.sort(rng.choice(batch.n_rays, size=256, replace=False))
    qs_t = torch.from_numpy(qs).cuda()

    def sample_state(loss, aux, da, dx):
        return {"loss": float(loss), "f": to_host(aux["f"][qs_t]), "dx": to_host(dx[qs_t]),
                "q_count": int(aux["q_count"][0]), "n_hits": int(aux["n_hits"]),
                "da": to_host(da).astype(np.float64), "has": to_host(aux["has"])}

    print("[sfm-8m] eager step", flush=True)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        out = step()
        torch.cuda.synchronize()
        ref = sample_state(*out)
        # primary values of the sampled rays, for the hit checks
        T_ = batch.Q // (S * 64)
        f0_rays = to_host(out[1]["f"].view(T_, S, 64, C)[:, :, :, 0].permute(0, 2, 1).reshape(-1, S)[
            torch.from_numpy(rays).cuda()])
        del out
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    print(f"[sfm-8m] hits {ref['n_hits']} shadow rows {ref['q_count']}", flush=True)
    assert 0.02 * batch.n_rays < ref["n_hits"] < batch.n_rays
    assert np.isfinite(ref["loss"]) and np.all(np.isfinite(ref["da"])) and np.all(np.isfinite(ref["dx"]))

    print("[sfm-8m] capture + replays", flush=True)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        g_out = step()
    for r in range(2):
        graph.replay()
        torch.cuda.synchronize()
        st = sample_state(*g_out)
        assert st["q_count"] == ref["q_count"] and st["loss"] == ref["loss"], f"replay {r}"
        assert np.array_equal(st["f"], ref["f"]) and np.array_equal(st["dx"], ref["dx"]), f"replay {r}"
        assert np.max(np.abs(st["da"] - ref["da"])) <= 1e-5 * np.abs(ref["da"]).max(), f"replay {r}"
    P.dps_check(tree)
    del graph, g_out
    torch.cuda.synchronize()

    print("[sfm-8m] oracle tree and sampled queries", flush=True)
    T = orc.Tree(p, n, A, mu, 16)
    xh = to_host(batch.x[qs_t])
    ro = T.query(xh, BETA, EPS)
    assert norm_err(ref["f"], ro["f"], ro["sf"]) <= TOL_BF16
    e = norm_err_all(ref["f"], ro["f"], ro["sf"])
    print(f"[sfm-8m] sampled primaries: max {e.max():.3g} p99.9 {np.percentile(e, 99.9):.3g}", flush=True)
    # hit decisions of sampled rays: equal wherever no sample is within the
    # BF16 bound of 1/2; an undecided ray must still be a valid crossing
    T_ = batch.Q // (S * 64)
    tile, lane = rays // 64, rays % 64
    qidx = (tile[:, None] * S + np.arange(S)[None, :]) * 64 + lane[:, None]
    xr = to_host(batch.x[torch.from_numpy(qidx.reshape(-1)).cuda()]).reshape(-1, S, 3)
    rr = T.query(xr.reshape(-1, 3), BETA, EPS, want_grad=False)
    fo = rr["f"][:, 0].reshape(-1, S)
    so = rr["sf"][:, 0].reshape(-1, S)
    has_o, j_o, hit_o = R.primary_hits_numpy(fo, xr.astype(np.float64))
    c = f0_rays >= 0.5
    cross = c[:, 1:] != c[:, :-1]
    has_g, j_g = cross.any(axis=1), np.argmax(cross, axis=1)
    assert np.array_equal(has_g, ref["has"][rays])
    robust = np.all(np.abs(fo - 0.5) > TOL_BF16 * so, axis=1)
    assert np.array_equal(has_g[robust], has_o[robust])
    assert np.array_equal(j_g[robust & has_o], j_o[robust & has_o])
    # shadow values at oracle-placed samples of the sampled hit rays
    hr = np.nonzero(has_o)[0][:64]
    if hr.size:
        light = to_host(batch.ray_light[torch.from_numpy(rays[hr]).cuda()]).astype(np.float64)
        u = to_host(batch.shadow_u[torch.from_numpy(rays[hr]).cuda()]).astype(np.float64)
        xs = R.shadow_samples_numpy(hit_o[hr], np.ones(hr.size, bool), light, u).reshape(-1, 3).astype(np.float32)
        (xsd,) = to_dev(xs)
        fs, _ = P.dps_query_channels(tree, xsd, BETA, EPS, 0, 1, grad=False)
        rs = T.query(xs, BETA, EPS, want_grad=False)
        assert norm_err(to_host(fs)[:, 0], rs["f"][:, 0], rs["sf"][:, 0]) <= TOL_BF16
    P.dps_check(tree)


def test_sfm_8m_subbatch_against_oracle(P, orc):
    """The batched workload's kernels in the benchmark's configuration
    (8,388,608 points, BF16 storage, autotuned persistent launch) on a
    multi-view, tile-aligned sub-batch, element by element against the
    oracle: 6 tiles near the image centre of each of the 8 views (primary rows
    in [tile, sample, lane] order), the shadow rows of the oracle's own hits
    (64 samples, the compacted [group, sample, lane] layout, a device row
    count) and one hit-point row per hit.  Forward values and the adjoint with
    seeded cotangents -- values of the primaries, channel 0 of the shadow
    rows, values and gradients of the hit points -- run in one captured graph;
    two replays are each compared with the oracle (dL/dmu and dL/dx exactly
    against the FP64 sums, values and dL/dx against the sums of the values as
    stored)."""
    import torch
    print("[sfm-8m sub] generating the scene", flush=True)
    p, n, A, mu = workloads.sfm_8m_cloud()
    batch = workloads.make_ray_batch()
    S, K, C = batch.S, batch.S_shadow, mu.shape[1]
    G = 64
    tiles = []
    for v, res in enumerate(batch.res):
        side = res // 8
        t0 = batch.ray_offsets[v] // G
        mid = (side // 2) * side + side // 2
        # four tiles at the image centre (rays that hit) and the two first
        # tiles of the view (a corner: rays that miss)
        tiles += [t0 + mid + k for k in (-side - 1, -side, -1, 0)] + [t0, t0 + 1]
    tiles = np.array(sorted(tiles))
    rows = ((tiles[:, None] * S + np.arange(S)[None, :]) * G)[:, :, None] + np.arange(G)[None, None, :]
    rows_t = torch.from_numpy(rows.reshape(-1)).cuda()
    xp = to_host(batch.x[rows_t])  # primary rows of the sub-batch, [tile, sample, lane]
    ray_ids = (tiles[:, None] * G + np.arange(G)[None, :]).reshape(-1)
    light = to_host(batch.ray_light[torch.from_numpy(ray_ids).cuda()]).astype(np.float64)
    su = to_host(batch.shadow_u[torch.from_numpy(ray_ids).cuda()]).astype(np.float64)
    del batch
    torch.cuda.empty_cache()

    print(f"[sfm-8m sub] oracle tree, {xp.shape[0]} primary rows", flush=True)
    T = orc.Tree(p, n, A, mu, 16)
    T.set_storage("bf16", 3)
    nt = tiles.size
    f0 = T.query(xp, BETA, EPS, want_grad=False)["f"][:, 0].reshape(nt, S, G).transpose(0, 2, 1).reshape(-1, S)
    xr = xp.reshape(nt, S, G, 3).transpose(0, 2, 1, 3).reshape(-1, S, 3).astype(np.float64)
    has, _, hit = R.primary_hits_numpy(f0, xr)
    n_hits = int(has.sum())
    print(f"[sfm-8m sub] oracle hits {n_hits} of {has.size} rays", flush=True)
    assert 64 <= n_hits < has.size
    # shadow rows: hit rays in ray order, groups of 64 rays, [sample, lane] inside a group
    hr = np.flatnonzero(has)
    xs = R.shadow_samples_numpy(hit[hr], np.ones(n_hits, bool), light[hr], su[hr])  # [n_hits, K, 3]
    n_groups = (n_hits + G - 1) // G
    cap = n_groups * G
    xs_pad = np.concatenate([xs, np.broadcast_to(light[hr[:1]][:, None, :], (cap - n_hits, K, 3))])
    xs_rows = xs_pad.reshape(n_groups, G, K, 3).transpose(0, 2, 1, 3).reshape(-1, 3).astype(np.float32)
    xh = np.concatenate([hit[hr], np.broadcast_to(hit[hr[:1]], (cap - n_hits, 3))]).astype(np.float32)
    rng = np.random.default_rng(62)
    dfp = rng.standard_normal((xp.shape[0], C)).astype(np.float32)
    dfs = rng.standard_normal((xs_rows.shape[0], 1)).astype(np.float32)
    dfh = rng.standard_normal((cap, C)).astype(np.float32)
    dgh = rng.standard_normal((cap, C, 3)).astype(np.float32)
    # only the evaluated rows carry cotangents: shadow rows up to the last
    # started group (the device count), hit rows up to n_hits
    qs_count, qh_count = xs_rows.shape[0], n_hits
    dfh[n_hits:] = 0.0
    dgh[n_hits:] = 0.0

    print("[sfm-8m sub] oracle forward and adjoint", flush=True)
    rf = T.query(xp, BETA, EPS)
    rs = T.query(xs_rows, BETA, EPS, want_grad=False)
    rh = T.query(xh[:n_hits], BETA, EPS)
    dfs_full = np.zeros((xs_rows.shape[0], C), np.float32)
    dfs_full[:, 0] = dfs[:, 0]
    a1 = T.adjoint(xp, BETA, EPS, dfp)
    a2 = T.adjoint(xs_rows, BETA, EPS, dfs_full)
    a3 = T.adjoint(xh[:n_hits], BETA, EPS, dfh[:n_hits], dg=dgh[:n_hits])
    dmu = a1["dmu"] + a2["dmu"] + a3["dmu"]
    sdmu = a1["sdmu"] + a2["sdmu"] + a3["sdmu"]

    pd, nd, Ad, mud = to_dev(p, n, A, mu)
    tree = P.dps_build(pd, nd, Ad, mud, leaf_size=16, storage="bf16")
    xpd, xsd, xhd, dfpd, dfsd, dfhd, dghd = to_dev(xp, xs_rows, xh, dfp, dfs, dfh, dgh)
    qs = torch.tensor([qs_count], dtype=torch.int64, device="cuda")
    qh = torch.tensor([qh_count], dtype=torch.int64, device="cuda")
    Qp, Qs = xp.shape[0], xs_rows.shape[0]
    out = {"f": torch.empty((Qp, C), device="cuda"), "g": torch.empty((Qp, C, 3), device="cuda"),
           "fs": torch.empty((Qs, 1), device="cuda"), "fh": torch.empty((cap, C), device="cuda"),
           "gh": torch.empty((cap, C, 3), device="cuda"), "dxp": torch.empty((Qp, 3), device="cuda"),
           "dxs": torch.empty((Qs, 3), device="cuda"), "dxh": torch.empty((cap, 3), device="cuda"),
           "da": torch.empty((p.shape[0], C), device="cuda")}

    def step():
        P.dps_set_attributes(tree, mud)
        P.dps_query(tree, xpd, BETA, EPS, f_out=out["f"], g_out=out["g"])
        P.dps_query_channels(tree, xsd, BETA, EPS, 0, 1, grad=False, f_out=out["fs"], q_count=qs)
        P.dps_query_channels(tree, xhd, BETA, EPS, 0, C, f_out=out["fh"], g_out=out["gh"], q_count=qh)
        P.dps_adjoint_zero(tree)
        P.dps_adjoint_accumulate(tree, xpd, BETA, EPS, dfpd, dx_out=out["dxp"])
        P.dps_adjoint_accumulate_channels(tree, xsd, BETA, EPS, 0, 1, dfsd, dx_out=out["dxs"], q_count=qs)
        P.dps_adjoint_accumulate_grad(tree, xhd, BETA, EPS, dghd, df=dfhd, dx_out=out["dxh"], q_count=qh)
        P.dps_adjoint_finalize(tree, dattrs_out=out["da"])

    # the launch the autotuner picks for the whole batch (persistent tile
    # queue, 4 queries per lane in the query, 2 in the adjoint), and a plain
    # grid with one query per lane
    for launch in ((4, 2, P.LAUNCH_PERSISTENT_QUERY | P.LAUNCH_PERSISTENT_ADJOINT), (1, 1, 0)):
        P.dps_set_launch(tree, *launch)
        print(f"[sfm-8m sub] launch {launch}", flush=True)
        _subbatch_replays(P, tree, step, out, n_hits, rf, rs, rh, a1, a2, a3, dmu, sdmu)
    P.dps_destroy(tree)


def _subbatch_replays(P, tree, step, out, n_hits, rf, rs, rh, a1, a2, a3, dmu, sdmu):
    import torch
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step()  # warm-up outside the capture
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=side):
            step()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    for rep in range(2):
        for v in out.values():
            v.fill_(float("nan"))
        graph.replay()
        torch.cuda.synchronize()
        P.dps_check(tree)
        h = {k: to_host(v) for k, v in out.items()}
        checks = {
            "primary f": norm_err_all(h["f"], rf["f"], rf["sf"]),
            "primary grad": norm_err_all(h["g"], rf["g"], rf["sg"]),
            "shadow f": norm_err_all(h["fs"][:, 0], rs["f"][:, 0], rs["sf"][:, 0]),
            "hit f": norm_err_all(h["fh"][:n_hits], rh["f"], rh["sf"]),
            "hit grad": norm_err_all(h["gh"][:n_hits], rh["g"], rh["sg"]),
            "dL/dmu": norm_err_all(h["da"], dmu, sdmu),
            "primary dL/dx": norm_err_all(h["dxp"], a1["dx"], a1["sdx"]),
            "shadow dL/dx": norm_err_all(h["dxs"], a2["dx"], a2["sdx"]),
            "hit dL/dx": norm_err_all(h["dxh"][:n_hits], a3["dx"], a3["sdx"]),
        }
        for k, e in checks.items():
            print(f"[sfm-8m sub] replay {rep} {k}: max {e.max():.3g}", flush=True)
        bad = {k: float(e.max()) for k, e in checks.items() if not e.max() <= TOL_FP32}
        assert not bad, bad
