"""Storage parity: the moments the GPU refit stores and the results computed
from them, against the FP64 oracle evaluated from values rounded exactly as
that storage holds them (``Tree.set_storage``).

- FP32 storage: every stored node moment is the FP64 moment (eq.
  farfield_dipole_features, Sec. 6.1) rounded once to FP32 -- the refit's
  compensated FP32 sums make that exact up to a rare one-ulp tie.
- BF16 storage: point attributes are rounded to bfloat16, node moments to
  FP32 and then bfloat16, except the nodes of depth <= 3, which stay FP32.
  The GPU's query, adjoint and gradient-cotangent results are held to the
  FP32 bar (1e-5) against the oracle evaluated from those rounded values, so
  a decode or layout error of the reduced-precision path cannot hide under
  the 2^-8 rounding bound.  Rounding-boundary flips (a stored value one unit
  away from the oracle's rounding) are counted and bounded.
- FP32 storage is also held to 1e-5 with the stricter error scale of a node
  term, the magnitude of its own moment |D_t| instead of its absolute mass.

Every test prints the normwise error ||gpu - oracle||_2 / ||oracle||_2 next to
the normalised maximum.
"""
import numpy as np
import pytest

import workloads
from parity import TOL_BF16, TOL_FP32, norm_err_all, normwise, to_dev, to_host

pytestmark = pytest.mark.gpu

FP32_LEVELS = 3  # nodes of depth <= 3 keep FP32 moments under BF16 storage


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
    # (generator, leaf size)
    "sphere-8k": (lambda: workloads.sphere_cloud(8192, 1), 16),
    "sphere-8k-leaf1": (lambda: workloads.sphere_cloud(8192, 1), 1),
    "random-3001-c5": (lambda: _random_cloud(3001, 8, C=5), 4),
    "random-2000-c1": (lambda: _random_cloud(2000, 9, C=1), 16),
    "sfm-63k": (lambda: workloads.sfm_cloud(60000, 3000, 61), 16),
}


def _ulp(v, fmt):
    """Unit in the last place of |v| in FP32 or bfloat16 (8 significant bits)."""
    a = np.abs(np.asarray(v, np.float64))
    if fmt == "fp32":
        return np.spacing(a.astype(np.float32)).astype(np.float64)
    e = np.floor(np.log2(np.maximum(a, 2.0 ** -133)))
    return 2.0 ** np.maximum(e - 7, -133)


def _stored_flips(ex_mom, T, storage, levels):
    """Compares the GPU's stored moments with the oracle's rounding of its
    FP64 moments; returns the number of values that differ (each must be one
    unit in the last place of its format at most)."""
    Ds, _ = T.export_stored()
    got = ex_mom.astype(np.float64)
    diff = got != Ds
    fmt = np.where(levels[:, None, None] <= FP32_LEVELS, 0, 1) if storage == "bf16" else np.zeros_like(levels)[:, None, None]
    fmt = np.broadcast_to(fmt, Ds.shape)
    ulp = np.where(fmt == 0, _ulp(Ds, "fp32"), _ulp(Ds, "bf16"))
    assert np.all(np.abs(got - Ds) <= ulp * (1 + 1e-12)), "stored moment off by more than one unit"
    return int(diff.sum())


def _build(P, orc, name, storage):
    gen, leaf = CLOUDS[name]
    p, n, A, mu = gen()
    tree = P.dps_build(*to_dev(p, n, A, mu), leaf_size=leaf, storage=storage)
    T = orc.Tree(p, n, A, mu, leaf)
    T.set_storage(storage, FP32_LEVELS)
    return (p, n, A, mu), tree, T


@pytest.mark.parametrize("storage", ["fp32", "bf16"])
@pytest.mark.parametrize("name", sorted(CLOUDS))
def test_moments_rounded_as_stored(P, orc, name, storage):
    (p, n, A, mu), tree, T = _build(P, orc, name, storage)
    ex = P.dps_export_tree(tree)
    levels = to_host(ex["nodes"])[:, 0]
    flips = _stored_flips(to_host(ex["moments"]), T, storage, levels)
    total = ex["moments"].numel()
    print(f"[storage] {name} {storage}: {flips} of {total} stored moments differ by one unit from the oracle's "
          f"rounding; nodes of depth <= {FP32_LEVELS}: {int((levels <= FP32_LEVELS).sum())} of {levels.size}",
          flush=True)
    assert flips <= max(1, total // 10000)
    # after a refit with new attributes the stored copy follows
    mu2 = np.random.default_rng(5).standard_normal(mu.shape).astype(np.float32)
    (mu2d,) = to_dev(mu2)
    P.dps_set_attributes(tree, mu2d)
    T.set_attrs(mu2)
    ex = P.dps_export_tree(tree)
    flips2 = _stored_flips(to_host(ex["moments"]), T, storage, levels)
    assert flips2 <= max(1, total // 10000)


def _report(tag, err, got, ref):
    mx = float(err.max()) if err.size else 0.0
    print(f"[storage] {tag}: max {mx:.3g}, 99.9th pct {float(np.percentile(err, 99.9)) if err.size else 0:.3g}, "
          f"normwise {normwise(got, ref):.3g}", flush=True)
    return mx


def _check_emulated(err, flips, tag):
    """At the FP32 bar against the emulated store; with rounding-boundary
    flips in the stored moments, the few results that use a flipped moment may
    carry up to one unit of its format (and stay inside the BF16 bound)."""
    over = int((err > TOL_FP32).sum())
    print(f"[storage] {tag}: {over} of {err.size} results above {TOL_FP32:g} with {flips} flipped moments",
          flush=True)
    if flips == 0:
        assert over == 0
    else:
        assert over <= max(1, err.size // 100) and float(err.max()) <= TOL_BF16


@pytest.mark.parametrize("eps", [0.05, 0.0])
@pytest.mark.parametrize("name", sorted(CLOUDS))
def test_bf16_against_emulated_storage(P, orc, name, eps):
    (p, n, A, mu), tree, T = _build(P, orc, name, "bf16")
    ex = P.dps_export_tree(tree)
    flips = _stored_flips(to_host(ex["moments"]), T, "bf16", to_host(ex["nodes"])[:, 0])
    Q, C = 4099, mu.shape[1]
    x = workloads.sphere_queries(Q, 2)
    x = np.concatenate([x, p[:61]])  # queries exactly at points
    Q = x.shape[0]
    df = workloads.cotangents(Q, C, 17)
    dg = np.random.default_rng(18).standard_normal((Q, C, 3)).astype(np.float32)
    xd, dfd, dgd = to_dev(x, df, dg)
    f, g = P.dps_query(tree, xd, 2.0, eps)
    ref = T.query(x, 2.0, eps)
    assert np.array_equal(to_host(P.dps_query_counts(tree, xd, 2.0)), ref["counts"])
    ef = norm_err_all(to_host(f), ref["f"], ref["sf"])
    eg = norm_err_all(to_host(g), ref["g"], ref["sg"])
    _report(f"{name} eps={eps} f", ef, to_host(f), ref["f"])
    _report(f"{name} eps={eps} grad", eg, to_host(g), ref["g"])
    _check_emulated(ef, flips, f"{name} eps={eps} f")
    _check_emulated(eg, flips, f"{name} eps={eps} grad")
    # value adjoint: dL/dmu does not read stored values; dL/dx does
    dattrs, dx = P.dps_adjoint(tree, xd, 2.0, eps, dfd)
    adj = T.adjoint(x, 2.0, eps, df)
    e1 = norm_err_all(to_host(dattrs), adj["dmu"], adj["sdmu"])
    e2 = norm_err_all(to_host(dx), adj["dx"], adj["sdx"])
    _report(f"{name} eps={eps} adjoint dmu", e1, to_host(dattrs), adj["dmu"])
    _report(f"{name} eps={eps} adjoint dx", e2, to_host(dx), adj["dx"])
    assert e1.max() <= TOL_FP32
    _check_emulated(e2, flips, f"{name} eps={eps} adjoint dx")
    # gradient cotangents (Hessian adjoint)
    P.dps_adjoint_zero(tree)
    dxg = P.dps_adjoint_accumulate_grad(tree, xd, 2.0, eps, dgd, df=dfd)
    dag = P.dps_adjoint_finalize(tree)
    adg = T.adjoint(x, 2.0, eps, df, dg=dg)
    e3 = norm_err_all(to_host(dag), adg["dmu"], adg["sdmu"])
    e4 = norm_err_all(to_host(dxg), adg["dx"], adg["sdx"])
    _report(f"{name} eps={eps} grad-cotangent dmu", e3, to_host(dag), adg["dmu"])
    _report(f"{name} eps={eps} grad-cotangent dx", e4, to_host(dxg), adg["dx"])
    _check_emulated(e3, flips, f"{name} eps={eps} grad-cotangent dmu")
    _check_emulated(e4, flips, f"{name} eps={eps} grad-cotangent dx")
    P.dps_check(tree)


@pytest.mark.parametrize("eps", [0.05, 0.0])
@pytest.mark.parametrize("name", sorted(CLOUDS))
def test_fp32_at_moment_scale(P, orc, name, eps):
    """FP32 storage against the exact oracle with each node term scaled by
    |D_t| (not its absolute mass): holds because the stored moments are the
    FP64 moments rounded once."""
    (p, n, A, mu), tree, T = _build(P, orc, name, "fp32")
    T.set_storage("exact")
    T.set_scale("moment")
    Q, C = 4099, mu.shape[1]
    x = np.concatenate([workloads.sphere_queries(Q, 2), p[:61]])
    Q = x.shape[0]
    df = workloads.cotangents(Q, C, 17)
    xd, dfd = to_dev(x, df)
    f, g = P.dps_query(tree, xd, 2.0, eps)
    ref = T.query(x, 2.0, eps)
    ef = norm_err_all(to_host(f), ref["f"], ref["sf"])
    eg = norm_err_all(to_host(g), ref["g"], ref["sg"])
    _report(f"{name} eps={eps} fp32 |D_t|-scale f", ef, to_host(f), ref["f"])
    _report(f"{name} eps={eps} fp32 |D_t|-scale grad", eg, to_host(g), ref["g"])
    assert ef.max() <= TOL_FP32 and eg.max() <= TOL_FP32
    dattrs, dx = P.dps_adjoint(tree, xd, 2.0, eps, dfd)
    adj = T.adjoint(x, 2.0, eps, df)
    e2 = norm_err_all(to_host(dx), adj["dx"], adj["sdx"])
    _report(f"{name} eps={eps} fp32 |D_t|-scale adjoint dx", e2, to_host(dx), adj["dx"])
    assert e2.max() <= TOL_FP32
