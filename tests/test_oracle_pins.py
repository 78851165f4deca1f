"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test ties a part of the oracle to something other than its own formulas:
library distributions (chi, noncentral chi-square), closed forms derived from
the paper's propositions, worked values, finite differences, transposition,
Monte Carlo, brute force.  A dropped 1/(4 pi), a flipped sign of d = p - x, a
wrong rho convention or a transposed operand fails at least one of them.
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.stats as st

import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")


# --------------------------------------------------------------------------
# radial functions
# --------------------------------------------------------------------------
def test_rho_series_equals_closed_form(orc):
    # the two branches are independent expressions of rho (Sec. 4.1)
    for t in (0.05, 0.2, 0.35, 0.5, 0.65, 0.8):
        assert abs(orc.rho_series(t) - orc.rho_closed(t)) <= 2e-14 * max(1.0, orc.rho_closed(t)) + 1e-15


def test_rho_is_chi3_cdf(orc):
    # Prop. 2 (App. A.2): the regularized kernel is the point-cloud kernel
    # averaged over Gaussian position noise; for isotropic noise of per-axis
    # variance eps^2/2 the average of the Coulomb field of a point is the field
    # of the mass within radius r, i.e. the chi(3) CDF at r/(eps/sqrt 2).
    for t in np.linspace(0.01, 4.0, 41):
        assert abs(orc.rho(t) - st.chi(3).cdf(math.sqrt(2.0) * t)) < 1e-12


def test_psi_definition(orc):
    # psi(t) = 3 rho(t) - t rho'(t), rho' by central differences of the oracle
    for t in (0.1, 0.4, 0.6, 1.0, 2.0, 3.0):
        h = 1e-5
        d = (orc.rho(t + h) - orc.rho(t - h)) / (2 * h)
        assert abs(orc.psi(t) - (3 * orc.rho(t) - t * d)) < 1e-8


def test_kernel_limit_matches_paper_constant(orc):
    # Sec. 4.1 prints the finite value 3^-1 eps^-3 pi^-3/2 of the regularized
    # kernel at coincident points (reading: the coefficient kappa(0))
    g = json.load(open(GOLDEN))["kernel_value_at_coincidence"]["coefficient_times_eps3"]
    for eps in (0.01, 0.05, 1.0):
        kap, lam = orc.radial(0.0, eps)
        assert abs(kap * eps ** 3 - g) < 1e-14
        assert abs(kap * eps ** 3 - 1.0 / (3.0 * math.pi ** 1.5)) < 1e-14


def test_unregularized_limit(orc):
    # eps = 0 is the classic dipole (rho = 1, psi = 3), Sec. 3.2 eq. (wn)
    for r in (0.1, 1.0, 3.0):
        kap, lam = orc.radial(r, 0.0)
        assert kap == pytest.approx(1.0 / (4 * math.pi * r ** 3), rel=1e-15)
        assert lam == pytest.approx(3.0 / (4 * math.pi * r ** 5), rel=1e-15)
    # and far from the source the regularized kernel tends to it
    kap, lam = orc.radial(1.0, 0.05)
    assert kap == pytest.approx(1.0 / (4 * math.pi), rel=1e-12)


# --------------------------------------------------------------------------
# direct sum
# --------------------------------------------------------------------------
def test_single_source_worked_example(orc):
    # p = (0,0,1), n = (0,0,1), A = 4 pi, mu = 1, x = 0, eps = 0:
    # f = A n.(p-x) / (4 pi |p-x|^3) = 1; along z, f(z) = 1/(1-z)^2 so
    # df/dz = 2 at z = 0 and the transverse derivatives vanish.
    p = np.array([[0, 0, 1]], np.float32)
    n = np.array([[0, 0, 1]], np.float32)
    A = np.array([4 * math.pi], np.float32)
    mu = np.ones((1, 1), np.float32)
    r = orc.direct(p, n, A, mu, np.zeros((1, 3), np.float32), 0.0)
    assert r["f"][0, 0] == pytest.approx(float(np.float32(4 * math.pi)) / (4 * math.pi), rel=1e-12)
    assert np.allclose(r["g"][0, 0], [0, 0, 2 * float(np.float32(4 * math.pi)) / (4 * math.pi)], atol=1e-12)


def _wsphere(a, R, eps):
    # indicator of the ball of radius R blurred by an isotropic Gaussian of
    # per-axis variance eps^2/2: P(|a e + Z| < R) via the noncentral chi-square
    s2 = eps * eps / 2.0
    return st.ncx2.cdf(R * R / s2, 3, a * a / s2)


@pytest.mark.parametrize("eps", [0.05, 0.1])
def test_sphere_closed_form(orc, eps):
    # Prop. 1: the regularized winding number solves the Poisson problem whose
    # solution for a closed surface is its indicator convolved with the
    # Gaussian; a dense Fibonacci sphere approximates the continuous surface
    p, n, A = workloads.fibonacci_sphere(40000)
    mu = np.ones((p.shape[0], 1), np.float32)
    radii = np.array([0.0, 0.3, 0.7, 0.9, 0.97, 1.0, 1.03, 1.1, 1.3, 2.0])
    x = np.zeros((radii.size, 3), np.float32)
    d = np.array([0.3, -0.5, 0.81])
    d /= np.linalg.norm(d)
    x[:] = (radii[:, None] * d[None, :]).astype(np.float32)
    got = orc.direct(p, n, A, mu, x, eps)["f"][:, 0]
    for a, v in zip(np.linalg.norm(x.astype(np.float64), axis=1), got):
        assert abs(v - _wsphere(a, 1.0, eps)) < 2e-3, (a, v, _wsphere(a, 1.0, eps))


def test_gauss_lemma_unregularized(orc):
    # Sec. 3.2, eq. (gauss): winding number 1 inside, 0 outside (eps = 0)
    g = json.load(open(GOLDEN))["gauss_lemma"]
    p, n, A = workloads.fibonacci_sphere(40000)
    mu = np.ones((p.shape[0], 1), np.float32)
    on, ins, out = workloads.sphere_probes(64, 3)
    fi = orc.direct(p, n, A, mu, ins, 0.0)["f"][:, 0]
    fo = orc.direct(p, n, A, mu, out, 0.0)["f"][:, 0]
    assert np.all(np.abs(fi - g["inside"]) < 2e-3)
    assert np.all(np.abs(fo - g["outside"]) < 2e-3)


def test_gauss_lemma_random_sphere(orc):
    # config sphere-8k: random points are an unbiased quadrature; 6 sigma bound
    p, n, A, mu = workloads.sphere_cloud(8192, 1)
    on, ins, out = workloads.sphere_probes(256, 3)
    for x, want in ((ins, 1.0), (out, 0.0)):
        f = orc.direct(p, n, A, mu[:, :1], x, 0.0)["f"][:, 0]
        # per-term spread: each term is A P(x, p_m); sigma of the mean estimate
        d = p[None, :, :].astype(np.float64) - x[:, None, :].astype(np.float64)
        r = np.linalg.norm(d, axis=2)
        terms = np.sum(d * n[None].astype(np.float64), axis=2) / (4 * math.pi * r ** 3) * 4 * math.pi
        sig = terms.std(axis=1) / math.sqrt(p.shape[0])
        assert np.all(np.abs(f - want) <= 6 * sig + 1e-9)
    # on the surface, eps > 0: 1/2 - eps/(2 sqrt(pi) R) to first order, and the
    # exact blurred-indicator value at a = R
    f = orc.direct(p, n, A, mu[:, :1], on, 0.05)["f"][:, 0]
    assert abs(np.mean(f) - _wsphere(1.0, 1.0, 0.05)) < 5e-3


def test_centre_of_unit_sphere_exact(orc):
    # every term at x = 0 equals rho(1/eps) mu_m / N (n = p, |p| = 1, A = 4 pi / N)
    p, n, A, mu = workloads.sphere_cloud(4096, 1)
    eps = 0.3
    r = orc.direct(p, n, A, mu, np.zeros((1, 3), np.float32), eps)
    pd = p.astype(np.float64)
    rr = np.linalg.norm(pd, axis=1)
    # exact up to the FP32 rounding of |p| = 1: use the true radii
    want = np.array([np.sum(A.astype(np.float64) * orc_rho_vec(orc, rr / eps) * mu[:, c] / (4 * math.pi * rr ** 2))
                     for c in range(mu.shape[1])])
    assert np.allclose(r["f"][0], want, rtol=1e-12)
    assert np.allclose(r["f"][0], orc.rho(1 / eps) * mu.astype(np.float64).mean(0), rtol=2e-6)
    gw = -(orc.rho(1 / eps) - orc.psi(1 / eps)) * (mu.astype(np.float64)[:, :, None] * pd[:, None, :]).mean(0)
    assert np.allclose(r["g"][0], gw, rtol=1e-4, atol=1e-7)


def orc_rho_vec(orc, t):
    return np.array([orc.rho(v) for v in t])


def test_gradient_matches_finite_differences(orc):
    # grad_x of eq. (dipole_sum) against central differences of the values
    p, n, A, mu = workloads.sfm_cloud(3000, 200, 10)
    x = workloads.sphere_queries(40, 5, half=1.0).astype(np.float64)
    h = 2.0 ** -14
    for eps in (0.05, 0.0):
        r = orc.direct(p, n, A, mu, x.astype(np.float32), eps)
        for k in range(3):
            xp, xm = x.copy(), x.copy()
            xp[:, k] += h
            xm[:, k] -= h
            xp32, xm32 = xp.astype(np.float32), xm.astype(np.float32)
            fp = orc.direct(p, n, A, mu, xp32, eps)["f"]
            fm = orc.direct(p, n, A, mu, xm32, eps)["f"]
            dxk = xp32[:, k].astype(np.float64) - xm32[:, k].astype(np.float64)
            fd = (fp - fm) / dxk[:, None]
            assert np.max(np.abs(fd - r["g"][:, :, k]) / r["sg"]) < 1e-4


def test_linearity_in_attributes(orc):
    p, n, A, mu = workloads.sfm_cloud(2000, 100, 10)
    nu = np.random.default_rng(4).standard_normal(mu.shape).astype(np.float32)
    a, b = 0.75, -1.25
    x = workloads.sphere_queries(50, 6, half=1.0)
    lhs = orc.direct(p, n, A, (a * mu.astype(np.float64) + b * nu).astype(np.float32), x, 0.02)
    f1 = orc.direct(p, n, A, mu, x, 0.02)["f"]
    f2 = orc.direct(p, n, A, nu, x, 0.02)["f"]
    comb = (a * mu.astype(np.float64) + b * nu).astype(np.float32).astype(np.float64)
    # exact linearity holds for the attributes actually passed (FP32-rounded)
    lin = orc.direct(p, n, A, comb.astype(np.float32), x, 0.02)["f"]
    assert np.allclose(lhs["f"], lin, rtol=0, atol=0)
    assert np.max(np.abs(lhs["f"] - (a * f1 + b * f2)) / lhs["sf"]) < 1e-6
    T = orc.Tree(p, n, A, mu, 16)
    g1 = T.query(x, 2.0, 0.02)["f"]
    T.set_attrs(nu)
    g2 = T.query(x, 2.0, 0.02)["f"]
    T.set_attrs(np.float32(a) * mu + np.float32(b) * nu)
    g3 = T.query(x, 2.0, 0.02)
    assert np.max(np.abs(g3["f"] - (a * g1 + b * g2)) / g3["sf"]) < 1e-6


def test_direct_adjoint_is_transpose(orc):
    p, n, A, mu = workloads.sfm_cloud(1500, 100, 10)
    x = workloads.sphere_queries(300, 7, half=1.0)
    df = workloads.cotangents(300, mu.shape[1], 17)
    eps = 0.02
    f = orc.direct(p, n, A, mu, x, eps)["f"]
    dmu, dx = orc.direct_adjoint(p, n, A, mu, x, eps, df)
    lhs = np.sum(df.astype(np.float64) * f)
    rhs = np.sum(dmu * mu.astype(np.float64))
    assert abs(lhs - rhs) <= 1e-12 * np.sum(np.abs(df.astype(np.float64) * f)) + 1e-14
    # dL/dx with L = sum df . f equals sum_c df_c grad f_c
    g = orc.direct(p, n, A, mu, x, eps)["g"]
    assert np.allclose(dx, np.einsum("qc,qck->qk", df.astype(np.float64), g), rtol=1e-10, atol=1e-12)


def test_numpy_crosscheck_tiny(orc):
    # an independent NumPy/scipy evaluation of eq. (dipole_sum) on a tiny input
    from scipy.special import erf
    rng = np.random.default_rng(9)
    M, Q, C, eps = 40, 25, 3, 0.3
    p = rng.uniform(-1, 1, (M, 3)).astype(np.float32)
    n = rng.standard_normal((M, 3))
    n = (n / np.linalg.norm(n, axis=1, keepdims=True)).astype(np.float32)
    A = rng.uniform(0.01, 0.1, M).astype(np.float32)
    mu = rng.standard_normal((M, C)).astype(np.float32)
    x = rng.uniform(-1, 1, (Q, 3)).astype(np.float32)
    d = p[None].astype(np.float64) - x[:, None].astype(np.float64)
    r = np.linalg.norm(d, axis=2)
    t = r / eps
    rho = erf(t) - 2 * t / math.sqrt(math.pi) * np.exp(-t * t)
    w = A[None] * rho * np.sum(n[None] * d, axis=2) / (4 * math.pi * r ** 3)
    want = w @ mu.astype(np.float64)
    got = orc.direct(p, n, A, mu, x, eps)["f"]
    assert np.allclose(got, want, rtol=1e-10, atol=1e-13)


def test_scale_invariance(orc):
    # scaling p, x, eps by s and A by s^2 leaves every term unchanged
    p, n, A, mu = workloads.sfm_cloud(1000, 50, 10)
    x = workloads.sphere_queries(30, 8, half=1.0)
    s = 2.0  # power of two: the scaling is exact in FP32
    f1 = orc.direct(p, n, A, mu, x, 0.03)["f"]
    f2 = orc.direct(p * s, n, A * s * s, mu, x * s, 0.03 * s)["f"]
    assert np.allclose(f1, f2, rtol=1e-12, atol=1e-14)


def test_prop2_monte_carlo(orc):
    # Prop. 2 (App. A.2): the regularized sum equals the expected unregularized
    # winding number of a point cloud with Gaussian position noise of per-axis
    # variance eps^2/2 and mean normal mu_m n_m.
    rng = np.random.default_rng(21)
    M, eps, K = 4, 0.2, 400000
    p = rng.uniform(-0.3, 0.3, (M, 3))
    n = rng.standard_normal((M, 3))
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    A = rng.uniform(0.5, 1.0, M)
    mu = rng.uniform(0.2, 1.0, M)
    x = np.array([[0.55, -0.1, 0.2], [-0.5, 0.45, -0.3]])
    want = orc.direct(p.astype(np.float32), n.astype(np.float32), A.astype(np.float32),
                      mu.astype(np.float32)[:, None], x.astype(np.float32), eps)["f"][:, 0]
    sig = eps / math.sqrt(2.0)
    est = np.zeros(len(x))
    for m in range(M):
        y = p[m] + sig * rng.standard_normal((K, 3))
        for q in range(len(x)):
            d = y - x[q]
            r = np.linalg.norm(d, axis=1)
            est[q] += np.mean(A[m] * mu[m] * (d @ n[m]) / (4 * math.pi * r ** 3))
    # the alternative reading (per-axis variance eps^2) is far off
    assert np.all(np.abs(est - want) < 0.01 * np.abs(want).max() + 2e-3), (est, want)


# --------------------------------------------------------------------------
# canonical octree
# --------------------------------------------------------------------------
def _check_tree(orc, p, A, leaf):
    from fractions import Fraction
    T = orc.Tree(p, p, A, None, leaf)
    e = T.export()
    M = p.shape[0]
    lo = p.min(axis=0)
    side = float(max(float(p[:, k].max()) - float(lo[k]) for k in range(3))) or 1.0
    # Morton code of each point from exact rational arithmetic; FP64 rounding of
    # (p - lo) * scale can only move a cell index across an exact boundary
    for i in np.random.default_rng(0).choice(M, size=min(M, 300), replace=False):
        code = int(e["codes_in"][i])
        for k, sh in ((0, 2), (1, 1), (2, 0)):
            q = 0
            for b in range(21):
                q |= ((code >> (3 * b + sh)) & 1) << b
            v = (Fraction(float(p[i, k])) - Fraction(float(lo[k]))) * (2 ** 21) / Fraction(side)
            fl = min(int(v), 2 ** 21 - 1)
            assert abs(q - fl) <= 1 or (q == fl)
            if v.denominator == 1 or abs(v - round(v)) > Fraction(1, 10 ** 6):
                assert q == fl
    codes, perm, nodes, geom = e["codes"], e["perm"], e["nodes"], e["geom"]
    assert np.all(np.diff(codes.astype(object)) >= 0)
    assert np.array_equal(codes, e["codes_in"][perm])
    # ties keep the input order (stable sort)
    same = codes[1:] == codes[:-1]
    assert np.all(perm[1:][same] > perm[:-1][same])
    assert sorted(perm.tolist()) == list(range(M))
    N = nodes.shape[0]
    assert nodes[0].tolist()[:2] == [0, -1] and nodes[0, 4] == 0 and nodes[0, 5] == M
    for t in range(N):
        lvl, par, fc, nc, b, c = nodes[t].tolist()
        if nc == 0:
            assert c <= leaf or lvl == 21
        else:
            assert c > leaf and lvl < 21
            ch = nodes[fc:fc + nc]
            assert np.all(ch[:, 1] == t) and np.all(ch[:, 0] == lvl + 1)
            assert ch[0, 4] == b and int(ch[:, 5].sum()) == c
            assert np.all(ch[1:, 4] == ch[:-1, 4] + ch[:-1, 5])
            sh = 3 * (20 - lvl)
            dig = [(int(codes[k[4]]) >> sh) & 7 for k in ch]
            assert dig == sorted(set(dig))
        pref = codes[b:b + c] >> np.uint64(3 * (21 - lvl))
        assert np.all(pref == pref[0])
        # node geometry, eq. (farfield_dipole): area-weighted centroid and radius
        pts = p[perm[b:b + c]].astype(np.float64)
        w = A[perm[b:b + c]].astype(np.float64)
        cen = (w[:, None] * pts).sum(0) / w.sum()
        assert np.allclose(geom[t, :3], cen, rtol=0, atol=4e-7 * (1 + np.abs(cen).max()))
        d2 = ((pts - geom[t, :3].astype(np.float64)) ** 2).sum(1).max()
        assert abs(geom[t, 3] - d2) <= 1e-6 * max(d2, 1e-30) + 1e-12
        assert e["area"][t] == pytest.approx(w.sum(), rel=1e-12)
    # breadth-first numbering: levels non-decreasing, parents in order
    assert np.all(np.diff(nodes[:, 0]) >= 0)
    assert np.all(np.diff(nodes[1:, 1]) >= 0)
    return T


@pytest.mark.parametrize("M,leaf", [(1, 16), (2, 1), (17, 16), (500, 1), (3000, 16), (3000, 5)])
def test_tree_invariants_random(orc, M, leaf):
    rng = np.random.default_rng(M)
    p = rng.uniform(-1, 1, (M, 3)).astype(np.float32)
    A = rng.uniform(0.1, 1.0, M).astype(np.float32)
    _check_tree(orc, p, A, leaf)


def test_tree_duplicates_reach_level_21(orc):
    # identical points cannot be separated: the leaf sits at level 21
    p = np.zeros((40, 3), np.float32)
    p[20:] = [1e-3, 0, 0]
    A = np.ones(40, np.float32)
    T = _check_tree(orc, p, A, 16)
    e = T.export()
    assert e["nodes"][:, 0].max() == 21


def test_tree_moments_are_point_sums(orc):
    p, n, A, mu = workloads.sfm_cloud(3000, 100, 10)
    T = orc.Tree(p, n, A, mu, 16)
    e = T.export()
    D = e["D"]
    for t in np.random.default_rng(1).choice(T.N, 200, replace=False):
        b, c = e["nodes"][t, 4], e["nodes"][t, 5]
        idx = e["perm"][b:b + c]
        want = np.einsum("m,mc,mk->ck", A[idx].astype(np.float64), mu[idx].astype(np.float64),
                         n[idx].astype(np.float64))
        assert np.allclose(D[t], want, rtol=1e-12, atol=1e-15)


# --------------------------------------------------------------------------
# Barnes-Hut traversal
# --------------------------------------------------------------------------
def test_bh_converges_to_direct(orc):
    # Algorithm 1 / Sec. 6.1: larger beta opens more nodes; once beta exceeds
    # every distance/radius ratio along the way, BH is the direct sum.
    p, n, A, mu = workloads.sfm_cloud(4000, 200, 10)
    x = workloads.sphere_queries(200, 9, half=1.0)
    d = orc.direct(p, n, A, mu, x, 0.02)
    T = orc.Tree(p, n, A, mu, 16)
    errs = []
    for beta in (1.0, 2.0, 4.0, 8.0):
        b = T.query(x, beta, 0.02)
        errs.append(np.mean(np.abs(b["f"] - d["f"]) / d["sf"]))
    assert errs[0] > errs[1] > errs[2] > errs[3]
    b = T.query(x, 1e4, 0.02)
    assert np.max(np.abs(b["f"] - d["f"]) / d["sf"]) < 1e-12
    assert np.max(np.abs(b["g"] - d["g"]) / d["sg"][..., None]) < 1e-12
    # only zero-radius nodes (single points) can still be far: their term is exact
    n_zero = int(np.sum(T.export()["geom"][:, 3] == 0.0))
    assert np.all(b["counts"][:, 1] <= n_zero)


def test_bh_single_point_leaf_is_exact(orc):
    # a leaf holding one point has r = 0, so its far-field term is exact
    p, n, A, mu = workloads.sfm_cloud(800, 40, 10)
    x = workloads.sphere_queries(100, 10, half=1.0)
    T = orc.Tree(p, n, A, mu, 1)
    d = orc.direct(p, n, A, mu, x, 0.0)
    b = T.query(x, 1e-6, 0.0)  # tiny beta: every node is far field at once
    assert np.all(b["counts"][:, 0] == 1)
    T2 = orc.Tree(p[:1], n[:1], A[:1], mu[:1], 1)
    assert np.allclose(T2.query(x, 2.0, 0.0)["f"], orc.direct(p[:1], n[:1], A[:1], mu[:1], x, 0.0)["f"],
                       rtol=1e-12)
    assert d is not None


def test_bh_adjoint_is_transpose(orc):
    p, n, A, mu = workloads.sfm_cloud(4000, 200, 10)
    x = workloads.sphere_queries(500, 11, half=1.0)
    df = workloads.cotangents(500, mu.shape[1], 17)
    T = orc.Tree(p, n, A, mu, 16)
    for beta in (1.0, 2.0):
        f = T.query(x, beta, 0.02)["f"]
        a = T.adjoint(x, beta, 0.02, df)
        lhs = np.sum(df.astype(np.float64) * f)
        rhs = np.sum(a["dmu"] * mu.astype(np.float64))
        assert abs(lhs - rhs) <= 1e-12 * np.sum(np.abs(df * f))
        g = T.query(x, beta, 0.02)["g"]
        assert np.allclose(a["dx"], np.einsum("qc,qck->qk", df.astype(np.float64), g), rtol=1e-10, atol=1e-13)


def test_bh_adjoint_matches_direct_adjoint_at_large_beta(orc):
    p, n, A, mu = workloads.sfm_cloud(1500, 50, 10)
    x = workloads.sphere_queries(200, 12, half=1.0)
    df = workloads.cotangents(200, mu.shape[1], 17)
    T = orc.Tree(p, n, A, mu, 16)
    a = T.adjoint(x, 1e4, 0.02, df)
    dmu, dx = orc.direct_adjoint(p, n, A, mu, x, 0.02, df)
    assert np.allclose(a["dmu"], dmu, rtol=1e-10, atol=1e-14)
    assert np.allclose(a["dx"], dx, rtol=1e-10, atol=1e-14)


def test_bh_adjoint_dx_matches_finite_differences(orc):
    # L = sum df . f_BH; away from decision boundaries f_BH is smooth in x
    p, n, A, mu = workloads.sfm_cloud(3000, 100, 10)
    T = orc.Tree(p, n, A, mu, 16)
    x = workloads.sphere_queries(60, 13, half=1.0).astype(np.float64)
    df = workloads.cotangents(60, mu.shape[1], 17).astype(np.float64)
    a = T.adjoint(x.astype(np.float32), 2.0, 0.05, df.astype(np.float32))
    h = 2.0 ** -14
    base = T.query(x.astype(np.float32), 2.0, 0.05)
    checked = 0
    for k in range(3):
        xp, xm = x.copy(), x.copy()
        xp[:, k] += h
        xm[:, k] -= h
        rp = T.query(xp.astype(np.float32), 2.0, 0.05)
        rm = T.query(xm.astype(np.float32), 2.0, 0.05)
        same = np.all(rp["counts"] == base["counts"], axis=1) & np.all(rm["counts"] == base["counts"], axis=1)
        dxk = (xp[:, k].astype(np.float32).astype(np.float64) - xm[:, k].astype(np.float32).astype(np.float64))
        fd = np.sum(df * (rp["f"] - rm["f"]), axis=1) / dxk
        scale = np.sum(np.abs(df) * base["sg"], axis=1)
        assert np.all(np.abs(fd - a["dx"][:, k])[same] / scale[same] < 1e-3)
        checked += int(same.sum())
    assert checked > 100


def test_visits_grow_logarithmically(orc):
    # Sec. 6.1 / 6.2: O(log M) work per query
    x = workloads.sphere_queries(400, 14, half=1.5)
    v = []
    for M in (4096, 16384, 65536, 262144):
        p, n, A, mu = workloads.sphere_cloud(M, 1)
        T = orc.Tree(p, n, A, mu[:, :1], 16)
        v.append(T.query(x, 2.0, 0.05, want_grad=False)["counts"][:, 0].mean())
    inc = np.diff(v)
    assert np.all(inc > 0)
    # additive growth per factor 4 of M, far below linear growth
    assert v[-1] / v[0] < 3.0
    assert inc.max() < 2.0 * inc.min() + 40


def test_far_test_worked_example(orc):
    # Algorithm 1 / Sec. 6.1: two points of equal area at (+-0.5, 0, 0), leaf
    # size 1.  The root has centroid 0 and radius 0.5, so with beta = 2 it is a
    # far field iff |x| > 1; its children are single-point leaves (radius 0),
    # which the far test (evaluated before the leaf test) always accepts.
    p = np.array([[-0.5, 0, 0], [0.5, 0, 0]], np.float32)
    n = np.array([[0, 0, 1], [0, 1, 0]], np.float32)
    A = np.ones(2, np.float32)
    mu = np.ones((2, 1), np.float32)
    T = orc.Tree(p, n, A, mu, 1)
    e = T.export()
    assert e["nodes"].shape[0] == 3
    assert np.allclose(e["geom"][0], [0, 0, 0, 0.25])
    x = np.array([[0, 1.01, 0], [0, 0.99, 0], [0, 0, 1.0], [-1.001, 0, 0]], np.float32)
    c = T.query(x, 2.0, 0.0)["counts"]
    assert c[0].tolist() == [1, 1, 0, 0]   # root accepted as far field
    assert c[1].tolist() == [3, 2, 0, 0]   # root opened, both leaves far
    assert c[2].tolist() == [3, 2, 0, 0]   # |x| = beta r exactly: not far (strict)
    assert c[3].tolist() == [1, 1, 0, 0]
    # the far-field term of the root is the dipole of the summed moment at the
    # centroid (eq. farfield); each single-point leaf term is exact
    r = T.query(x[:2], 2.0, 0.0)
    D = np.array([0.0, 1.0, 1.0])  # sum of A n mu
    d0 = -x[0].astype(np.float64)
    assert r["f"][0, 0] == pytest.approx(D @ d0 / (4 * math.pi * np.linalg.norm(d0) ** 3), rel=1e-12)
    assert r["f"][1, 0] == pytest.approx(orc.direct(p, n, A, mu, x[1:2], 0.0)["f"][0, 0], rel=1e-12)


def test_far_field_scale_is_the_absolute_mass(orc):
    # The error scale of a far-field node term is kappa r times the node's
    # absolute dipole mass sum_m |A_m mu_m n_m|, not |D_t|: two points whose
    # dipoles cancel exactly (D_t = 0) still give the scale of two unit
    # sources, while the value is 0.  With beta large enough to open the root
    # the scale is the direct sum's, each leaf being one point.
    p = np.array([[-0.5, 0, 0], [0.5, 0, 0]], np.float32)
    n = np.array([[0, 0, 1], [0, 0, 1]], np.float32)
    A = np.ones(2, np.float32)
    mu = np.array([[1.0], [-1.0]], np.float32)
    T = orc.Tree(p, n, A, mu, 1)
    x = np.array([[0, 3.0, 0]], np.float32)
    far = T.query(x, 2.0, 0.0)
    assert far["counts"][0].tolist() == [1, 1, 0, 0]
    assert far["f"][0, 0] == 0.0
    d = -x[0].astype(np.float64)
    r = np.linalg.norm(d)
    kap = 1.0 / (4 * math.pi * r ** 3)
    assert far["sf"][0, 0] == pytest.approx(kap * 2.0 * r, rel=1e-12)
    assert far["sg"][0, 0] == pytest.approx(2.0 * (kap + 3 * kap / r ** 2 * r ** 2), rel=1e-12)
    opened = T.query(x, 10.0, 0.0)
    direct = orc.direct(p, n, A, mu, x, 0.0)
    assert opened["counts"][0].tolist() == [3, 2, 0, 0]
    assert opened["sf"][0, 0] == pytest.approx(direct["sf"][0, 0], rel=1e-12)
    # the same for the monopole kernel: charges +1 and -1 cancel, scale 2 m(r)
    Tm = orc.Tree(p, n, A, mu, 1, kind="monopole")
    fm = Tm.query(x, 2.0, 0.0)
    assert fm["f"][0, 0] == 0.0
    assert fm["sf"][0, 0] == pytest.approx(2.0 / (4 * math.pi * r ** 2), rel=1e-12)
    # and in the adjoint: the dL/dx scale of the far node uses the mass too
    a = T.adjoint(x, 2.0, 0.0, np.ones((1, 1), np.float32))
    assert a["sdx"][0] == pytest.approx(2.0 * (kap + 3 * kap), rel=1e-12)


def test_bh_adjoint_through_render_loss_matches_fd(orc):
    # the oracle adjoint, driven by dL/df of the render proxy, against central
    # differences of the same loss: attributes perturbed through linearity,
    # sample positions perturbed and re-queried
    import torch
    from workloads.render import fd_linear, fd_position, loss_numpy, loss_torch
    p, n, A, mu = workloads.sfm_cloud(20000, 1000, 10)
    R, S, eps, h = 16, 64, 0.03, 1e-4
    pix, x = workloads.pixel_ray_samples(workloads.sfm_camera(11), 64, 64, S, 12, R, 14)
    target = np.random.default_rng(13).uniform(size=(R, 3))
    T = orc.Tree(p, n, A, mu, 16)
    base = T.query(x, 2.0, eps)
    f0 = base["f"]
    ft = torch.tensor(f0, requires_grad=True)
    loss_torch(ft, R, S, torch.tensor(target)).backward()
    df = ft.grad.numpy()
    adj = T.adjoint(x, 2.0, eps, df.astype(np.float32))
    loss = lambda ff: loss_numpy(ff, R, S, target)
    worst = 0.0
    for m in np.random.default_rng(15).choice(p.shape[0], 24, replace=False):
        e = np.zeros_like(mu)
        e[m] = 1.0
        T.set_attrs(e)
        fe = T.query(x, 2.0, eps, want_grad=False)["f"]
        for c in range(4):
            fd = fd_linear(f0, fe[:, c], c, loss, h)
            worst = max(worst, abs(adj["dmu"][m, c] - fd) / (adj["sdmu"][m, c] + 1e-300))
    assert worst < 1e-5
    T.set_attrs(mu)
    worst, used = 0.0, 0
    for q in np.random.default_rng(16).choice(x.shape[0], 24, replace=False):
        for k in range(3):
            fd = fd_position(T, x, f0, base["counts"], q, k, S, target, h, 2.0, eps)
            if fd is None:
                continue
            scale = np.sum(np.abs(df[q]) * base["sg"][q])
            worst = max(worst, abs(adj["dx"][q, k] - fd) / scale)
            used += 1
    assert used >= 36 and worst < 1e-4


# --------------------------------------------------------------------------
# gradient cotangents: the Hessian factor nu and the adjoint of grad D
# --------------------------------------------------------------------------
def test_chi_series_equals_closed_form(orc):
    # chi(t) = 5 psi(t) - t psi'(t): series branch vs erf / exp branch
    for t in (0.05, 0.2, 0.35, 0.5, 0.65, 0.8):
        ref = orc.chi(t) if t >= 0.5 else orc.chi_series(t)
        closed = 15 * orc.rho_closed(t) - 4 / math.sqrt(math.pi) * (5 * t ** 3 + 2 * t ** 5) * math.exp(-t * t)
        assert abs(orc.chi_series(t) - closed) <= 1e-12 * max(1e-3, abs(closed)) + 1e-15
        assert abs(ref - closed) <= 1e-12 * max(1e-3, abs(closed)) + 1e-15


def test_chi_definition(orc):
    # chi(t) = 5 psi(t) - t psi'(t), psi' by central differences of the oracle
    for t in (0.1, 0.4, 0.6, 1.0, 2.0, 3.0):
        h = 1e-5
        d = (orc.psi(t + h) - orc.psi(t - h)) / (2 * h)
        assert abs(orc.chi(t) - (5 * orc.psi(t) - t * d)) < 1e-8


def test_nu_is_minus_lambda_prime_over_r(orc):
    # the Hessian factor is nu = -lambda'(r)/r; lambda' by central differences
    for eps in (0.05, 0.0):
        for r in (0.01, 0.04, 0.07, 0.2, 1.0):
            h = r * 1e-5
            lp = (orc.radial(r + h, eps)[1] - orc.radial(r - h, eps)[1]) / (2 * h)
            nu = orc.radial_nu(r, eps)
            assert abs(nu + lp / r) <= 1e-6 * abs(nu)
    # coincident limit of the regularized kernel, and the unregularized r^-7 law
    assert abs(orc.radial_nu(0.0, 0.05) * 4 * math.pi * 0.05 ** 7 - 16 / (7 * math.sqrt(math.pi))) < 1e-13
    assert abs(orc.radial_nu(2.0, 0.0) - 15 / (4 * math.pi * 2.0 ** 7)) < 1e-15


def _axis_cotangents(Q, C, k, seed):
    """dg[q,c,:] = a_qc e_k with a ~ N(0,1)."""
    a = np.random.default_rng(seed).standard_normal((Q, C))
    dg = np.zeros((Q, C, 3), np.float32)
    dg[:, :, k] = a
    return dg


def test_direct_grad_cotangent_dx_is_hessian(orc):
    # with dg = a e_k, dL/dx = sum_c a_c d(grad f_c)/dx_k: central differences
    # of the (pinned) gradient along axis k
    p, n, A, mu = workloads.sfm_cloud(2000, 100, 10)
    x = workloads.sphere_queries(40, 5, half=1.0).astype(np.float64)
    h = 2.0 ** -14
    for eps in (0.05, 0.0):
        for k in range(3):
            dg = _axis_cotangents(40, mu.shape[1], k, 30 + k)
            _, dx = orc.direct_adjoint(p, n, A, mu, x.astype(np.float32), eps, None, dg=dg)
            xp, xm = x.copy(), x.copy()
            xp[:, k] += h
            xm[:, k] -= h
            xp32, xm32 = xp.astype(np.float32), xm.astype(np.float32)
            gp = orc.direct(p, n, A, mu, xp32, eps)["g"]
            gm = orc.direct(p, n, A, mu, xm32, eps)["g"]
            dxk = xp32[:, k].astype(np.float64) - xm32[:, k].astype(np.float64)
            fd = np.einsum("qc,qcj->qj", dg[:, :, k].astype(np.float64), gp - gm) / dxk[:, None]
            scale = np.max(np.abs(fd), axis=1, keepdims=True) + 1e-9
            assert np.max(np.abs(fd - dx) / scale) < 1e-4


def test_direct_grad_cotangent_dmu_is_transpose(orc):
    # grad f is linear in mu: <dg, g(mu)> = <dmu, mu>
    p, n, A, mu = workloads.sfm_cloud(1500, 100, 10)
    x = workloads.sphere_queries(300, 7, half=1.0)
    rng = np.random.default_rng(31)
    dg = rng.standard_normal((300, mu.shape[1], 3)).astype(np.float32)
    for eps in (0.02, 0.0):
        g = orc.direct(p, n, A, mu, x, eps)["g"]
        dmu, _ = orc.direct_adjoint(p, n, A, mu, x, eps, None, dg=dg)
        lhs = np.sum(dg.astype(np.float64) * g)
        rhs = np.sum(dmu * mu.astype(np.float64))
        assert abs(lhs - rhs) <= 1e-12 * np.sum(np.abs(dg.astype(np.float64) * g)) + 1e-14
    # value and gradient cotangents add
    df = workloads.cotangents(300, mu.shape[1], 17)
    a = orc.direct_adjoint(p, n, A, mu, x, 0.02, df)
    b = orc.direct_adjoint(p, n, A, mu, x, 0.02, None, dg=dg)
    c = orc.direct_adjoint(p, n, A, mu, x, 0.02, df, dg=dg)
    assert np.allclose(c[0], a[0] + b[0], rtol=1e-12, atol=1e-15)
    assert np.allclose(c[1], a[1] + b[1], rtol=1e-12, atol=1e-15)


def test_bh_grad_cotangent_is_transpose(orc):
    p, n, A, mu = workloads.sfm_cloud(4000, 200, 10)
    x = workloads.sphere_queries(500, 11, half=1.0)
    rng = np.random.default_rng(32)
    dg = rng.standard_normal((500, mu.shape[1], 3)).astype(np.float32)
    T = orc.Tree(p, n, A, mu, 16)
    for beta in (1.0, 2.0):
        g = T.query(x, beta, 0.02)["g"]
        a = T.adjoint(x, beta, 0.02, None, dg=dg)
        lhs = np.sum(dg.astype(np.float64) * g)
        rhs = np.sum(a["dmu"] * mu.astype(np.float64))
        assert abs(lhs - rhs) <= 1e-12 * np.sum(np.abs(dg * g))
        assert np.all(a["sdmu"] >= np.abs(a["dmu"]) * (1 - 1e-12))
        assert np.all(a["sdx"] >= np.linalg.norm(a["dx"], axis=1) * (1 - 1e-12))


def test_bh_grad_cotangent_matches_direct_at_large_beta(orc):
    p, n, A, mu = workloads.sfm_cloud(1500, 50, 10)
    x = workloads.sphere_queries(200, 12, half=1.0)
    rng = np.random.default_rng(33)
    dg = rng.standard_normal((200, mu.shape[1], 3)).astype(np.float32)
    df = workloads.cotangents(200, mu.shape[1], 17)
    T = orc.Tree(p, n, A, mu, 16)
    a = T.adjoint(x, 1e4, 0.02, df, dg=dg)
    dmu, dx = orc.direct_adjoint(p, n, A, mu, x, 0.02, df, dg=dg)
    assert np.allclose(a["dmu"], dmu, rtol=1e-10, atol=1e-14)
    assert np.allclose(a["dx"], dx, rtol=1e-10, atol=1e-14)


def test_bh_grad_cotangent_dx_matches_finite_differences(orc):
    # L = sum dg . grad f_BH; smooth in x away from decision boundaries
    p, n, A, mu = workloads.sfm_cloud(3000, 100, 10)
    T = orc.Tree(p, n, A, mu, 16)
    x = workloads.sphere_queries(60, 13, half=1.0).astype(np.float64)
    h = 2.0 ** -14
    base = T.query(x.astype(np.float32), 2.0, 0.05)
    checked = 0
    for k in range(3):
        dg = _axis_cotangents(60, mu.shape[1], k, 40 + k)
        a = T.adjoint(x.astype(np.float32), 2.0, 0.05, None, dg=dg)
        xp, xm = x.copy(), x.copy()
        xp[:, k] += h
        xm[:, k] -= h
        rp = T.query(xp.astype(np.float32), 2.0, 0.05)
        rm = T.query(xm.astype(np.float32), 2.0, 0.05)
        same = np.all(rp["counts"] == base["counts"], axis=1) & np.all(rm["counts"] == base["counts"], axis=1)
        dxk = (xp[:, k].astype(np.float32).astype(np.float64) - xm[:, k].astype(np.float32).astype(np.float64))
        fd = np.einsum("qc,qcj->qj", dg[:, :, k].astype(np.float64), rp["g"] - rm["g"]) / dxk[:, None]
        err = np.linalg.norm(fd - a["dx"], axis=1) / a["sdx"]
        assert np.all(err[same] < 1e-3)
        checked += int(same.sum())
    assert checked > 100


# --------------------------------------------------------------------------
# derivatives in the normals and in eps (both optimised in Sec. 5.2)
# --------------------------------------------------------------------------
def test_eps_derivatives_of_radial(orc):
    # d kappa / d eps and d lambda / d eps against central differences in eps
    for eps in (0.02, 0.05, 0.3):
        for r in (0.0, 0.005, 0.02, 0.06, 0.2):
            h = eps * 1e-5
            kp, lp = orc.radial(r, eps + h)
            km, lm = orc.radial(r, eps - h)
            ke, le = orc.radial_eps(r, eps)
            assert abs((kp - km) / (2 * h) - ke) <= 1e-6 * abs(ke) + 1e-9 * abs(kp)
            assert abs((lp - lm) / (2 * h) - le) <= 1e-6 * abs(le) + 1e-9 * abs(lp)
    assert orc.radial_eps(0.1, 0.0) == (0.0, 0.0)


def _loss_direct(orc, p, n, A, mu, x, eps, df, dg):
    r = orc.direct(p, n, A, mu, x, eps)
    return float(np.sum(df.astype(np.float64) * r["f"]) + np.sum(dg.astype(np.float64) * r["g"]))


def _loss_bh(orc, p, n, A, mu, x, eps, df, dg, beta=2.0):
    r = orc.Tree(p, n, A, mu, 16).query(x, beta, eps)
    return float(np.sum(df.astype(np.float64) * r["f"]) + np.sum(dg.astype(np.float64) * r["g"]))


def test_direct_normal_and_eps_derivatives_fd(orc):
    # L = sum df . f + sum dg . grad f; linear in each normal component, so
    # central differences are exact up to rounding; smooth in eps
    p, n, A, mu = workloads.sfm_cloud(400, 20, 10)
    x = workloads.sphere_queries(150, 5, half=1.0)
    df = workloads.cotangents(150, mu.shape[1], 17)
    dg = np.random.default_rng(41).standard_normal((150, mu.shape[1], 3)).astype(np.float32)
    eps = 0.05
    _, _, dn, deps = orc.direct_adjoint(p, n, A, mu, x, eps, df, dg=dg, extra=True)
    rng = np.random.default_rng(42)
    for m in rng.choice(p.shape[0], size=6, replace=False):
        for k in range(3):
            npl, nmi = n.copy(), n.copy()
            npl[m, k] += np.float32(2.0 ** -8)
            nmi[m, k] -= np.float32(2.0 ** -8)
            step = float(npl[m, k]) - float(nmi[m, k])
            fd = (_loss_direct(orc, p, npl, A, mu, x, eps, df, dg) -
                  _loss_direct(orc, p, nmi, A, mu, x, eps, df, dg)) / step
            assert abs(fd - dn[m, k]) <= 1e-7 * (abs(dn[m, k]) + np.abs(dn).max())
    cd = {h: (_loss_direct(orc, p, n, A, mu, x, eps + h, df, dg) -
              _loss_direct(orc, p, n, A, mu, x, eps - h, df, dg)) / (2 * h) for h in (1e-4, 5e-5)}
    fd = (4 * cd[5e-5] - cd[1e-4]) / 3
    assert abs(fd - deps) <= 1e-6 * abs(deps)


def test_bh_normal_and_eps_derivatives(orc):
    p, n, A, mu = workloads.sfm_cloud(3000, 100, 10)
    x = workloads.sphere_queries(200, 13, half=1.0)
    df = workloads.cotangents(200, mu.shape[1], 17)
    dg = np.random.default_rng(43).standard_normal((200, mu.shape[1], 3)).astype(np.float32)
    eps = 0.05
    T = orc.Tree(p, n, A, mu, 16)
    a = T.adjoint(x, 2.0, eps, df, dg=dg, extra=True)
    assert np.all(a["sdn"] >= np.linalg.norm(a["dn"], axis=1) * (1 - 1e-12))
    assert a["sdeps"] >= abs(a["deps"])
    # the Barnes-Hut sum is linear in the normals (node dipoles are sums of
    # A mu n; the tree geometry does not involve normals)
    rng = np.random.default_rng(44)
    for m in rng.choice(p.shape[0], size=4, replace=False):
        for k in range(3):
            npl, nmi = n.copy(), n.copy()
            npl[m, k] += np.float32(2.0 ** -8)
            nmi[m, k] -= np.float32(2.0 ** -8)
            step = float(npl[m, k]) - float(nmi[m, k])
            fd = (_loss_bh(orc, p, npl, A, mu, x, eps, df, dg) - _loss_bh(orc, p, nmi, A, mu, x, eps, df, dg)) / step
            assert abs(fd - a["dn"][m, k]) <= 1e-7 * (abs(a["dn"][m, k]) + np.abs(a["dn"]).max())
    # eps does not enter the far decisions: the BH sum is smooth in eps
    cd = {h: (_loss_bh(orc, p, n, A, mu, x, eps + h, df, dg) -
              _loss_bh(orc, p, n, A, mu, x, eps - h, df, dg)) / (2 * h) for h in (1e-4, 5e-5)}
    fd = (4 * cd[5e-5] - cd[1e-4]) / 3
    assert abs(fd - a["deps"]) <= 1e-6 * a["sdeps"]
    # large beta: the direct adjoint
    b = T.adjoint(x, 1e4, eps, df, dg=dg, extra=True)
    _, _, dn, deps = orc.direct_adjoint(p, n, A, mu, x, eps, df, dg=dg, extra=True)
    assert np.allclose(b["dn"], dn, rtol=1e-10, atol=1e-14 * np.abs(dn).max())
    assert abs(b["deps"] - deps) <= 1e-10 * b["sdeps"]


# --------------------------------------------------------------------------
# monopole kernel (appearance channels with the foreshortening term skipped)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("R,eps", [(1.0, 0.0), (0.5, 0.0), (0.5, 0.2), (1.0, 0.7)])
def test_monopole_sphere_centre_closed_form(orc, R, eps):
    # every point of a sphere of radius R is at distance R from the centre:
    # sum_m A_m nu rho(R/eps)/(4 pi R^2) = nu rho(R/eps) when sum A = 4 pi R^2
    p, n, A, mu = workloads.sphere_cloud(4096, 1)
    p = (p * np.float32(R)).astype(np.float32)
    A = (A * np.float32(R * R)).astype(np.float32)
    r = orc.direct_mono(p, A, mu, np.zeros((1, 3), np.float32), eps)
    pr = p.astype(np.float64)
    dist = np.linalg.norm(pr, axis=1)
    rho = np.array([orc.rho(v / eps) if eps > 0 else 1.0 for v in dist])
    expect = np.sum(A.astype(np.float64)[:, None] * mu * (rho / (4 * math.pi * dist ** 2))[:, None], axis=0)
    assert np.allclose(r["f"][0], expect, rtol=1e-12)
    # and the closed form itself, up to the FP32 rounding of areas and radii
    assert abs(r["f"][0, 0] - (orc.rho(R / eps) if eps > 0 else 1.0)) < 1e-5


def test_monopole_numpy_crosscheck_tiny(orc):
    from scipy.special import erf
    rng = np.random.default_rng(61)
    M, Q, C, eps = 40, 25, 3, 0.3
    p = rng.uniform(-1, 1, (M, 3)).astype(np.float32)
    A = rng.uniform(0.01, 0.1, M).astype(np.float32)
    mu = rng.standard_normal((M, C)).astype(np.float32)
    x = rng.uniform(-1, 1, (Q, 3)).astype(np.float32)
    d = p[None].astype(np.float64) - x[:, None].astype(np.float64)
    r = np.linalg.norm(d, axis=2)
    t = r / eps
    rho = erf(t) - 2 * t / math.sqrt(math.pi) * np.exp(-t * t)
    drho = 4 / math.sqrt(math.pi) * t * t * np.exp(-t * t)
    m = rho / (4 * math.pi * r * r)
    dm = (drho / eps * r * r - 2 * r * rho) / (4 * math.pi * r ** 4)  # d m / d r
    w = A.astype(np.float64)[None, :, None] * mu.astype(np.float64)[None]
    f = np.sum(w * m[..., None], axis=1)
    g = np.einsum("qmc,qmk->qck", w * (-dm / r)[..., None], d)  # grad_x r = -d / r
    out = orc.direct_mono(p, A, mu, x, eps)
    assert np.allclose(out["f"], f, rtol=1e-12, atol=1e-15)
    assert np.allclose(out["g"], g, rtol=1e-10, atol=1e-14)


def test_monopole_gradient_and_adjoint(orc):
    p, n, A, mu = workloads.sfm_cloud(1500, 100, 10)
    x = workloads.sphere_queries(200, 7, half=1.0).astype(np.float64)
    eps = 0.05
    r = orc.direct_mono(p, A, mu, x.astype(np.float32), eps)
    h = 2.0 ** -14
    for k in range(3):
        xp, xm = x.copy(), x.copy()
        xp[:, k] += h
        xm[:, k] -= h
        xp32, xm32 = xp.astype(np.float32), xm.astype(np.float32)
        fp = orc.direct_mono(p, A, mu, xp32, eps)["f"]
        fm = orc.direct_mono(p, A, mu, xm32, eps)["f"]
        dxk = xp32[:, k].astype(np.float64) - xm32[:, k].astype(np.float64)
        fd = (fp - fm) / dxk[:, None]
        assert np.max(np.abs(fd - r["g"][:, :, k]) / r["sg"]) < 1e-4
    df = workloads.cotangents(200, mu.shape[1], 17)
    dmu, dx = orc.direct_mono_adjoint(p, A, mu, x.astype(np.float32), eps, df)
    lhs = np.sum(df.astype(np.float64) * r["f"])
    assert abs(lhs - np.sum(dmu * mu.astype(np.float64))) <= 1e-12 * np.sum(np.abs(df * r["f"]))
    assert np.allclose(dx, np.einsum("qc,qck->qk", df.astype(np.float64), r["g"]), rtol=1e-10, atol=1e-13)


def test_monopole_barnes_hut(orc):
    p, n, A, mu = workloads.sfm_cloud(4000, 200, 10)
    x = workloads.sphere_queries(400, 11, half=1.0)
    df = workloads.cotangents(400, mu.shape[1], 17)
    eps = 0.02
    T = orc.Tree(p, n, A, mu, 16, kind="monopole")
    ref = orc.direct_mono(p, A, mu, x, eps)
    errs = []
    for beta in (1.0, 2.0, 4.0):
        q = T.query(x, beta, eps)
        errs.append(np.max(np.abs(q["f"] - ref["f"]) / ref["sf"]))
        # adjoint = transpose of the Barnes-Hut forward
        a = T.adjoint(x, beta, eps, df)
        lhs = np.sum(df.astype(np.float64) * q["f"])
        assert abs(lhs - np.sum(a["dmu"] * mu.astype(np.float64))) <= 1e-12 * np.sum(np.abs(df * q["f"]))
        assert np.allclose(a["dx"], np.einsum("qc,qck->qk", df.astype(np.float64), q["g"]), rtol=1e-10,
                           atol=1e-13)
        assert np.all(a["sdmu"] >= np.abs(a["dmu"]) * (1 - 1e-12))
    assert errs[0] > errs[1] > errs[2]
    # large beta: the direct sum and its adjoint
    q = T.query(x, 1e4, eps)
    assert np.allclose(q["f"], ref["f"], rtol=1e-10, atol=1e-14)
    assert np.allclose(q["g"], ref["g"], rtol=1e-10, atol=1e-14)
    a = T.adjoint(x, 1e4, eps, df)
    dmu, dx = orc.direct_mono_adjoint(p, A, mu, x, eps, df)
    assert np.allclose(a["dmu"], dmu, rtol=1e-10, atol=1e-14)
    assert np.allclose(a["dx"], dx, rtol=1e-10, atol=1e-14)
    # node charges are point sums; gradient cotangents are not defined here
    with pytest.raises(ValueError):
        T.adjoint(x, 2.0, eps, df, dg=np.zeros((400, mu.shape[1], 3), np.float32))


def _f32_nearest(fr):
    """The float32 nearest to the rational fr, ties to even (exact)."""
    from fractions import Fraction
    c = np.float32(float(fr))
    best = None
    for cand in (np.nextafter(c, np.float32(-np.inf)), c, np.nextafter(c, np.float32(np.inf))):
        key = (abs(Fraction(float(cand)) - fr), int(np.float32(cand).view(np.uint32)) & 1)
        if best is None or key < best[0]:
            best = (key, np.float32(cand))
    return best[1]


def _dist2_fused(a, b):
    """The far-test squared distance of Algorithm 1 as read here (R31): FP32
    differences, dx*dx rounded, then two fused multiply-adds each rounded
    once, evaluated in exact rational arithmetic."""
    from fractions import Fraction
    d = [np.float32(np.float32(a[k]) - np.float32(b[k])) for k in range(3)]
    t = np.float32(d[0] * d[0])
    u = _f32_nearest(Fraction(float(d[1])) ** 2 + Fraction(float(t)))
    return _f32_nearest(Fraction(float(d[2])) ** 2 + Fraction(float(u)))


def test_node_radius_is_the_fused_squared_distance(orc):
    """R31: a node's squared radius is the largest far-test squared distance
    between its centroid and its points.  Every exported radius equals the
    exact-rational evaluation of the fused sequence bit for bit, and an
    unfused evaluation of the same distances differs for some nodes, so the
    pin tells the two readings apart."""
    rng = np.random.default_rng(61)
    p = rng.uniform(-1, 1, (2000, 3)).astype(np.float32)
    n = rng.standard_normal((2000, 3)).astype(np.float32)
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    A = np.full(2000, 1e-3, np.float32)
    mu = np.ones((2000, 1), np.float32)
    T = orc.Tree(p, n, A, mu, 16)
    e = T.export()
    ps = p[e["perm"].astype(np.int64)]
    differs = 0
    for i in range(e["nodes"].shape[0]):
        b, c = int(e["nodes"][i, 4]), int(e["nodes"][i, 5])
        ctr = e["geom"][i, :3]
        fused = max(_dist2_fused(ps[j], ctr) for j in range(b, b + c))
        assert fused.view(np.uint32) == e["geom"][i, 3].view(np.uint32), i
        d = ps[b:b + c] - ctr
        unfused = np.max((d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2])
        differs += int(unfused.view(np.uint32) != fused.view(np.uint32))
    assert differs > 0
