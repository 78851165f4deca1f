"""Pins of the ray front-end oracle (``oracle/rays.py``): the march positions
against their exact FP64 definition, the first-crossing search against a
brute-force scan, the crossing point against the closed-form blurred-sphere
field (Prop. 1, the noncentral chi-square CDF) on a dense sphere, and the
sample placement against the properties any correct placement has (segment
counts, one sample per stratum, the window around the interpolated crossing,
positions on the ray)."""
import math

import numpy as np
import pytest
import scipy.optimize as so
import scipy.stats as st

import workloads

F = np.float32


def _rays(R, seed, dist=3.0, impact=(0.0, 0.8)):
    """Rays from points at distance `dist` aimed past the origin at an impact
    parameter drawn from `impact`; near / far limits of the sphere |x| <= 2."""
    rng = np.random.default_rng(seed)
    o = rng.standard_normal((R, 3))
    o = dist * o / np.linalg.norm(o, axis=1, keepdims=True)
    # a unit vector orthogonal to o, scaled by the impact parameter
    v = rng.standard_normal((R, 3))
    v -= np.sum(v * o, axis=1, keepdims=True) * o / dist ** 2
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    b = rng.uniform(*impact, size=(R, 1))
    d = b * v - o
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    bb = np.sum(d * o, axis=1)
    c = dist * dist - 4.0
    s = np.sqrt(bb * bb - c)
    return o.astype(F), d.astype(F), (-bb - s).astype(F), (-bb + s).astype(F)


def test_march_positions_match_their_definition(orc):
    from oracle import rays
    o, d, tn, tf = _rays(64, 1)
    n = 1024
    t, h = rays.march_t(tn, tf, n)
    exact = tn.astype(np.float64)[:, None] + (np.arange(n) + 0.5)[None, :] * (
        (tf.astype(np.float64) - tn.astype(np.float64)) / n)[:, None]
    # three FP32 roundings (h, k h, the sum), each within half an ulp
    bound = 3 * 2.0 ** -24 * (np.abs(tn)[:, None] + 2 * np.abs(exact))
    assert np.all(np.abs(t - exact) <= bound)
    assert np.all(np.diff(t, axis=1) > 0) and np.all(t[:, 0] > tn) and np.all(t[:, -1] < tf)
    x = rays.positions(o, d, t)
    on = o.astype(np.float64)[:, None, :] + t.astype(np.float64)[..., None] * d.astype(np.float64)[:, None, :]
    assert np.max(np.abs(x - on)) <= 4 * 2.0 ** -24 * 4.0


def test_first_crossing_brute_force(orc):
    from oracle import rays
    rng = np.random.default_rng(2)
    v = rng.choice(np.array([0.1, 0.49, 0.5, 0.51, 0.9]), size=(500, 12))
    v[:40] = 0.2  # no crossing
    v[40:80] = 0.8
    j = rays.first_crossing(v, 0.5)
    for r in range(v.shape[0]):
        want = -1
        for k in range(v.shape[1] - 1):
            if (v[r, k] >= 0.5) != (v[r, k + 1] >= 0.5):
                want = k
                break
        assert j[r] == want
    assert np.all(j[:80] == -1)


def _wsphere(a, R, eps):
    s2 = eps * eps / 2.0
    return st.ncx2.cdf(R * R / s2, 3, a * a / s2)


@pytest.mark.parametrize("eps", [0.05, 0.1])
def test_march_finds_the_blurred_sphere_surface(orc, eps):
    """The geometry field of a dense sphere with unit attributes is the
    ball's indicator blurred by a Gaussian of per-axis variance eps^2/2
    (Prop. 1).  Rays that pass within 0.8 of the centre cross the 1/2 level
    where that closed form equals 1/2; rays that pass beyond 1.25 do not
    cross.  beta = 100 makes the sums practically direct, so what is tested
    is the march, the crossing search and the interpolation (at beta = 4 the
    Barnes-Hut error alone moves the crossing by about 1e-3)."""
    from oracle import rays
    p, n, A = workloads.fibonacci_sphere(40000)
    mu = np.ones((p.shape[0], 1), F)
    T = orc.Tree(p, n, A, mu, 16)
    o, d, tn, tf = _rays(12, 3)
    m = rays.march(T, o, d, tn, tf, 1024, 100.0, eps)
    j, t, v = m["j"], m["t"].astype(np.float64), m["v"]
    assert np.all(j >= 0)
    for r in range(len(j)):
        k = j[r]
        w = (0.5 - v[r, k]) / (v[r, k + 1] - v[r, k])
        ts = t[r, k] + w * (t[r, k + 1] - t[r, k])
        oo, dd = o[r].astype(np.float64), d[r].astype(np.float64)
        tmid = -float(np.dot(oo, dd))  # closest approach to the centre

        def g(s):
            return _wsphere(np.linalg.norm(oo + s * dd), 1.0, eps) - 0.5

        tc = so.brentq(g, float(tn[r]), tmid)
        assert abs(ts - tc) < 1e-4, (r, ts, tc)
    o, d, tn, tf = _rays(12, 4, impact=(1.25, 1.6))
    m = rays.march(T, o, d, tn, tf, 1024, 4.0, eps)
    assert np.all(m["j"] == -1)


def _synthetic_march(R, n, seed):
    o, d, tn, tf = _rays(R, seed)
    j, vj, vj1, u = workloads.synthetic_crossings(R, n, seed)
    return o, d, tn, tf, j, vj, vj1, u


def test_resample_placement_properties(orc):
    from oracle import rays
    n = 1024
    o, d, tn, tf, j, vj, vj1, u = _synthetic_march(200, n, 5)
    t, x, ts = rays.resample(o, d, tn, tf, n, j, vj, vj1, u)
    assert t.shape == (200, 80) and t.dtype == F
    t64 = t.astype(np.float64)
    tn64, tf64 = tn.astype(np.float64), tf.astype(np.float64)
    h = (tf64 - tn64) / n
    ulp = 2.0 ** -22 * np.maximum(np.abs(tn64), np.abs(tf64))  # a few FP32 roundings
    for r in range(200):
        assert np.all(np.diff(t64[r]) >= -ulp[r]), r
        assert t64[r, 0] >= tn64[r] - ulp[r] and t64[r, -1] <= tf64[r] + ulp[r]
        if j[r] < 0:
            assert math.isnan(ts[r])
            segs = [(tn64[r], tf64[r], 80, 0)]
        else:
            # the interpolated crossing lies between the two samples and
            # reproduces the level by linear interpolation
            tj = tn64[r] + (j[r] + 0.5) * h[r]
            assert tj - ulp[r] <= ts[r] <= tj + h[r] + ulp[r]
            w = (ts[r] - tj) / h[r]
            assert abs((1 - w) * vj[r] + w * vj1[r] - 0.5) < 1e-4
            a = max(tn64[r], ts[r] - 8 * h[r])
            b = min(tf64[r], ts[r] + 8 * h[r])
            segs = [(tn64[r], a, 24, 0), (a, b, 48, 24), (b, tf64[r], 8, 72)]
        for lo, hi, m, off in segs:
            step = (hi - lo) / m
            for i in range(m):
                # one sample per stratum, at its jittered position
                assert lo + i * step - ulp[r] <= t64[r, off + i] <= lo + (i + 1) * step + ulp[r]
                assert abs(t64[r, off + i] - (lo + (i + u[r, off + i]) * step)) <= 2 * ulp[r]
    on = o.astype(np.float64)[:, None, :] + t64[..., None] * d.astype(np.float64)[:, None, :]
    assert np.max(np.abs(x - on)) <= 4 * 2.0 ** -24 * 4.0


def test_harnack_step_solves_its_equations(orc):
    """s(a) is the root in [0, 1) of (1 - s) = a (1 + s)^2 for a < 1 (the
    field above the level, Harnack's lower bound) and of (1 + s) = a (1 - s)^2
    for a > 1 (below it, the upper bound); s(1) = 0."""
    from oracle import rays
    a = np.concatenate([np.geomspace(1e-3, 0.999, 200), np.geomspace(1.001, 1e3, 200)])
    s = rays.harnack_s(a)
    assert np.all((s >= 0) & (s < 1))
    lo = a < 1
    np.testing.assert_allclose((1 - s[lo]) / (1 + s[lo]) ** 2, a[lo], rtol=1e-10)
    np.testing.assert_allclose((1 + s[~lo]) / (1 - s[~lo]) ** 2, a[~lo], rtol=1e-10)
    assert rays.harnack_s(1.0) == 0.0
    assert np.all(rays.harnack_radius([0.1, -0.3], 0.5, -0.25, [1.0, 1.0]) == [rays.harnack_radius(0.1, 0.5, -0.25, 1.0), 0.0])


def test_harnack_radius_is_safe_for_a_harmonic_function(orc):
    """u(y) = 1/|y - p0| is positive and harmonic away from p0.  From a point
    at distance R of p0, u changes fastest along the line through p0, so the
    Harnack radius must keep u on its side of the level along that line:
    1/(R - rho) < level above u, 1/(R + rho) > level below it, and the same on
    random directions."""
    from oracle import rays
    rng = np.random.default_rng(7)
    for _ in range(400):
        R = rng.uniform(0.2, 3.0)
        u0 = 1.0 / R
        level = u0 * (rng.uniform(1.05, 6.0) if rng.random() < 0.5 else rng.uniform(0.1, 0.95))
        rho = float(rays.harnack_radius(u0, level, 0.0, R))
        assert 0 < rho < R
        if level > u0:
            assert 1.0 / (R - rho) < level
        else:
            assert 1.0 / (R + rho) > level
        x = np.array([R, 0.0, 0.0])
        dirs = rng.standard_normal((64, 3))
        dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
        for r in (0.25 * rho, 0.5 * rho, 0.999 * rho):
            u = 1.0 / np.linalg.norm(x[None, :] + r * dirs, axis=1)
            assert np.all((u >= level) == (u0 >= level))


@pytest.mark.parametrize("scene", ["sphere", "winding"])
def test_harnack_march_matches_the_dense_march(orc, scene):
    """The Harnack-accelerated march returns the dense march's first crossing
    and the same values there on every ray (rays that cross and rays that
    miss), with far fewer field evaluations."""
    from oracle import rays
    if scene == "sphere":
        p, n, A = workloads.fibonacci_sphere(40000)
        mu = np.ones((p.shape[0], 1), F)
        o, d, tn, tf = _rays(48, 11, impact=(0.0, 1.6))
        eps = 0.05
    else:
        p, n, A, mu = workloads.winding_cloud(20000, 1000, 90)
        o, d, tn, tf = workloads.tile_camera_rays(workloads.sfm_camera(91), 16)
        sel = np.arange(0, o.shape[0], 4)
        o, d, tn, tf = o[sel], d[sel], tn[sel], tf[sel]
        eps = 0.01414
    T = orc.Tree(p, n, A, mu, 16)
    dense = rays.march(T, o, d, tn, tf, 1024, 2.0, eps)
    hm = rays.harnack_march(T, p, o, d, tn, tf, 1024, 2.0, eps, level=0.5, lower=-0.25)
    assert np.array_equal(hm["j"], dense["j"]), np.nonzero(hm["j"] != dense["j"])
    hit = dense["j"] >= 0
    assert 0 < hit.sum() < len(hit)
    rr = np.nonzero(hit)[0]
    assert np.array_equal(hm["vj"][rr], dense["v"][rr, dense["j"][rr]])
    assert np.array_equal(hm["vj1"][rr], dense["v"][rr, dense["j"][rr] + 1])
    needed = np.where(hit, dense["j"] + 2, 1024)
    print(f"[harnack] {scene}: {len(hit)} rays, {hit.sum()} cross; evaluations {hm['evals'].mean():.1f} per ray "
          f"(dense march needs {needed.mean():.1f})", flush=True)
    assert hm["evals"].mean() < 0.5 * needed.mean()
