"""Ray front-end of the reconstruction (test infrastructure only): the dense
march that finds each ray's first crossing of the geometry level set, and the
sample placement that follows it (Sec. 7.1, ray sampling).

The paper marches 1024 samples from the near to the far limit of a camera
ray, takes the first interval over which the geometry field f = 1/2 - D_0
changes sign, and then puts 24 samples from the near limit up to that
crossing, 48 close to it and 8 from it to the far limit; a ray without a
crossing gets 80 evenly spread samples.  Where the samples sit inside those
ranges is left open; the readings taken here are:

  march positions  t_k = t_n + (k + 1/2) h, h = (t_f - t_n) / n, k < n (the
                   midpoints of n equal intervals), x_k = o + t_k d;
  first crossing   the smallest j with (D(x_j) >= level) != (D(x_{j+1}) >= level),
                   level = 1/2 (f = 0), or -1;
  crossing point   t* = t_j + w (t_{j+1} - t_j), w = (level - D_j)/(D_{j+1} - D_j)
                   (linear interpolation of D between the two samples);
  dense window     [a, b] = [max(t_n, t* - W h), min(t_f, t* + W h)], W march
                   steps on each side (W = 8);
  placement        stratified: sample i of the n_s in [lo, hi] at
                   lo + (i + u_i) (hi - lo) / n_s with the caller's jitter
                   u_i in [0, 1); segments [t_n, a], [a, b], [b, t_f] with
                   24 / 48 / 8 samples, or [t_n, t_f] with 80.

Positions are produced in FP32 one rounding per operation (NumPy float32
arithmetic, no fused multiply-add), the precision the GPU kernels use, so the
two sides agree bit for bit on them; the field values of the march are the
FP64 Barnes-Hut values of ``oracle.Tree`` at those FP32 positions.
"""
from __future__ import annotations

import numpy as np

F = np.float32


def march_t(tn, tf, n):
    """FP32 march parameters t[R, n] and the step h[R]."""
    tn = np.asarray(tn, F).reshape(-1)
    tf = np.asarray(tf, F).reshape(-1)
    h = (tf - tn) / F(n)
    k = np.arange(n, dtype=F) + F(0.5)
    return tn[:, None] + k[None, :] * h[:, None], h


def positions(o, d, t):
    """x = o + t d per component in FP32: [R, S, 3] from o, d [R, 3], t [R, S]."""
    o = np.asarray(o, F)
    d = np.asarray(d, F)
    t = np.asarray(t, F)
    return o[:, None, :] + t[:, :, None] * d[:, None, :]


def first_crossing(v, level=0.5):
    """Index j of the first sign change of v - level between consecutive
    samples (per row), or -1."""
    a = np.asarray(v) >= level
    ch = a[:, 1:] != a[:, :-1]
    j = np.argmax(ch, axis=1).astype(np.int64)
    j[~np.any(ch, axis=1)] = -1
    return j


def march(tree, o, d, tn, tf, n, beta, eps, channel=0, level=0.5):
    """The dense march on the oracle tree: returns dict t[R,n] (FP32), v[R,n]
    and sv[R,n] (FP64 values of the channel and their absolute scales), j[R]
    (first crossing or -1)."""
    t, _ = march_t(tn, tf, n)
    x = positions(o, d, t).reshape(-1, 3)
    q = tree.query(x, beta, eps, want_grad=False)
    R = t.shape[0]
    v = q["f"][:, channel].reshape(R, n)
    sv = q["sf"][:, channel].reshape(R, n)
    return {"t": t, "v": v, "sv": sv, "j": first_crossing(v, level)}


def resample(o, d, tn, tf, n_march, j, vj, vj1, u, level=0.5, counts=(24, 48, 8), window=8.0):
    """Sample placement after the march.  j[R] (first crossing or -1),
    vj, vj1 [R] the field at samples j and j+1 (FP32), u[R, S] jitter,
    S = sum(counts).  Returns t[R, S] and x[R, S, 3] (FP32) and t*[R]
    (NaN without a crossing)."""
    nb, nd, na = (int(c) for c in counts)
    S = nb + nd + na
    tn = np.asarray(tn, F).reshape(-1)
    tf = np.asarray(tf, F).reshape(-1)
    j = np.asarray(j).reshape(-1)
    vj = np.asarray(vj, F).reshape(-1)
    vj1 = np.asarray(vj1, F).reshape(-1)
    u = np.asarray(u, F)
    R = tn.shape[0]
    h = (tf - tn) / F(n_march)
    hit = j >= 0
    jf = np.where(hit, j, 0).astype(F)
    tj = tn + (jf + F(0.5)) * h
    tj1 = tn + (jf + F(1.5)) * h
    with np.errstate(divide="ignore", invalid="ignore"):
        w = (F(level) - vj) / (vj1 - vj)
    ts = tj + w * (tj1 - tj)
    half = F(window) * h
    a = np.maximum(tn, ts - half)
    b = np.minimum(tf, ts + half)
    t = np.empty((R, S), F)
    s = np.arange(S)
    for r in range(R):
        if hit[r]:
            lo = np.where(s < nb, tn[r], np.where(s < nb + nd, a[r], b[r])).astype(F)
            hi = np.where(s < nb, a[r], np.where(s < nb + nd, b[r], tf[r])).astype(F)
            i = np.where(s < nb, s, np.where(s < nb + nd, s - nb, s - nb - nd)).astype(F)
            m = np.where(s < nb, nb, np.where(s < nb + nd, nd, na)).astype(F)
        else:
            lo = np.full(S, tn[r], F)
            hi = np.full(S, tf[r], F)
            i = s.astype(F)
            m = np.full(S, S, F)
        t[r] = lo + (i + u[r]) * ((hi - lo) / m)
    ts = np.where(hit, ts, F(np.nan))
    return t, positions(o, d, t), ts


# ---------------------------------------------------------------------------
# Harnack-accelerated march (Sec. 7.1: the first crossing can be found with
# Harnack tracing instead of evaluating every march sample).
#
# Harnack's inequality: a harmonic function u > 0 on a ball of radius R
# around x in 3D satisfies, at distance r < R from x,
#     u(x) R (R - r) / (R + r)^2  <=  u  <=  u(x) R (R + r) / (R - r)^2.
# With u = D - lower (lower a bound of D below) and a = (level - lower) /
# (D(x) - lower), D cannot reach the level within r < s R, where s solves
# (1 - s) = a (1 + s)^2 when D(x) is above the level (a < 1) and
# (1 + s) = a (1 - s)^2 when it is below (a > 1):
#     s = |sqrt(8 a + 1) - (2 a + 1)| / (2 a).
# The dipole sum is harmonic away from its points, outside the regularised
# zone of each (|y - p| >= 4.5 eps, where rho(t) = 1 to 8e-9), so R is the
# distance to the nearest point less 4.5 eps.
#
# The march keeps the dense march's samples and its definition of the
# crossing (the first j with (D_j >= level) != (D_{j+1} >= level)); from an
# evaluated sample k it skips the samples strictly within safety * s R of x_k
# (their side of the level is the one of D_k), evaluates the first sample
# past them, and, if that one lies on the other side, the sample before it:
# if the latter is still on D_k's side, the crossing is the pair between
# them; if not (the field did not obey the bound), the march goes on sample
# by sample from k.  Where the bound holds the result is the dense march's.
# ---------------------------------------------------------------------------
def harnack_s(a):
    """s(a) = |sqrt(8a + 1) - (2a + 1)| / (2a) for a > 0 (0 at a = 1)."""
    a = np.asarray(a, dtype=np.float64)
    return np.abs(np.sqrt(8.0 * a + 1.0) - (2.0 * a + 1.0)) / (2.0 * a)


def harnack_radius(v, level, lower, R):
    """Radius around a point with field value v within which a harmonic
    field bounded below by `lower` stays on v's side of `level`: s(a) R,
    0 where v <= lower or R <= 0."""
    v = np.asarray(v, dtype=np.float64)
    R = np.asarray(R, dtype=np.float64)
    ok = (v > lower) & (R > 0)
    with np.errstate(divide="ignore", invalid="ignore"):
        a = (level - lower) / np.where(ok, v - lower, 1.0)
        rho = np.where(ok, harnack_s(np.where(ok, a, 1.0)) * R, 0.0)
    return rho


def harnack_march(tree, points, o, d, tn, tf, n, beta, eps, level=0.5, lower=-0.25, channel=0, safety=0.99):
    """Harnack-accelerated march with the dense march's output: j[R] (first
    crossing or -1), vj, vj1 [R] (FP64 values at samples j, j + 1), evals[R]
    (field evaluations made).  `points` [M, 3] are the cloud's points, for
    the distance to the nearest one (scipy's k-d tree)."""
    from scipy.spatial import cKDTree
    kd = cKDTree(np.asarray(points, dtype=np.float64))
    o = np.asarray(o, F)
    d = np.asarray(d, F)
    tn = np.asarray(tn, F).reshape(-1)
    tf = np.asarray(tf, F).reshape(-1)
    Rn = tn.shape[0]
    h = (tf - tn) / F(n)
    step = h.astype(np.float64) * np.linalg.norm(d.astype(np.float64), axis=1)  # sample spacing in space
    reg = 4.5 * eps if eps > 0 else 0.0

    def x_at(r, k):
        t = tn[r] + (np.asarray(k).astype(F) + F(0.5)) * h[r]
        return o[r] + t[:, None] * d[r]

    def value(r, k):
        if r.size == 0:
            return np.zeros(0)
        return tree.query(x_at(r, k), beta, eps, want_grad=False)["f"][:, channel]

    j = np.full(Rn, -1, np.int64)
    vj = np.zeros(Rn)
    vj1 = np.zeros(Rn)
    evals = np.ones(Rn, np.int64)
    all_r = np.arange(Rn)
    k = np.zeros(Rn, np.int64)
    vk = value(all_r, k)
    k2 = np.zeros(Rn, np.int64)
    v2 = np.zeros(Rn)
    mode = np.zeros(Rn, np.int64)  # 0 step from k, 1 candidate k2, 2 confirm k2 - 1, 3 dense, 4 done
    mode[k >= n - 1] = 4
    ge = lambda v: v >= level
    while np.any(mode != 4):
        st = np.nonzero(mode == 0)[0]
        if st.size:
            dist, _ = kd.query(x_at(st, k[st]).astype(np.float64))
            rho = harnack_radius(vk[st], level, lower, dist - reg)
            m = np.floor(safety * rho / step[st]).astype(np.int64)
            k2[st] = np.minimum(k[st] + m + 1, n - 1)
            mode[st] = 1
        ev = np.nonzero((mode == 1) | (mode == 2) | (mode == 3))[0]
        e = np.where(mode[ev] == 1, k2[ev], np.where(mode[ev] == 2, k2[ev] - 1, k[ev] + 1))
        w = value(ev, e)
        evals[ev] += 1
        for r, wr, mr in zip(ev, w, mode[ev].copy()):
            if mr == 1:
                if ge(wr) == ge(vk[r]):
                    k[r], vk[r] = k2[r], wr
                    mode[r] = 4 if k[r] >= n - 1 else 0
                elif k2[r] == k[r] + 1:
                    j[r], vj[r], vj1[r], mode[r] = k[r], vk[r], wr, 4
                else:
                    v2[r], mode[r] = wr, 2
            elif mr == 2:
                if ge(wr) == ge(vk[r]):
                    j[r], vj[r], vj1[r], mode[r] = k2[r] - 1, wr, v2[r], 4
                else:
                    mode[r] = 3
            else:
                if ge(wr) != ge(vk[r]):
                    j[r], vj[r], vj1[r], mode[r] = k[r], vk[r], wr, 4
                else:
                    k[r], vk[r] = k[r] + 1, wr
                    if k[r] >= n - 1:
                        mode[r] = 4
    return {"j": j, "vj": vj, "vj1": vj1, "evals": evals}
