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
