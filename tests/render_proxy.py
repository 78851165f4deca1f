"""Smooth value-only volume-rendering proxy used to drive the adjoint (test
and benchmark harness, not part of the method).

Geometry field g = 1/2 - D_0 (Sec. 4.2, eq. geometry_field) and vacancy
v = Phi(s g) (Sec. 3.1, eq. vacancy, fixed s = 10).  The paper's attenuation
is |w . grad v| / v = s phi(s g) |w . grad g| / Phi(s g) (eq. surface_density);
this proxy uses values only and replaces |w . grad g| by a constant, giving the
smooth density sigma_j = K phi(s g_j) / Phi(s g_j).  Opacity
alpha_j = 1 - exp(-sigma_j), transmittance T_j = prod_{i<j} (1 - alpha_i)
(eq. quadrature, read with 1 - exp(-sigma delta) and i < j), colour
C = sum_j T_j alpha_j D_{1:3}(x_j), loss = sum over rays |C - C*|^2.
Everything is smooth in the field values, so central differences converge.
"""
import math

import numpy as np

S_VAC = 10.0
K_DENS = 0.5


def loss_torch(f, n_rays, S, target):
    import torch
    f = f.reshape(n_rays, S, -1)
    z = S_VAC * (0.5 - f[..., 0])
    pdf = torch.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)
    cdf = 0.5 * (1.0 + torch.erf(z / math.sqrt(2.0)))
    alpha = 1.0 - torch.exp(-K_DENS * pdf / cdf)
    trans = torch.cumprod(torch.cat([torch.ones_like(alpha[:, :1]), 1.0 - alpha[:, :-1]], dim=1), dim=1)
    col = torch.sum((trans * alpha)[..., None] * f[..., 1:4], dim=1)
    return torch.sum((col - target) ** 2)


def loss_numpy(f, n_rays, S, target):
    from scipy.special import erf
    f = f.reshape(n_rays, S, -1)
    z = S_VAC * (0.5 - f[..., 0])
    pdf = np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)
    cdf = 0.5 * (1.0 + erf(z / math.sqrt(2.0)))
    alpha = 1.0 - np.exp(-K_DENS * pdf / cdf)
    trans = np.cumprod(np.concatenate([np.ones_like(alpha[:, :1]), 1.0 - alpha[:, :-1]], axis=1), axis=1)
    col = np.sum((trans * alpha)[..., None] * f[..., 1:4], axis=1)
    return float(np.sum((col - target) ** 2))


def fd_linear(f0, fe, c, loss, h):
    """Central-difference derivative of loss(f) along the attribute direction
    whose field response (channel c) is fe: the step moves the field by at
    most h (so the FP64 loss resolves it), with Richardson extrapolation over
    steps h and h/2 to cancel the O(h^2) term."""
    scale = max(float(np.abs(fe).max()), 1e-300)

    def cd(step):
        s = step / scale
        fp, fm = f0.copy(), f0.copy()
        fp[:, c] += s * fe
        fm[:, c] -= s * fe
        return (loss(fp) - loss(fm)) / (2 * s)

    return (4.0 * cd(h / 2) - cd(h)) / 3.0


def loss_rays_numpy(f, n_rays, S, target):
    """Per-ray terms of ``loss_numpy`` (their sum is the loss)."""
    from scipy.special import erf
    f = f.reshape(n_rays, S, -1)
    z = S_VAC * (0.5 - f[..., 0])
    pdf = np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)
    cdf = 0.5 * (1.0 + erf(z / math.sqrt(2.0)))
    alpha = 1.0 - np.exp(-K_DENS * pdf / cdf)
    trans = np.cumprod(np.concatenate([np.ones_like(alpha[:, :1]), 1.0 - alpha[:, :-1]], axis=1), axis=1)
    col = np.sum((trans * alpha)[..., None] * f[..., 1:4], axis=1)
    return np.sum((col - target) ** 2, axis=1)


def fd_position(T, x, f0, counts0, q, k, S, target, h, beta, eps):
    """Central-difference derivative of the loss w.r.t. coordinate k of query
    q (ray-major layout, S samples per ray), with f re-evaluated by the oracle
    tree T at the perturbed FP32 position.  Only the term of the ray holding q
    changes, so only that term is differenced.  Richardson over steps h, h/2.
    Returns None if the visited set of the query changes within the step (the
    Barnes-Hut sum is discontinuous there)."""
    r = q // S
    blk = f0[r * S:(r + 1) * S].copy()
    tgt = target[r:r + 1]

    def cd(step):
        xp, xm = x[q:q + 1].astype(np.float64).copy(), x[q:q + 1].astype(np.float64).copy()
        xp[0, k] += step
        xm[0, k] -= step
        xp32, xm32 = xp.astype(np.float32), xm.astype(np.float32)
        rp, rm = T.query(xp32, beta, eps), T.query(xm32, beta, eps)
        if not (np.array_equal(rp["counts"][0], counts0[q]) and np.array_equal(rm["counts"][0], counts0[q])):
            return None
        bp, bm = blk.copy(), blk.copy()
        bp[q - r * S] = rp["f"][0]
        bm[q - r * S] = rm["f"][0]
        lp = loss_rays_numpy(bp, 1, S, tgt)[0]
        lm = loss_rays_numpy(bm, 1, S, tgt)[0]
        return (lp - lm) / float(xp32[0, k] - xm32[0, k])

    a, b = cd(h), cd(h / 2)
    if a is None or b is None:
        return None
    return (4.0 * b - a) / 3.0
