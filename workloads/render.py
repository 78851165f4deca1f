"""Smooth value-only volume-rendering proxy used to drive the adjoint (test
and benchmark harness, not part of the method).

Geometry field g = 1/2 - D_0 (Sec. 4.2, eq. geometry_field) and vacancy
v = Phi(s g) (Sec. 3.1, eq. vacancy, fixed s = 10).  The paper's attenuation
is |w . grad v| / v = s phi(s g) |w . grad g| / Phi(s g) (eq. surface_density);
this proxy uses values only and replaces |w . grad g| by a constant, giving the
smooth density sigma_j = K phi(s g_j) / Phi(s g_j).  Opacity
alpha_j = 1 - exp(-sigma_j), transmittance T_j = prod_{i<j} (1 - alpha_i)
= exp(-sum_{i<j} sigma_i) (eq. quadrature, read with 1 - exp(-sigma delta) and
i < j), colour C = sum_j T_j alpha_j D_{1:3}(x_j), loss = sum over rays
|C - C*|^2.  Everything is smooth in the field values, so central differences
converge.  phi / Phi is evaluated as exp(log phi - log Phi) so that it stays
finite deep inside the shapes (D_0 near 1, s g near -5 and below).

The torch forms contain no host synchronisation (no data-dependent shapes, no
products whose backward inspects the data), so a forward + backward built from
them can be captured in a graph.

Batched workload with shadow rays (multi-view batch of ``workloads.batched``):
the primary hit of a ray is the first sample interval [j, j+1] where D_0
crosses 1/2, placed by linear interpolation of D_0 between the two samples.
A ray with a hit casts one shadow ray from hit + 1e-3 l (l the unit direction
to its view's light) to the exit of the |x| <= sqrt(3) bound, with stratified
samples; its shadow transmittance is T_s = exp(-sum_k sigma(D_0(x_k))).  The
pixel adds the direct illumination of eq. direct at the hit x_h,
L_d = albedo T_s n.(l - x_h) / |l - x_h|^3 with the albedo D_{1:3}(x_h) and the
implicit normal n = grad g / |grad g| = -grad D_0 / |grad D_0| (Sec. 5.1),
both from a query at the hit point itself (values and gradients, one row per
ray), to the volume colour: C + L_d (C alone for rays without a hit), the
volume colour standing in for the MLP term of eq. radiance_field_shadow_rays.
The shadow batch and the hit queries are compacted so that hits come first,
in ray order, 64 hits per group; inside a shadow group the query rows are
[sample, lane], like the primaries.
"""
import math

import numpy as np

S_VAC = 10.0
K_DENS = 0.5
LOG_SQRT_2PI = 0.5 * math.log(2.0 * math.pi)
SHADOW_OFFSET = 1e-3
BOUND2 = 3.0
GROUP = 64


# ----------------------------------------------------------------------------
# single-view proxy (samples of a ray contiguous)
# ----------------------------------------------------------------------------
def sigma_torch(f0):
    import torch
    z = S_VAC * (0.5 - f0)
    return K_DENS * torch.exp(-0.5 * z * z - LOG_SQRT_2PI - torch.special.log_ndtr(z))


def sigma_numpy(f0):
    from scipy.special import log_ndtr
    z = S_VAC * (0.5 - f0)
    return K_DENS * np.exp(-0.5 * z * z - LOG_SQRT_2PI - log_ndtr(z))


def _weights_torch(sig, dim):
    import torch
    before = torch.cumsum(sig, dim=dim) - sig
    return torch.exp(-before) * -torch.expm1(-sig)


def _weights_numpy(sig, axis):
    before = np.cumsum(sig, axis=axis) - sig
    return np.exp(-before) * -np.expm1(-sig)


def loss_torch(f, n_rays, S, target):
    import torch
    f = f.reshape(n_rays, S, -1)
    w = _weights_torch(sigma_torch(f[..., 0]), 1)
    col = torch.sum(w[..., None] * f[..., 1:4], dim=1)
    return torch.sum((col - target) ** 2)


def loss_rays_numpy(f, n_rays, S, target):
    """Per-ray terms of ``loss_numpy`` (their sum is the loss)."""
    f = f.reshape(n_rays, S, -1)
    w = _weights_numpy(sigma_numpy(f[..., 0]), 1)
    col = np.sum(w[..., None] * f[..., 1:4], axis=1)
    return np.sum((col - target) ** 2, axis=1)


def loss_numpy(f, n_rays, S, target):
    return float(np.sum(loss_rays_numpy(f, n_rays, S, target)))


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


# ----------------------------------------------------------------------------
# batched multi-view proxy with shadow rays (primary layout [tile, sample, lane])
# ----------------------------------------------------------------------------
def primary_hits_torch(f0, x):
    """f0 [T,S,64], x [T,S,64,3] -> (has [T,64] bool, hit [T,64,3])."""
    import torch
    c = f0 >= 0.5
    cross = c[:, 1:] != c[:, :-1]
    has = cross.any(dim=1)
    j = cross.to(torch.uint8).argmax(dim=1, keepdim=True)
    fj = f0.gather(1, j).squeeze(1)
    fj1 = f0.gather(1, j + 1).squeeze(1)
    jx = j[..., None].expand(-1, -1, -1, 3)
    xj = x.gather(1, jx).squeeze(1)
    xj1 = x.gather(1, jx + 1).squeeze(1)
    w = (0.5 - fj) / torch.where(has, fj1 - fj, torch.ones_like(fj))
    return has, xj + w[..., None] * (xj1 - xj)


def shadow_samples_torch(hit, has, light, u):
    """hit [n,3], has [n], light [n,3], u [n,K] -> shadow samples [n,K,3]
    (rays without a hit get K copies of their light position)."""
    import torch
    K = u.shape[1]
    l = light - hit
    ln = l / torch.linalg.vector_norm(l, dim=1, keepdim=True)
    s0 = hit + SHADOW_OFFSET * ln
    b = torch.sum(s0 * ln, dim=1)
    c = torch.sum(s0 * s0, dim=1) - BOUND2
    t_exit = torch.clamp(-b + torch.sqrt(torch.clamp(b * b - c, min=1e-12)), min=0.0)
    k = torch.arange(K, device=u.device, dtype=u.dtype)
    t = (k[None, :] + u) * (t_exit[:, None] / K)
    xs = s0[:, None, :] + t[..., None] * ln[:, None, :]
    return torch.where(has[:, None, None], xs, light[:, None, :].expand(-1, K, -1))


def shadow_layout(has, K):
    """Compacted shadow-query layout for rays has[n] (n a multiple of 64).

    Returns (rows[n,K] int64: query row of sample k of each ray, inv[n*K]:
    the ray-sample index held by each row, q_count[1] int64: rows to evaluate,
    i.e. 64*K per started group of hits, n_hits 0-d tensor, slot[n]: the
    ray's slot).  Rays with a hit take slots 0..n_hits-1 in ray order, the
    others follow, so every row holds exactly one ray-sample."""
    import torch
    n = has.numel()
    hi = has.reshape(-1).to(torch.int64)
    rank = torch.cumsum(hi, 0)
    n_hits = rank[-1]
    slot = torch.where(hi.bool(), rank - 1, n_hits + torch.cumsum(1 - hi, 0) - 1)
    k = torch.arange(K, device=has.device, dtype=torch.int64)
    rows = ((slot // GROUP) * K)[:, None] * GROUP + k[None, :] * GROUP + (slot % GROUP)[:, None]
    inv = torch.empty(n * K, device=has.device, dtype=torch.int64)
    inv[rows.reshape(-1)] = torch.arange(n * K, device=has.device, dtype=torch.int64)
    q_count = (((n_hits + (GROUP - 1)) // GROUP) * (GROUP * K)).reshape(1)
    return rows, inv, q_count, n_hits, slot


def direct_term_torch(fh, gh, hit, light):
    """eq. direct without the transmittance: albedo D_{1:3}(x_h) times
    n.(l - x_h) / |l - x_h|^3, n = -grad D_0 / |grad D_0|.  fh [n,C], gh [n,C,3]
    at the hits, hit, light [n,3]."""
    import torch
    l = light - hit
    r2 = torch.clamp(torch.sum(l * l, dim=1), min=1e-12)
    g0 = gh[:, 0, :]
    gn = torch.sqrt(torch.clamp(torch.sum(g0 * g0, dim=1), min=1e-30))
    cos = -torch.sum(g0 * l, dim=1) / (gn * r2 * torch.sqrt(r2))
    return fh[:, 1:4] * cos[:, None]


def tree_sum(v):
    """Sum of a 1-D tensor through reductions of 64 elements per output
    (zero-padded), so no reduction splits one output across workgroups;
    such split reductions clear their semaphores with a memset, which is kept
    out of captured graphs."""
    import torch
    while v.numel() > GROUP:
        pad = (-v.numel()) % GROUP
        if pad:
            v = torch.nn.functional.pad(v, (0, pad))
        v = v.view(-1, GROUP).sum(dim=1)
    return v.sum()


class _query_packet:
    """Context: the tree's query packet set to k (None: unchanged), restored
    on exit.  A host-side setting read at launch, so it also holds for
    launches recorded into a graph."""

    def __init__(self, tree, k):
        self.tree, self.k, self.prev = tree, k, None

    def __enter__(self):
        if self.k is not None:
            from paper_2405_16788_amd import binding as B
            self.prev = B.dps_get_launch(self.tree)["query"]
            B.dps_set_launch(self.tree, self.k, 0, -1)
        return self

    def __exit__(self, *exc):
        if self.k is not None:
            from paper_2405_16788_amd import binding as B
            B.dps_set_launch(self.tree, self.prev, 0, -1)
        return False


def batched_forward(dipole_sum, attrs, x, tree, batch, beta, eps, primary_grad=True, refit=True,
                    ray_weight=None, shadow_packet=2, hit_packet=1):
    """Loss of the batched proxy and its intermediates.

    dipole_sum: the differentiable query (``paper_2405_16788_amd.dipole_sum``);
    x [Q,3] the primary samples (batch layout), batch a ``RayBatch``.
    ray_weight: optional [n_rays] weights of the per-ray loss terms.
    shadow_packet, hit_packet: query packets (queries per lane) of the shadow
    and the hit-point queries, or None for the tree's own.  These rows start
    at the surface and are far fewer than the primary samples the tree's
    packet is tuned on.  Measured on the sfm-8m batch (BF16, persistent
    queue): the 29.8M shadow rows take 42 ms at 2, 50 ms at 1 or 4; the
    465k hit-point rows 11 ms at 1, 16 ms at 2.  Only the forward queries
    are affected; the adjoints keep the tree's packet.
    Returns (loss, aux) with aux holding f [Q,C], has, hit, xs_rows, rows,
    q_count, n_hits, fs [n_rays*K, 1], fh [n_rays, C] and gh [n_rays, C, 3]
    (hit queries in slot order), hit_count (their device row count) and
    direct [n_rays, 3] (L_d before masking)."""
    import torch
    S, K = batch.S, batch.S_shadow
    f, _ = dipole_sum(attrs, x, tree, beta, eps, grad=primary_grad, refit=refit)
    C = f.shape[1]
    T = x.shape[0] // (S * GROUP)
    ft = f.view(T, S, GROUP, C)
    w = _weights_torch(sigma_torch(ft[..., 0]), 1)
    col = torch.sum(w[..., None] * ft[..., 1:4], dim=1).reshape(-1, 3)
    has, hit = primary_hits_torch(ft[..., 0], x.view(T, S, GROUP, 3))
    has, hit = has.reshape(-1), hit.reshape(-1, 3)
    xs = shadow_samples_torch(hit, has, batch.ray_light, batch.shadow_u)
    rows, inv, q_count, n_hits, slot = shadow_layout(has, K)
    xs_rows = xs.reshape(-1, 3).index_select(0, inv)
    with _query_packet(tree, shadow_packet):
        fs, _ = dipole_sum(attrs, xs_rows, tree, beta, eps, channels=(0, 1), q_count=q_count, grad=False,
                           refit=False)
    fsr = fs.reshape(-1).index_select(0, rows.reshape(-1)).reshape(-1, K)
    ts = torch.exp(-torch.sum(sigma_torch(fsr), dim=1))
    # values and gradients at the hit points, one row per ray in slot order
    n = has.numel()
    inv_slot = torch.empty(n, device=has.device, dtype=torch.int64)
    inv_slot[slot] = torch.arange(n, device=has.device, dtype=torch.int64)
    x_hit = hit.index_select(0, inv_slot)
    qh = (((n_hits + (GROUP - 1)) // GROUP) * GROUP).reshape(1)
    with _query_packet(tree, hit_packet):
        fh_rows, gh_rows = dipole_sum(attrs, x_hit, tree, beta, eps, q_count=qh, grad=True, refit=False)
    fh, gh = fh_rows.index_select(0, slot), gh_rows.index_select(0, slot)
    ld = direct_term_torch(fh, gh, hit, batch.ray_light) * ts[:, None]
    pix = col + torch.where(has[:, None], ld, torch.zeros_like(ld))
    terms = torch.sum((pix - batch.target) ** 2, dim=1)
    if ray_weight is not None:
        terms = terms * ray_weight
    loss = tree_sum(terms)
    aux = {"f": f, "has": has, "hit": hit, "xs_rows": xs_rows, "rows": rows, "q_count": q_count,
           "n_hits": n_hits, "fs": fs, "fh": fh_rows, "gh": gh_rows, "hit_count": qh, "direct": ld}
    return loss, aux


# numpy (FP64) forms of the same proxy, for the oracle side of the tests
def primary_hits_numpy(f0, x):
    """f0 [n,S], x [n,S,3] (samples of a ray contiguous) -> (has, j, hit)."""
    c = f0 >= 0.5
    cross = c[:, 1:] != c[:, :-1]
    has = cross.any(axis=1)
    j = np.argmax(cross, axis=1)
    r = np.arange(f0.shape[0])
    fj, fj1 = f0[r, j], f0[r, j + 1]
    w = (0.5 - fj) / np.where(has, fj1 - fj, 1.0)
    hit = x[r, j] + w[:, None] * (x[r, j + 1] - x[r, j])
    return has, j, hit


def shadow_samples_numpy(hit, has, light, u):
    K = u.shape[1]
    l = light - hit
    ln = l / np.linalg.norm(l, axis=1, keepdims=True)
    s0 = hit + SHADOW_OFFSET * ln
    b = np.sum(s0 * ln, axis=1)
    c = np.sum(s0 * s0, axis=1) - BOUND2
    t_exit = np.maximum(-b + np.sqrt(np.maximum(b * b - c, 1e-12)), 0.0)
    t = (np.arange(K)[None, :] + u) * (t_exit[:, None] / K)
    xs = s0[:, None, :] + t[..., None] * ln[:, None, :]
    return np.where(has[:, None, None], xs, np.broadcast_to(light[:, None, :], xs.shape))


def direct_term_numpy(fh, gh, hit, light):
    l = light - hit
    r2 = np.maximum(np.sum(l * l, axis=1), 1e-12)
    g0 = gh[:, 0, :]
    gn = np.sqrt(np.maximum(np.sum(g0 * g0, axis=1), 1e-30))
    cos = -np.sum(g0 * l, axis=1) / (gn * r2 * np.sqrt(r2))
    return fh[:, 1:4] * cos[:, None]


def batched_ray_terms_numpy(f, fs, has, target, fh, gh, hit, light):
    """Per-ray loss terms from primary values f [n,S,C] (ray-major), shadow
    channel-0 values fs [n,K], and the values fh [n,C] and gradients gh
    [n,C,3] at the hits."""
    w = _weights_numpy(sigma_numpy(f[..., 0]), 1)
    col = np.sum(w[..., None] * f[..., 1:4], axis=1)
    ts = np.exp(-np.sum(sigma_numpy(fs), axis=1))
    ld = direct_term_numpy(fh, gh, hit, light) * ts[:, None]
    pix = col + np.where(has[:, None], ld, 0.0)
    return np.sum((pix - target) ** 2, axis=1)
