"""Synthetic point clouds and ray samples shaped like the paper's workloads.

The paper reconstructs DTU / BlendedMVS objects from dense structure-from-motion
point clouds and traces batches of camera rays with up to 128 samples each
(Sec. 7.1).  Those datasets are not available, so these generators stand in for
them: unions of noisy spheres / tori with outliers and jittered normals, and
stratified samples along pinhole camera rays.

Every draw uses NumPy's PCG64 ``default_rng(seed)`` in float64; results are cast
once to float32, which is the precision both the reference and the GPU read.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


# ----------------------------------------------------------------------------
# workload table (sizes, seeds, beta / eps / leaf size)
# ----------------------------------------------------------------------------
@dataclass(frozen=True)
class Config:
    name: str
    n_points: int
    beta: float
    eps: float
    leaf_size: int
    seeds: tuple


CONFIGS = {
    # 8,192 points on the unit sphere; 32,768 uniform queries; forward only.
    "sphere-8k": Config("sphere-8k", 8192, 2.0, 0.05, 16, (1, 2, 3)),
    # 1M-point SfM-like cloud, 512x512 rays x 128 samples = 33,554,432 queries.
    "sfm-1m": Config("sfm-1m", 1_000_000, 2.0, math.sqrt(2.0) * 0.01, 16, (10, 11, 12)),
    # 4,194,304 points on the unit sphere (precision study, beta in {1,2,4}).
    "sphere-4m": Config("sphere-4m", 4_194_304, 2.0, 0.05, 16, (20, 21)),
    # 4,194,304-point SfM-like cloud (the 1M scene's distributions), 32,768 ray
    # samples of its camera (precision study, beta in {1,2,4}).
    "sfm-4m": Config("sfm-4m", 4_194_304, 2.0, math.sqrt(2.0) * 0.01, 16, (40, 11, 41)),
    # 8,388,608-point SfM-like cloud, 8 uneven views + shadow rays.
    "sfm-8m": Config("sfm-8m", 8_388_608, 2.0, math.sqrt(2.0) * 0.01, 16, (30, 31, 32)),
}

SFM_1M_SURFACE = 950_000
SFM_1M_OUTLIERS = 50_000
SFM_4M_SURFACE = 3_984_589   # 4,194,304 points with 5% outliers
SFM_4M_OUTLIERS = 209_715
SFM_8M_SURFACE = 7_969_178
SFM_8M_OUTLIERS = 419_430


def _unit(v):
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


# ----------------------------------------------------------------------------
# a cloud whose octree reaches the last level
# ----------------------------------------------------------------------------
DEEP_CENTRE = np.array([0.3, -0.2, 0.1])


def deep_cluster_cloud(seed: int, C: int = 4):
    """1500 points uniform in [-1, 1]^3, clusters of 24 points of half-width
    2^-2, 2^-4, ..., 2^-20 around DEEP_CENTRE and 20 copies of one point next
    to it: with 21 Morton levels over the cloud's cube, the octree reaches its
    last level.  Unit normals, areas U(0.5, 1.5) * 4/M, N(0,1) attributes.
    Returns float32 p[M,3], n[M,3], A[M], attrs[M,C]."""
    rng = np.random.default_rng(seed)
    parts = [rng.uniform(-1, 1, size=(1500, 3))]
    for k in range(2, 21, 2):
        parts.append(DEEP_CENTRE + rng.uniform(-1, 1, size=(24, 3)) * 2.0 ** -k)
    parts.append(np.repeat(DEEP_CENTRE[None] + 2.0 ** -22, 20, axis=0))
    p = np.concatenate(parts)
    M = p.shape[0]
    n = _unit(rng.standard_normal((M, 3)))
    A = rng.uniform(0.5, 1.5, size=M) * (4.0 / M)
    mu = rng.standard_normal((M, C))
    return p.astype(np.float32), n.astype(np.float32), A.astype(np.float32), mu.astype(np.float32)


def deep_cluster_probes(p, seed: int):
    """Queries around DEEP_CENTRE at every scale 2^-1 .. 2^-22 (40 each) and
    at the last 60 points of a deep_cluster_cloud p (the duplicates among them)."""
    rng = np.random.default_rng(seed)
    near = [DEEP_CENTRE + rng.uniform(-1, 1, size=(40, 3)) * 2.0 ** -k for k in range(1, 23)]
    return np.concatenate(near + [p[-60:]]).astype(np.float32)


# ----------------------------------------------------------------------------
# unit sphere cloud
# ----------------------------------------------------------------------------
def sphere_cloud(M: int, seed: int, n_rgb: int = 3):
    """Points uniform on the unit sphere (normalised Gaussians), exact outward
    normals n = p, equal areas 4*pi/M, attribute 0 = 1.0 and ``n_rgb`` U(0,1)
    colour channels.  Returns float32 arrays p[M,3], n[M,3], A[M], attrs[M,C]."""
    rng = np.random.default_rng(seed)
    p = _unit(rng.standard_normal((M, 3)))
    attrs = np.empty((M, 1 + n_rgb))
    attrs[:, 0] = 1.0
    attrs[:, 1:] = rng.uniform(size=(M, n_rgb))
    A = np.full(M, 4.0 * math.pi / M)
    return (p.astype(np.float32), p.astype(np.float32), A.astype(np.float32),
            attrs.astype(np.float32))


def sphere_queries(Q: int, seed: int, half: float = 1.5):
    """Query points uniform in the cube [-half, half]^3."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-half, half, size=(Q, 3)).astype(np.float32)


def sphere_probes(n: int, seed: int):
    """Probe sets for the unit sphere: ``n`` points on the sphere, ``n//2``
    inside (|x| <= 0.8) and ``n - n//2`` outside (1.2 <= |x| <= 1.5)."""
    rng = np.random.default_rng(seed)
    on = _unit(rng.standard_normal((n, 3)))
    d_in = _unit(rng.standard_normal((n // 2, 3)))
    r_in = 0.8 * rng.uniform(size=(n // 2, 1)) ** (1.0 / 3.0)
    d_out = _unit(rng.standard_normal((n - n // 2, 3)))
    r_out = rng.uniform(1.2, 1.5, size=(n - n // 2, 1))
    return (on.astype(np.float32), (d_in * r_in).astype(np.float32),
            (d_out * r_out).astype(np.float32))


# ----------------------------------------------------------------------------
# SfM-like cloud: union of 3 spheres / tori + noise + outliers
# ----------------------------------------------------------------------------
def _random_rotation(rng):
    q = _unit(rng.standard_normal(4))
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


def _split_counts(total, weights):
    w = np.asarray(weights, dtype=np.float64)
    raw = total * w / w.sum()
    cnt = np.floor(raw).astype(np.int64)
    rem = total - cnt.sum()
    order = np.argsort(-(raw - cnt), kind="stable")
    cnt[order[:rem]] += 1
    return cnt


def _sample_torus(rng, n, R, a):
    """Uniform-by-area samples on a torus (major R, minor a) in local frame."""
    th = rng.uniform(0, 2 * math.pi, size=n)
    ph = np.empty(n)
    filled = 0
    while filled < n:
        k = (n - filled) * 2 + 64
        cand = rng.uniform(0, 2 * math.pi, size=k)
        keep = rng.uniform(size=k) * (R + a) < (R + a * np.cos(cand))
        cand = cand[keep][: n - filled]
        ph[filled:filled + cand.size] = cand
        filled += cand.size
    ring = R + a * np.cos(ph)
    pts = np.stack([ring * np.cos(th), ring * np.sin(th), a * np.sin(ph)], axis=1)
    nrm = np.stack([np.cos(ph) * np.cos(th), np.cos(ph) * np.sin(th), np.sin(ph)], axis=1)
    return pts, nrm


def sfm_cloud(n_surface: int, n_outliers: int, seed: int, n_rgb: int = 3,
              noise: float = 0.01, tilt_deg: float = 5.0):
    """SfM-shaped oriented cloud.

    Three shapes (sphere or torus with probability 1/2 each), centres
    U([-0.5,0.5]^3), radii U(0.2,0.6), torus minor radius R/3 and a random
    rotation.  ``n_surface`` points uniform by area, split across shapes in
    proportion to area, with N(0, noise^2 I) position noise and normals tilted
    by U(0, tilt_deg) degrees about a random tangent axis.  ``n_outliers``
    points U([-1,1]^3) with random unit normals.  Every point gets the area
    total_surface_area / n_surface.  Attribute 0 ~ N(0,1), colours ~ U(0,1).
    The point order is shuffled.
    """
    rng = np.random.default_rng(seed)
    shapes = []
    for _ in range(3):
        kind = "sphere" if rng.uniform() < 0.5 else "torus"
        centre = rng.uniform(-0.5, 0.5, size=3)
        R = rng.uniform(0.2, 0.6)
        rot = _random_rotation(rng)
        area = 4 * math.pi * R * R if kind == "sphere" else 4 * math.pi ** 2 * R * (R / 3)
        shapes.append((kind, centre, R, rot, area))
    counts = _split_counts(n_surface, [s[4] for s in shapes])
    P, N = [], []
    for (kind, centre, R, rot, _), k in zip(shapes, counts):
        if kind == "sphere":
            nrm = _unit(rng.standard_normal((k, 3)))
            pts = nrm * R
        else:
            pts, nrm = _sample_torus(rng, k, R, R / 3)
        P.append(pts @ rot.T + centre)
        N.append(nrm @ rot.T)
    P = np.concatenate(P)
    N = np.concatenate(N)
    P = P + noise * rng.standard_normal(P.shape)
    # tilt each normal about a random tangent axis
    v = rng.standard_normal(N.shape)
    t = _unit(v - np.sum(v * N, axis=1, keepdims=True) * N)
    ang = np.deg2rad(rng.uniform(0.0, tilt_deg, size=(N.shape[0], 1)))
    N = _unit(N * np.cos(ang) + np.cross(t, N) * np.sin(ang))
    Po = rng.uniform(-1.0, 1.0, size=(n_outliers, 3))
    No = _unit(rng.standard_normal((n_outliers, 3)))
    p = np.concatenate([P, Po])
    n = np.concatenate([N, No])
    M = p.shape[0]
    total_area = sum(s[4] for s in shapes)
    A = np.full(M, total_area / n_surface)
    attrs = np.empty((M, 1 + n_rgb))
    attrs[:, 0] = rng.standard_normal(M)
    attrs[:, 1:] = rng.uniform(size=(M, n_rgb))
    perm = rng.permutation(M)
    return (p[perm].astype(np.float32), n[perm].astype(np.float32),
            A[perm].astype(np.float32), attrs[perm].astype(np.float32))


# ----------------------------------------------------------------------------
# camera rays and stratified samples
# ----------------------------------------------------------------------------
def camera_rays(eye, H: int, W: int, fov_deg: float = 50.0, bound: float = math.sqrt(3.0)):
    """Pinhole rays from ``eye`` looking at the origin with up +z.

    Returns float64 origins[H,W,3], unit directions[H,W,3] and the entry / exit
    distances t_in, t_out[H,W] of the bounding sphere |x| <= bound.  Raises if
    a ray misses the sphere."""
    eye = np.asarray(eye, dtype=np.float64)
    fwd = _unit(-eye)
    up = np.array([0.0, 0.0, 1.0])
    if abs(float(np.dot(fwd, up))) > 0.999:
        up = np.array([0.0, 1.0, 0.0])
    right = _unit(np.cross(fwd, up))
    cup = np.cross(right, fwd)
    th = math.tan(math.radians(fov_deg) / 2)
    ys = (1.0 - 2.0 * (np.arange(H) + 0.5) / H) * th
    xs = (2.0 * (np.arange(W) + 0.5) / W - 1.0) * th * (W / H)
    d = (fwd[None, None, :] + xs[None, :, None] * right[None, None, :]
         + ys[:, None, None] * cup[None, None, :])
    d = _unit(d)
    b = np.sum(d * eye, axis=-1)
    c = float(np.dot(eye, eye)) - bound * bound
    disc = b * b - c
    if np.any(disc <= 0):
        raise ValueError("a camera ray misses the bounding sphere")
    s = np.sqrt(disc)
    o = np.broadcast_to(eye, d.shape).copy()
    return o, d, -b - s, -b + s


def tile_order(H: int, W: int, S: int, tile: int = 8):
    """Flat index map for the tile-coherent query layout.

    Query k of the tiled layout is sample ``s`` of pixel ``(i, j)`` with
    k = ((tile_row * (W/tile) + tile_col) * S + s) * tile^2 + (i%tile)*tile + j%tile.
    Returns (pixel_flat[Q], sample[Q]) as int64 arrays; pixel_flat = i*W + j."""
    if H % tile or W % tile:
        raise ValueError("image size must be a multiple of the tile size")
    ty, tx = H // tile, W // tile
    T = np.arange(ty * tx)
    ti, tj = T // tx, T % tx
    ly, lx = np.divmod(np.arange(tile * tile), tile)
    i = ti[:, None, None] * tile + ly[None, None, :]
    j = tj[:, None, None] * tile + lx[None, None, :]
    pix = np.broadcast_to(i * W + j, (T.size, S, tile * tile))
    smp = np.broadcast_to(np.arange(S)[None, :, None], (T.size, S, tile * tile))
    return pix.reshape(-1).copy(), smp.reshape(-1).copy()


def ray_samples(eye, H: int, W: int, S: int, seed: int, order: str = "tile",
                tile: int = 8, fov_deg: float = 50.0):
    """Stratified samples t_j = t_in + (j + u_j)(t_out - t_in)/S, u ~ U(0,1)
    (drawn as an [H,W,S] array), on the rays of ``camera_rays``.

    order="ray": query index = (i*W + j)*S + s (samples of a ray contiguous).
    order="tile": the tile-coherent layout of ``tile_order``: 64 consecutive
    queries are one sample index of an 8x8 pixel tile.
    Returns float32 x[H*W*S, 3]."""
    o, d, t0, t1 = camera_rays(eye, H, W, fov_deg)
    rng = np.random.default_rng(seed)
    u = rng.uniform(size=(H, W, S))
    Q = H * W * S
    out = np.empty((Q, 3), dtype=np.float32)
    o = o.reshape(-1, 3)
    d = d.reshape(-1, 3)
    t0 = t0.reshape(-1)
    dt = (t1.reshape(-1) - t0) / S
    u = u.reshape(H * W, S)
    if order == "ray":
        step = max(1, (1 << 22) // S)
        for a in range(0, H * W, step):
            b = min(H * W, a + step)
            t = t0[a:b, None] + (np.arange(S)[None, :] + u[a:b]) * dt[a:b, None]
            x = o[a:b, None, :] + t[..., None] * d[a:b, None, :]
            out[a * S:b * S] = x.reshape(-1, 3)
    elif order == "tile":
        pix, smp = tile_order(H, W, S, tile)
        step = 1 << 22
        for a in range(0, Q, step):
            b = min(Q, a + step)
            pp, ss = pix[a:b], smp[a:b]
            t = t0[pp] + (ss + u[pp, ss]) * dt[pp]
            out[a:b] = o[pp] + t[:, None] * d[pp]
    else:
        raise ValueError(order)
    return out


def sfm_camera(seed: int, radius: float = 3.0):
    """Camera position radius * u with u uniform on the unit sphere."""
    rng = np.random.default_rng(seed)
    return radius * _unit(rng.standard_normal(3))


def cotangents(Q: int, C: int, seed: int):
    """Upstream gradients dL/df ~ N(0,1), float32 [Q, C]."""
    rng = np.random.default_rng(seed)
    out = np.empty((Q, C), dtype=np.float32)
    step = 1 << 22
    for a in range(0, Q, step):
        b = min(Q, a + step)
        out[a:b] = rng.standard_normal((b - a, C))
    return out


def appearance_attrs(M: int, K: int, seed: int):
    """K appearance attributes per point (the learned features that Sec. 7.1
    feeds to its radiance network), drawn N(0,1) as at a random
    initialisation.  float32 [M, K]."""
    rng = np.random.default_rng(seed)
    out = np.empty((M, K), dtype=np.float32)
    step = 1 << 20
    for a in range(0, M, step):
        b = min(M, a + step)
        out[a:b] = rng.standard_normal((b - a, K))
    return out


def sfm_1m(order: str = "tile", H: int = 512, W: int = 512, S: int = 128):
    """The 1M-point scene with its 512x512x128 query set."""
    p, n, A, attrs = sfm_cloud(SFM_1M_SURFACE, SFM_1M_OUTLIERS, 10)
    eye = sfm_camera(11)
    x = ray_samples(eye, H, W, S, 12, order=order)
    return p, n, A, attrs, x


def fibonacci_sphere(M: int, radius: float = 1.0):
    """Deterministic near-uniform points on a sphere (golden-angle spiral),
    outward normals, equal areas 4 pi R^2 / M.  float32 p, n, A."""
    i = np.arange(M, dtype=np.float64) + 0.5
    z = 1.0 - 2.0 * i / M
    r = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    phi = i * math.pi * (3.0 - math.sqrt(5.0))
    n = np.stack([r * np.cos(phi), r * np.sin(phi), z], axis=1)
    A = np.full(M, 4.0 * math.pi * radius * radius / M)
    return (radius * n).astype(np.float32), n.astype(np.float32), A.astype(np.float32)


def pixel_ray_samples(eye, H: int, W: int, S: int, seed: int, n_rays: int, pix_seed: int,
                      fov_deg: float = 50.0):
    """Stratified samples on ``n_rays`` pixels drawn (seed ``pix_seed``) from
    an H x W pinhole image.  Returns (pixels[n_rays], x[n_rays*S, 3]) with the
    samples of each ray contiguous."""
    o, d, t0, t1 = camera_rays(eye, H, W, fov_deg)
    pix = np.sort(np.random.default_rng(pix_seed).choice(H * W, size=n_rays, replace=False))
    u = np.random.default_rng(seed).uniform(size=(n_rays, S))
    o, d = o.reshape(-1, 3)[pix], d.reshape(-1, 3)[pix]
    t0, t1 = t0.reshape(-1)[pix], t1.reshape(-1)[pix]
    t = t0[:, None] + (np.arange(S)[None, :] + u) * ((t1 - t0) / S)[:, None]
    x = o[:, None, :] + t[..., None] * d[:, None, :]
    return pix, x.reshape(-1, 3).astype(np.float32)
