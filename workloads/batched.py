"""Uneven multi-view ray batch with point lights (the batched workload).

Several pinhole views of one scene at different square resolutions are traced
together: the stratified samples of every view are concatenated into one query
batch, each view in the tile-coherent layout of ``tile_order`` (64 consecutive
queries are one sample index of an 8 x 8 pixel tile).  Each view has one point
light; the render proxy in ``workloads.render`` turns the first crossing of
the geometry field into a shadow ray towards that light (Sec. 7.1 of the paper
uses shadow rays for direct illumination).

Only seeded draws and camera geometry live here.  Host-side draws use NumPy's
PCG64; the per-sample positions are assembled on the device in float64 and
cast once to float32.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from .scenes import SFM_8M_OUTLIERS, SFM_8M_SURFACE, _random_rotation, _unit, camera_rays, sfm_cloud

SFM_8M_RES = (256, 320, 384, 512, 640, 768, 896, 1024)
PRIMARY_SAMPLES = 128
SHADOW_SAMPLES = 64
TILE = 8
CAMERA_RADIUS = 3.0
LIGHT_RADIUS = 4.0
BOUND = math.sqrt(3.0)


def winding_cloud(n_surface: int, n_outliers: int, seed: int):
    """``sfm_cloud`` with the geometry attribute set to 1 for every point, so
    channel 0 is the regularized winding number (the paper's initialisation of
    the geometry field, Sec. 4): it is ~1 inside the shapes and ~0 outside and
    its 1/2 level set is the reconstructed surface.  Colours as in sfm_cloud."""
    p, n, A, attrs = sfm_cloud(n_surface, n_outliers, seed)
    attrs[:, 0] = 1.0
    return p, n, A, attrs


def sfm_8m_cloud():
    """8,388,608 points: 7,969,178 on the shapes plus 419,430 outliers."""
    return winding_cloud(SFM_8M_SURFACE, SFM_8M_OUTLIERS, 30)


def view_eyes(n_views: int, rng, radius: float = CAMERA_RADIUS):
    """Camera centres on the radius sphere: Fibonacci-spiral directions turned
    by one random rotation drawn from ``rng``."""
    i = np.arange(n_views, dtype=np.float64) + 0.5
    z = 1.0 - 2.0 * i / n_views
    r = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    phi = i * math.pi * (3.0 - math.sqrt(5.0))
    dirs = np.stack([r * np.cos(phi), r * np.sin(phi), z], axis=1)
    rot = _random_rotation(rng)
    return radius * _unit(dirs @ rot.T)


def tile_rays(res: int, tile: int = TILE):
    """Pixel index (i*res + j) of each ray in tile order: ray t*64 + lane is
    pixel (ti*tile + lane//tile, tj*tile + lane%tile) of tile t = ti*(res/tile) + tj."""
    if res % tile:
        raise ValueError("resolution must be a multiple of the tile size")
    nt = res // tile
    t = np.arange(nt * nt)
    ly, lx = np.divmod(np.arange(tile * tile), tile)
    i = (t // nt)[:, None] * tile + ly[None, :]
    j = (t % nt)[:, None] * tile + lx[None, :]
    return (i * res + j).reshape(-1)


def tile_camera_rays(eye, res: int, fov_deg: float = 50.0):
    """The rays of a res x res pinhole camera at ``eye`` (``camera_rays``) in
    tile order (``tile_rays``), FP32: o, d [R, 3], t_in, t_out [R]."""
    o, d, t0, t1 = camera_rays(eye, res, res, fov_deg)
    pix = tile_rays(res)
    return (np.ascontiguousarray(o.reshape(-1, 3)[pix], dtype=np.float32),
            np.ascontiguousarray(d.reshape(-1, 3)[pix], dtype=np.float32),
            np.ascontiguousarray(t0.reshape(-1)[pix], dtype=np.float32),
            np.ascontiguousarray(t1.reshape(-1)[pix], dtype=np.float32))


def synthetic_crossings(R: int, n: int, seed: int, S: int = 80):
    """Made-up results of a dense march over R rays of n samples, for testing
    the sample placement on its own: a crossing index j in [-1, n-2] (the
    first four rays fixed to 0, n-2, -1, 1), the two field values around it
    straddling 1/2 in either direction, and the placement jitter u [R, S] in
    [0, 1).  Returns (j int32, vj, vj1, u) as float32 arrays."""
    rng = np.random.default_rng(seed)
    j = rng.integers(-1, n - 1, size=R).astype(np.int32)
    j[:4] = np.array([0, n - 2, -1, 1])[:min(4, R)]
    lo = rng.uniform(0.0, 0.5, R).astype(np.float32)
    hi = rng.uniform(0.5, 1.0, R).astype(np.float32)
    hi[hi == np.float32(0.5)] = np.float32(0.75)
    up = rng.uniform(size=R) < 0.5
    vj = np.where(up, lo, hi).astype(np.float32)
    vj1 = np.where(up, hi, lo).astype(np.float32)
    u = rng.uniform(size=(R, S)).astype(np.float32)
    return j, vj, vj1, u


@dataclass
class RayBatch:
    """Device tensors of a multi-view batch (all rays in tile order, views
    concatenated).  x[Q,3] primary samples with Q = n_rays * S laid out as
    [tile, sample, lane]; ray_light[n_rays,3] the light of each ray's view;
    target[n_rays,3] the target colours; shadow_u[n_rays,S_shadow] the
    stratification jitter of the shadow samples."""
    x: object
    ray_light: object
    target: object
    shadow_u: object
    res: tuple
    S: int
    S_shadow: int
    eyes: np.ndarray
    lights: np.ndarray
    ray_offsets: tuple

    @property
    def n_rays(self):
        return self.target.shape[0]

    @property
    def Q(self):
        return self.x.shape[0]


def make_ray_batch(res=SFM_8M_RES, S: int = PRIMARY_SAMPLES, S_shadow: int = SHADOW_SAMPLES,
                   seeds=(31, 32), device="cuda", fov_deg: float = 50.0):
    """Builds the batch on ``device``.

    seeds[0]: view rotation, then the [res, res, S] sample jitter of each view
    in order; seeds[1]: the point lights (uniform on the radius-4 sphere), the
    U(0,1)^3 target colour of every ray, then the shadow-sample jitter.
    Samples t_j = t_in + (j + u_j)(t_out - t_in)/S on the part of each ray
    inside |x| <= sqrt(3)."""
    import torch
    n_views = len(res)
    rng_cam = np.random.default_rng(seeds[0])
    eyes = view_eyes(n_views, rng_cam)
    xs, offsets, rays_light_idx = [], [0], []
    for v, R in enumerate(res):
        o, d, t0, t1 = camera_rays(eyes[v], R, R, fov_deg, BOUND)
        u = rng_cam.uniform(size=(R * R, S)).astype(np.float32)
        pix = tile_rays(R)
        nt = pix.size // (TILE * TILE)
        dt = torch.from_numpy(d.reshape(-1, 3)[pix]).to(device).view(nt, 1, TILE * TILE, 3)
        ti = torch.from_numpy(t0.reshape(-1)[pix]).to(device).view(nt, 1, TILE * TILE)
        step = torch.from_numpy(((t1 - t0) / S).reshape(-1)[pix]).to(device).view(nt, 1, TILE * TILE)
        uu = torch.from_numpy(u[pix]).to(device).view(nt, TILE * TILE, S).transpose(1, 2).to(torch.float64)
        j = torch.arange(S, device=device, dtype=torch.float64).view(1, S, 1)
        t = ti + (j + uu) * step
        eye = torch.tensor(eyes[v], device=device, dtype=torch.float64)
        xs.append((eye + t[..., None] * dt).to(torch.float32).reshape(-1, 3))
        del dt, ti, step, uu, t
        offsets.append(offsets[-1] + R * R)
        rays_light_idx.append(np.full(R * R, v, dtype=np.int64))
    x = torch.cat(xs) if len(xs) > 1 else xs[0]
    del xs
    n_rays = offsets[-1]
    rng_l = np.random.default_rng(seeds[1])
    lights = LIGHT_RADIUS * _unit(rng_l.standard_normal((n_views, 3)))
    target = rng_l.uniform(size=(n_rays, 3)).astype(np.float32)
    shadow_u = np.empty((n_rays, S_shadow), dtype=np.float32)
    step = 1 << 20
    for a in range(0, n_rays, step):
        b = min(n_rays, a + step)
        shadow_u[a:b] = rng_l.uniform(size=(b - a, S_shadow))
    ray_light = torch.from_numpy(lights[np.concatenate(rays_light_idx)].astype(np.float32)).to(device)
    return RayBatch(x=x, ray_light=ray_light, target=torch.from_numpy(target).to(device),
                    shadow_u=torch.from_numpy(shadow_u).to(device), res=tuple(res), S=S, S_shadow=S_shadow,
                    eyes=eyes, lights=lights, ray_offsets=tuple(offsets))
