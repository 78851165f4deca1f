"""Seeded synthetic inputs for the regularized dipole-sum hot path.

This package only draws input arrays (oriented point clouds, query points on
camera rays, multi-view ray batches, cotangents) and, in ``render``, holds the
volume-rendering proxy that turns field values into a loss for the tests and
the benchmark.  It contains none of the dipole-sum arithmetic, so both the
FP64 reference in ``oracle/`` and the GPU library consume exactly the same
FP32 bits without sharing any of the method's code.
"""
from .scenes import (  # noqa: F401
    sphere_cloud, sphere_queries, sphere_probes, sfm_cloud, camera_rays, deep_cluster_cloud, deep_cluster_probes,
    ray_samples, tile_order, cotangents, appearance_attrs, sfm_camera, sfm_1m, fibonacci_sphere, pixel_ray_samples,
    CONFIGS,
    SFM_1M_SURFACE, SFM_1M_OUTLIERS, SFM_4M_SURFACE, SFM_4M_OUTLIERS, SFM_8M_SURFACE, SFM_8M_OUTLIERS,
)
from .batched import (  # noqa: F401
    SFM_8M_RES, PRIMARY_SAMPLES, SHADOW_SAMPLES, RayBatch, make_ray_batch, sfm_8m_cloud, tile_rays,
    tile_camera_rays, synthetic_crossings,
    view_eyes, winding_cloud,
)
