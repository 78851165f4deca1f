"""Helpers for GPU-vs-oracle comparisons (test infrastructure)."""
from __future__ import annotations

import numpy as np

# FP32-stored tolerance on errors normalised by the per-query absolute sums.
TOL_FP32 = 1e-5
# BF16-stored: round-to-nearest-even to 8 significant bits leaves each stored
# value within 2^-8 of itself (relative), and |dD.d| <= 2^-8 |D||d|
# (Cauchy-Schwarz), so the normalised error is bounded by 2^-8 (plus the FP32
# part) whatever the workload: the guaranteed bound.  With the top-level node
# moments kept in FP32, the stated 2e-3 target (TARGET_BF16) holds for every
# query of the 4M-point precision workloads; results computed from BF16 values
# are also held to the FP32 bar against an oracle fed the same rounded values.
TOL_BF16 = 2.0 ** -8 + TOL_FP32
TARGET_BF16 = 2e-3


def norm_err_all(got, ref, scale):
    """Per-element normalised errors (flattened)."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    scale = np.asarray(scale, dtype=np.float64)
    while scale.ndim < ref.ndim:
        scale = scale[..., None]
    return (np.abs(got - ref) / np.maximum(scale, 1e-300)).reshape(-1)


def norm_err(got, ref, scale):
    """max |got - ref| / scale (scale broadcast over trailing axes)."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    scale = np.asarray(scale, dtype=np.float64)
    while scale.ndim < ref.ndim:
        scale = scale[..., None]
    scale = np.maximum(scale, 1e-300)
    if got.size == 0:
        return 0.0
    return float(np.max(np.abs(got - ref) / scale))


def to_dev(*arrays):
    import torch
    return [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in arrays]


def to_host(t):
    return t.detach().cpu().numpy()


def node_abs_sums(perm, nodes, A, mu):
    """Per node and channel: sum over its points of A_m |mu_m,c| (|n_m| = 1):
    the absolute scale of the node dipole D_t,c."""
    w = (A.astype(np.float64)[perm][:, None] * np.abs(mu.astype(np.float64)[perm]))
    cs = np.concatenate([np.zeros((1, w.shape[1])), np.cumsum(w, axis=0)])
    b = nodes[:, 4].astype(np.int64)
    e = b + nodes[:, 5].astype(np.int64)
    return cs[e] - cs[b]


def normwise(got, ref):
    """||got - ref||_2 / ||ref||_2 over all elements (0 for an empty or zero reference)."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = float(np.linalg.norm(ref))
    return float(np.linalg.norm(got - ref)) / den if den > 0 else 0.0
