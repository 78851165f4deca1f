"""Thin ctypes binding of libdps.so (argument marshalling only).

Every function mirrors an entry point of ``include/dps.h`` under the same
name.  Tensors are torch CUDA float32 (int32 / int64 where stated), contiguous,
on the tree's device; work is enqueued on torch's current stream.  Nothing here
computes: every step runs in the HIP kernels of the library, and a missing
library raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes as ct
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdps.so")

DPS_OK, DPS_ERR_INVALID, DPS_ERR_OOM, DPS_ERR_DEVICE, DPS_ERR_STATE = range(5)
DPS_STORE_FP32, DPS_STORE_BF16 = 0, 1
STORAGE = {"fp32": DPS_STORE_FP32, "bf16": DPS_STORE_BF16}
DPS_KERNEL_DIPOLE, DPS_KERNEL_MONOPOLE = 0, 1
KERNEL = {"dipole": DPS_KERNEL_DIPOLE, "monopole": DPS_KERNEL_MONOPOLE}

EXPORTED = (
    "dps_build", "dps_build_kernel", "dps_get_kernel", "dps_set_attributes", "dps_query", "dps_query_counts", "dps_adjoint_zero",
    "dps_adjoint_accumulate", "dps_adjoint_finalize", "dps_adjoint", "dps_export_tree",
    "dps_tree_info", "dps_set_launch", "dps_get_launch", "dps_set_split", "dps_get_split", "dps_query_channels",
    "dps_adjoint_accumulate_channels", "dps_adjoint_accumulate_grad", "dps_adjoint_accumulate_ext",
    "dps_adjoint_accumulate_from_forward",
    "dps_adjoint_finalize_ext", "dps_set_normals", "dps_query_grid", "dps_ray_march", "dps_ray_march_harnack", "dps_ray_resample",
    "dps_adjoint_noalloc", "dps_check", "dps_set_step_limit", "dps_set_memory_limit", "dps_destroy",
    "dps_status_string", "dps_last_error",
)

_lib = None


class DpsError(RuntimeError):
    def __init__(self, status: int, fn: str, message: str):
        super().__init__(f"{fn} failed ({status}): {message}")
        self.status = status


def load():
    """Loads libdps.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2405_16788_amd.build`")
    try:  # share the HIP runtime torch already loaded, if any
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ct.CDLL(LIB_PATH)
    vp, i64, i32, f32 = ct.c_void_p, ct.c_int64, ct.c_int32, ct.c_float
    sig = {
        "dps_build": [vp, vp, vp, vp, i64, i32, i32, ct.c_int, vp, ct.POINTER(vp)],
        "dps_build_kernel": [vp, vp, vp, vp, i64, i32, i32, ct.c_int, ct.c_int, vp, ct.POINTER(vp)],
        "dps_get_kernel": [vp, ct.POINTER(i32)],
        "dps_set_attributes": [vp, vp, vp],
        "dps_query": [vp, vp, i64, f32, f32, vp, vp, vp],
        "dps_query_counts": [vp, vp, i64, f32, vp, vp],
        "dps_adjoint_zero": [vp, vp],
        "dps_check": [vp, vp],
        "dps_set_launch": [vp, i32, i32, i32],
        "dps_get_launch": [vp, ct.POINTER(i32), ct.POINTER(i32), ct.POINTER(i32)],
        "dps_set_split": [vp, i32, i32, i32],
        "dps_get_split": [vp, ct.POINTER(i32), ct.POINTER(i32), ct.POINTER(i32)],
        "dps_query_channels": [vp, vp, i64, vp, f32, f32, i32, i32, vp, vp, vp],
        "dps_adjoint_accumulate_channels": [vp, vp, i64, vp, f32, f32, i32, i32, vp, vp, vp],
        "dps_adjoint_accumulate_grad": [vp, vp, i64, vp, f32, f32, i32, i32, vp, vp, vp, vp],
        "dps_adjoint_accumulate_from_forward": [vp, vp, i64, vp, f32, f32, i32, i32, vp, vp, vp, vp],
        "dps_adjoint_accumulate_ext": [vp, vp, i64, vp, f32, f32, i32, i32, vp, vp, i32, vp, vp],
        "dps_adjoint_finalize_ext": [vp, vp, vp, vp, vp],
        "dps_set_normals": [vp, vp, vp],
        "dps_query_grid": [vp, vp, vp, vp, f32, f32, i32, i32, vp, vp, vp],
        "dps_ray_march": [vp, vp, vp, vp, vp, i64, i32, f32, f32, i32, f32, vp, vp, vp],
        "dps_ray_march_harnack": [vp, vp, vp, vp, vp, i64, i32, f32, f32, i32, f32, f32, vp, vp, vp, vp],
        "dps_ray_resample": [vp, vp, vp, vp, i64, i32, vp, vp, f32, vp, i32, i32, i32, f32, i32, vp, vp, vp],
        "dps_adjoint_accumulate": [vp, vp, i64, f32, f32, vp, vp, vp],
        "dps_adjoint_finalize": [vp, vp, vp],
        "dps_adjoint": [vp, vp, i64, f32, f32, vp, vp, vp, vp],
        "dps_adjoint_noalloc": [vp, vp, i64, f32, f32, vp, vp, vp, vp],
        "dps_export_tree": [vp, vp, vp, vp, vp, vp, vp],
        "dps_tree_info": [vp, ct.POINTER(i64), ct.POINTER(i32), ct.POINTER(i64), ct.POINTER(i64),
                          ct.POINTER(i32)],
        "dps_set_step_limit": [vp, i64],
        "dps_set_memory_limit": [i64],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ct.c_int
    lib.dps_destroy.argtypes = [vp]
    lib.dps_destroy.restype = None
    lib.dps_status_string.argtypes = [ct.c_int]
    lib.dps_status_string.restype = ct.c_char_p
    lib.dps_last_error.argtypes = []
    lib.dps_last_error.restype = ct.c_char_p
    _lib = lib
    return lib


def _check(status: int, fn: str):
    if status != DPS_OK:
        raise DpsError(status, fn, load().dps_last_error().decode(errors="replace"))


def _stream(device=None):
    import torch
    return ct.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t, dtype=None, shape=None, device=None, name="tensor"):
    """Validated device pointer of a contiguous CUDA tensor (None -> NULL)."""
    if t is None:
        return None
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if device is not None and t.device != device:
        raise ValueError(f"{name} is on {t.device}, the tree on {device}")
    return ct.c_void_p(t.data_ptr())


class Tree:
    """Owning handle of a dps_tree (destroyed with the object)."""

    def __init__(self, handle, device, M, C, storage, kernel="dipole"):
        self._h = handle
        self.device = device
        self.M = M
        self.C = C
        self.storage = storage
        self.kernel = kernel

    @property
    def handle(self):
        if self._h is None:
            raise ValueError("tree has been destroyed")
        return self._h

    def __del__(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _lib.dps_destroy(self._h)
            self._h = None


def dps_build(p, n, A, attrs, leaf_size: int = 16, storage: str = "fp32", kernel: str = "dipole") -> Tree:
    """Builds a tree (``dps_build_kernel``); kernel "dipole" or "monopole"
    (appearance channels with the foreshortening factor dropped)."""
    import torch
    lib = load()
    if kernel not in KERNEL:
        raise ValueError(f"kernel must be one of {sorted(KERNEL)}")
    M = p.shape[0]
    C = attrs.shape[1] if attrs.dim() == 2 else 1
    dev = p.device
    f = torch.float32
    args = (_ptr(p, f, (M, 3), name="p"), _ptr(n, f, (M, 3), dev, "n"), _ptr(A, f, (M,), dev, "A"),
            _ptr(attrs, f, (M, C) if attrs.dim() == 2 else (M,), dev, "attrs"))
    h = ct.c_void_p()
    with torch.cuda.device(dev):
        _check(lib.dps_build_kernel(*args, M, C, int(leaf_size), STORAGE[storage], KERNEL[kernel], _stream(dev),
                                    ct.byref(h)), "dps_build_kernel")
    return Tree(h, dev, M, C, storage, kernel)


def dps_get_kernel(tree: Tree) -> str:
    k = ct.c_int32()
    _check(load().dps_get_kernel(tree.handle, ct.byref(k)), "dps_get_kernel")
    return {v: n for n, v in KERNEL.items()}[k.value]


def dps_set_attributes(tree: Tree, attrs):
    import torch
    p = _ptr(attrs, torch.float32, (tree.M, tree.C) if attrs.dim() == 2 else (tree.M,), tree.device, "attrs")
    _check(load().dps_set_attributes(tree.handle, p, _stream(tree.device)), "dps_set_attributes")


def dps_query(tree: Tree, x, beta: float, eps: float, grad: bool = True, f_out=None, g_out=None):
    """Returns (f[Q,C], grad[Q,C,3] or None)."""
    import torch
    Q = x.shape[0]
    xp = _ptr(x, torch.float32, (Q, 3), tree.device, "x")
    f = f_out if f_out is not None else torch.empty((Q, tree.C), device=tree.device, dtype=torch.float32)
    g = g_out if g_out is not None else (
        torch.empty((Q, tree.C, 3), device=tree.device, dtype=torch.float32) if grad else None)
    _check(load().dps_query(tree.handle, xp, Q, float(beta), float(eps),
                            _ptr(f, torch.float32, (Q, tree.C), tree.device, "f"),
                            _ptr(g, torch.float32, (Q, tree.C, 3), tree.device, "grad"),
                            _stream(tree.device)), "dps_query")
    return f, g


def dps_query_counts(tree: Tree, x, beta: float):
    """Returns int32 [Q,4]: visited nodes, far-field nodes, leaves opened, near points."""
    import torch
    Q = x.shape[0]
    counts = torch.empty((Q, 4), device=tree.device, dtype=torch.int32)
    _check(load().dps_query_counts(tree.handle, _ptr(x, torch.float32, (Q, 3), tree.device, "x"), Q,
                                   float(beta), _ptr(counts, torch.int32), _stream(tree.device)),
           "dps_query_counts")
    return counts


def dps_adjoint_zero(tree: Tree):
    _check(load().dps_adjoint_zero(tree.handle, _stream(tree.device)), "dps_adjoint_zero")


def dps_adjoint_accumulate(tree: Tree, x, beta: float, eps: float, df, want_dx: bool = True, dx_out=None):
    """Stage 1; returns dx[Q,3] (or None)."""
    import torch
    Q = x.shape[0]
    dx = dx_out if dx_out is not None else (
        torch.empty((Q, 3), device=tree.device, dtype=torch.float32) if want_dx else None)
    _check(load().dps_adjoint_accumulate(
        tree.handle, _ptr(x, torch.float32, (Q, 3), tree.device, "x"), Q, float(beta), float(eps),
        _ptr(df, torch.float32, (Q, tree.C), tree.device, "df"),
        _ptr(dx, torch.float32, (Q, 3), tree.device, "dx"), _stream(tree.device)), "dps_adjoint_accumulate")
    return dx


def dps_adjoint_finalize(tree: Tree, dattrs_out=None):
    """Stage 2; returns dL/dattrs [M,C] in caller point order."""
    import torch
    d = dattrs_out if dattrs_out is not None else torch.empty((tree.M, tree.C), device=tree.device,
                                                              dtype=torch.float32)
    _check(load().dps_adjoint_finalize(tree.handle, _ptr(d, torch.float32, (tree.M, tree.C), tree.device,
                                                         "dattrs"), _stream(tree.device)),
           "dps_adjoint_finalize")
    return d


def dps_adjoint(tree: Tree, x, beta: float, eps: float, df, want_dx: bool = True):
    """zero + accumulate + finalize; returns (dattrs[M,C], dx[Q,3] or None)."""
    import torch
    Q = x.shape[0]
    d = torch.empty((tree.M, tree.C), device=tree.device, dtype=torch.float32)
    dx = torch.empty((Q, 3), device=tree.device, dtype=torch.float32) if want_dx else None
    _check(load().dps_adjoint(tree.handle, _ptr(x, torch.float32, (Q, 3), tree.device, "x"), Q,
                              float(beta), float(eps), _ptr(df, torch.float32, (Q, tree.C), tree.device, "df"),
                              _ptr(d, torch.float32), _ptr(dx, torch.float32), _stream(tree.device)),
           "dps_adjoint")
    return d, dx


def dps_adjoint_noalloc(tree: Tree, x, beta: float, eps: float, df, dattrs_out, dx_out=None):
    """dps_adjoint with its working buffers in the library's static per-device
    workspace (allocates nothing; outputs must be given).  Calls that overlap
    in time on one device race."""
    import torch
    Q = x.shape[0]
    _check(load().dps_adjoint_noalloc(tree.handle, _ptr(x, torch.float32, (Q, 3), tree.device, "x"), Q,
                                      float(beta), float(eps), _ptr(df, torch.float32, (Q, tree.C), tree.device, "df"),
                                      _ptr(dattrs_out, torch.float32, (tree.M, tree.C), tree.device, "dattrs"),
                                      _ptr(dx_out, torch.float32, (Q, 3), tree.device, "dx"), _stream(tree.device)),
           "dps_adjoint_noalloc")
    return dattrs_out, dx_out


def dps_tree_info(tree: Tree) -> dict:
    n, depth, b, m, c = ct.c_int64(), ct.c_int32(), ct.c_int64(), ct.c_int64(), ct.c_int32()
    _check(load().dps_tree_info(tree.handle, ct.byref(n), ct.byref(depth), ct.byref(b), ct.byref(m),
                                ct.byref(c)), "dps_tree_info")
    return {"n_nodes": n.value, "depth": depth.value, "bytes": b.value, "n_points": m.value,
            "channels": c.value}


def dps_export_tree(tree: Tree) -> dict:
    """Canonical arrays as CUDA tensors: codes (int64 view of uint64), perm
    (int32 view of uint32), nodes[N,6], geom[N,4], moments[N,C,3]."""
    import torch
    info = dps_tree_info(tree)
    N, M, C = info["n_nodes"], tree.M, tree.C
    dev = tree.device
    codes = torch.empty(M, device=dev, dtype=torch.int64)
    perm = torch.empty(M, device=dev, dtype=torch.int32)
    nodes = torch.empty((N, 6), device=dev, dtype=torch.int32)
    geom = torch.empty((N, 4), device=dev, dtype=torch.float32)
    mom = torch.empty((N, C, 3), device=dev, dtype=torch.float32)
    _check(load().dps_export_tree(tree.handle, _ptr(codes), _ptr(perm), _ptr(nodes), _ptr(geom), _ptr(mom),
                                  _stream(dev)), "dps_export_tree")
    return {"codes": codes, "perm": perm, "nodes": nodes, "geom": geom, "moments": mom}


LAUNCH_XCD_QUERY, LAUNCH_XCD_ADJOINT, LAUNCH_PERSISTENT_QUERY, LAUNCH_PERSISTENT_ADJOINT = 1, 2, 4, 8
LAUNCH_MARCH_WHOLE = 16  # dps_ray_march: one ray per lane instead of ray-major chunks


def dps_set_launch(tree: Tree, query_k: int = 0, adjoint_k: int = 0, flags: int = -1):
    """Queries per lane of the traversal kernels (1, 2, 4; 0 keeps) and the
    launch flags (LAUNCH_* bits; -1 keeps)."""
    _check(load().dps_set_launch(tree.handle, int(query_k), int(adjoint_k), int(flags)), "dps_set_launch")


def dps_get_launch(tree: Tree):
    a, b, c = ct.c_int32(), ct.c_int32(), ct.c_int32()
    _check(load().dps_get_launch(tree.handle, ct.byref(a), ct.byref(b), ct.byref(c)), "dps_get_launch")
    return {"query": a.value, "adjoint": b.value, "flags": c.value}


def dps_set_split(tree: Tree, query_parts: int = 0, adjoint_parts: int = 0, cut_level: int = -1):
    """Subtree-split walks for small batches: parts (1, 2, 4, 8; 0 keeps)
    for the query and the adjoint accumulation, and the cut level (-1
    keeps)."""
    _check(load().dps_set_split(tree.handle, int(query_parts), int(adjoint_parts), int(cut_level)), "dps_set_split")


def dps_get_split(tree: Tree):
    a, b, c = ct.c_int32(), ct.c_int32(), ct.c_int32()
    _check(load().dps_get_split(tree.handle, ct.byref(a), ct.byref(b), ct.byref(c)), "dps_get_split")
    return {"query": a.value, "adjoint": b.value, "cut": c.value}


def dps_query_channels(tree: Tree, x, beta: float, eps: float, c_begin: int, n_channels: int,
                       grad: bool = True, f_out=None, g_out=None, q_count=None):
    """Channels [c_begin, c_begin+n_channels) only; returns (f[Q,n], grad[Q,n,3] or None).
    q_count: optional int64 CUDA tensor [1]; only its first rows are processed."""
    import torch
    Q = x.shape[0]
    f = f_out if f_out is not None else torch.empty((Q, n_channels), device=tree.device, dtype=torch.float32)
    g = g_out if g_out is not None else (
        torch.empty((Q, n_channels, 3), device=tree.device, dtype=torch.float32) if grad else None)
    _check(load().dps_query_channels(tree.handle, _ptr(x, torch.float32, (Q, 3), tree.device, "x"), Q,
                                     _ptr(q_count, torch.int64, (1,), tree.device, "q_count"),
                                     float(beta), float(eps), int(c_begin), int(n_channels),
                                     _ptr(f, torch.float32, (Q, n_channels), tree.device, "f"),
                                     _ptr(g, torch.float32, (Q, n_channels, 3), tree.device, "grad"),
                                     _stream(tree.device)), "dps_query_channels")
    return f, g


def dps_adjoint_accumulate_channels(tree: Tree, x, beta: float, eps: float, c_begin: int, n_channels: int,
                                    df, want_dx: bool = True, dx_out=None, q_count=None):
    """Stage 1 for a channel range; df rows hold n_channels entries."""
    import torch
    Q = x.shape[0]
    dx = dx_out if dx_out is not None else (
        torch.empty((Q, 3), device=tree.device, dtype=torch.float32) if want_dx else None)
    _check(load().dps_adjoint_accumulate_channels(
        tree.handle, _ptr(x, torch.float32, (Q, 3), tree.device, "x"), Q,
        _ptr(q_count, torch.int64, (1,), tree.device, "q_count"), float(beta), float(eps), int(c_begin),
        int(n_channels), _ptr(df, torch.float32, (Q, n_channels), tree.device, "df"),
        _ptr(dx, torch.float32, (Q, 3), tree.device, "dx"), _stream(tree.device)), "dps_adjoint_accumulate_channels")
    return dx


def dps_adjoint_accumulate_grad(tree: Tree, x, beta: float, eps: float, dg, df=None, c_begin: int = 0,
                                n_channels=None, want_dx: bool = True, dx_out=None, q_count=None):
    """Stage 1 for gradient cotangents dg[Q,n,3] (and optional value cotangents
    df[Q,n]) of channels [c_begin, c_begin+n); returns dx[Q,3] (or None)."""
    import torch
    Q = x.shape[0]
    n = tree.C - c_begin if n_channels is None else n_channels
    dx = dx_out if dx_out is not None else (
        torch.empty((Q, 3), device=tree.device, dtype=torch.float32) if want_dx else None)
    _check(load().dps_adjoint_accumulate_grad(
        tree.handle, _ptr(x, torch.float32, (Q, 3), tree.device, "x"), Q,
        _ptr(q_count, torch.int64, (1,), tree.device, "q_count"), float(beta), float(eps), int(c_begin), int(n),
        _ptr(df, torch.float32, (Q, n), tree.device, "df"),
        _ptr(dg, torch.float32, (Q, n, 3), tree.device, "dg"),
        _ptr(dx, torch.float32, (Q, 3), tree.device, "dx"), _stream(tree.device)), "dps_adjoint_accumulate_grad")
    return dx


def dps_adjoint_accumulate_from_forward(tree: Tree, x, beta: float, eps: float, df, grad, c_begin: int = 0,
                                        n_channels=None, want_dx: bool = True, dx_out=None, q_count=None):
    """Stage 1 for value cotangents df[Q,n] of channels [c_begin, c_begin+n)
    with dL/dx = sum_c df_c grad_c formed from the forward's gradients
    grad[Q,n,3] (same x, beta, eps and attributes); returns dx[Q,3] (or None)."""
    import torch
    Q = x.shape[0]
    n = tree.C - c_begin if n_channels is None else n_channels
    dx = dx_out if dx_out is not None else (
        torch.empty((Q, 3), device=tree.device, dtype=torch.float32) if want_dx else None)
    _check(load().dps_adjoint_accumulate_from_forward(
        tree.handle, _ptr(x, torch.float32, (Q, 3), tree.device, "x"), Q,
        _ptr(q_count, torch.int64, (1,), tree.device, "q_count"), float(beta), float(eps), int(c_begin), int(n),
        _ptr(df, torch.float32, (Q, n), tree.device, "df"),
        _ptr(grad, torch.float32, (Q, n, 3), tree.device, "grad"),
        _ptr(dx, torch.float32, (Q, 3), tree.device, "dx"), _stream(tree.device)),
        "dps_adjoint_accumulate_from_forward")
    return dx


WANT_NORMALS = 1
WANT_EPS = 2


def dps_adjoint_accumulate_ext(tree: Tree, x, beta: float, eps: float, df=None, dg=None, want: int = 0,
                               c_begin: int = 0, n_channels=None, want_dx: bool = True, dx_out=None, q_count=None):
    """Stage 1 for value and/or gradient cotangents, optionally accumulating
    the near-field part of dL/dnormals (WANT_NORMALS) and dL/deps (WANT_EPS);
    returns dx[Q,3] (or None)."""
    import torch
    Q = x.shape[0]
    n = tree.C - c_begin if n_channels is None else n_channels
    dx = dx_out if dx_out is not None else (
        torch.empty((Q, 3), device=tree.device, dtype=torch.float32) if want_dx else None)
    _check(load().dps_adjoint_accumulate_ext(
        tree.handle, _ptr(x, torch.float32, (Q, 3), tree.device, "x"), Q,
        _ptr(q_count, torch.int64, (1,), tree.device, "q_count"), float(beta), float(eps), int(c_begin), int(n),
        _ptr(df, torch.float32, (Q, n), tree.device, "df"), _ptr(dg, torch.float32, (Q, n, 3), tree.device, "dg"),
        int(want), _ptr(dx, torch.float32, (Q, 3), tree.device, "dx"), _stream(tree.device)),
        "dps_adjoint_accumulate_ext")
    return dx


def dps_adjoint_finalize_ext(tree: Tree, attrs: bool = True, normals: bool = False, eps: bool = False,
                             dattrs_out=None, dnormals_out=None, deps_out=None):
    """Stage 2 with optional outputs; returns (dattrs[M,C] or None,
    dnormals[M,3] or None, deps float64 tensor [1] or None)."""
    import torch
    dev = tree.device
    da = dattrs_out if dattrs_out is not None else (
        torch.empty((tree.M, tree.C), device=dev, dtype=torch.float32) if attrs else None)
    dn = dnormals_out if dnormals_out is not None else (
        torch.empty((tree.M, 3), device=dev, dtype=torch.float32) if normals else None)
    de = deps_out if deps_out is not None else (torch.empty(1, device=dev, dtype=torch.float64) if eps else None)
    _check(load().dps_adjoint_finalize_ext(tree.handle, _ptr(da, torch.float32, (tree.M, tree.C), dev, "dattrs"),
                                           _ptr(dn, torch.float32, (tree.M, 3), dev, "dnormals"),
                                           _ptr(de, torch.float64, (1,), dev, "deps"), _stream(dev)),
           "dps_adjoint_finalize_ext")
    return da, dn, de


def dps_set_normals(tree: Tree, normals):
    """Replaces the point normals [M,3] (caller order); call dps_set_attributes
    before the next query so the node moments follow."""
    import torch
    _check(load().dps_set_normals(tree.handle, _ptr(normals, torch.float32, (tree.M, 3), tree.device, "normals"),
                                  _stream(tree.device)), "dps_set_normals")


def dps_query_grid(tree: Tree, origin, spacing, dims, beta: float, eps: float, c_begin: int = 0,
                   n_channels=None, grad: bool = False, f_out=None, g_out=None):
    """Field at the points origin + (i, j, k) * spacing of an nx x ny x nz grid
    (dims = (nx, ny, nz)); returns (f[nz,ny,nx,n], grad[nz,ny,nx,n,3] or None)."""
    import torch
    n = tree.C - c_begin if n_channels is None else n_channels
    nx, ny, nz = (int(v) for v in dims)
    o = (ct.c_float * 3)(*[float(v) for v in origin])
    h = (ct.c_float * 3)(*[float(v) for v in spacing])
    d = (ct.c_int64 * 3)(nx, ny, nz)
    f = f_out if f_out is not None else torch.empty((nz, ny, nx, n), device=tree.device, dtype=torch.float32)
    g = g_out if g_out is not None else (
        torch.empty((nz, ny, nx, n, 3), device=tree.device, dtype=torch.float32) if grad else None)
    _check(load().dps_query_grid(tree.handle, ct.cast(o, ct.c_void_p), ct.cast(h, ct.c_void_p),
                                 ct.cast(d, ct.c_void_p), float(beta), float(eps), int(c_begin), int(n),
                                 _ptr(f, torch.float32, (nz, ny, nx, n), tree.device, "f"),
                                 _ptr(g, torch.float32, (nz, ny, nx, n, 3), tree.device, "grad"),
                                 _stream(tree.device)), "dps_query_grid")
    return f, g


def dps_ray_march(tree: Tree, o, d, tnear, tfar, n_samples: int = 1024, beta: float = 2.0, eps: float = 0.0,
                  channel: int = 0, level: float = 0.5, hit_out=None, values_out=None):
    """First crossing of channel ``channel`` through ``level`` along each ray
    (dense march of n_samples midpoints between tnear and tfar).  Returns
    (hit_index int32[R], -1 without a crossing; hit_values float32[R, 2])."""
    import torch
    R = o.shape[0]
    dev = tree.device
    hit = hit_out if hit_out is not None else torch.empty(R, device=dev, dtype=torch.int32)
    hv = values_out if values_out is not None else torch.empty((R, 2), device=dev, dtype=torch.float32)
    f = torch.float32
    _check(load().dps_ray_march(tree.handle, _ptr(o, f, (R, 3), dev, "o"), _ptr(d, f, (R, 3), dev, "d"),
                                _ptr(tnear, f, (R,), dev, "tnear"), _ptr(tfar, f, (R,), dev, "tfar"), R,
                                int(n_samples), float(beta), float(eps), int(channel), float(level),
                                _ptr(hit, torch.int32, (R,), dev, "hit_index"), _ptr(hv, f, (R, 2), dev, "hit_values"),
                                _stream(dev)), "dps_ray_march")
    return hit, hv


def dps_ray_march_harnack(tree: Tree, o, d, tnear, tfar, n_samples: int = 1024, beta: float = 2.0, eps: float = 0.0,
                          channel: int = 0, level: float = 0.5, lower: float = -0.25, hit_out=None, values_out=None,
                          evals_out=None, want_evals: bool = False):
    """dps_ray_march's outputs through the Harnack-accelerated march
    (``dps_ray_march_harnack``); ``lower`` bounds the field from below.
    Returns (hit_index, hit_values, evals int32[R] or None)."""
    import torch
    R = o.shape[0]
    dev = tree.device
    hit = hit_out if hit_out is not None else torch.empty(R, device=dev, dtype=torch.int32)
    hv = values_out if values_out is not None else torch.empty((R, 2), device=dev, dtype=torch.float32)
    ev = evals_out if evals_out is not None else (
        torch.empty(R, device=dev, dtype=torch.int32) if want_evals else None)
    f = torch.float32
    _check(load().dps_ray_march_harnack(
        tree.handle, _ptr(o, f, (R, 3), dev, "o"), _ptr(d, f, (R, 3), dev, "d"), _ptr(tnear, f, (R,), dev, "tnear"),
        _ptr(tfar, f, (R,), dev, "tfar"), R, int(n_samples), float(beta), float(eps), int(channel), float(level),
        float(lower), _ptr(hit, torch.int32, (R,), dev, "hit_index"), _ptr(hv, f, (R, 2), dev, "hit_values"),
        _ptr(ev, torch.int32, (R,), dev, "evals"), _stream(dev)), "dps_ray_march_harnack")
    return hit, hv, ev


def dps_ray_resample(o, d, tnear, tfar, n_march: int, hit_index, hit_values, jitter, level: float = 0.5,
                     counts=(24, 48, 8), window: float = 8.0, tile_layout: bool = False, t_out=None, x_out=None):
    """Quadrature samples around each ray's first crossing (``dps_ray_resample``).
    jitter [R, S] in [0, 1), S = sum(counts).  Returns (t[R, S], x[R * S, 3])."""
    import torch
    R = o.shape[0]
    nb, nd, na = (int(c) for c in counts)
    S = nb + nd + na
    dev = o.device
    t = t_out if t_out is not None else torch.empty((R, S), device=dev, dtype=torch.float32)
    x = x_out if x_out is not None else torch.empty((R * S, 3), device=dev, dtype=torch.float32)
    f = torch.float32
    with torch.cuda.device(dev):
        _check(load().dps_ray_resample(_ptr(o, f, (R, 3), dev, "o"), _ptr(d, f, (R, 3), dev, "d"),
                                       _ptr(tnear, f, (R,), dev, "tnear"), _ptr(tfar, f, (R,), dev, "tfar"), R,
                                       int(n_march), _ptr(hit_index, torch.int32, (R,), dev, "hit_index"),
                                       _ptr(hit_values, f, (R, 2), dev, "hit_values"), float(level),
                                       _ptr(jitter, f, (R, S), dev, "jitter"), nb, nd, na, float(window),
                                       int(bool(tile_layout)), _ptr(t, f, (R, S), dev, "t_out"),
                                       _ptr(x, f, (R * S, 3), dev, "x_out"), _stream(dev)), "dps_ray_resample")
    return t, x


def dps_check(tree: Tree):
    """Synchronises and raises if a device-side failure was recorded."""
    _check(load().dps_check(tree.handle, _stream(tree.device)), "dps_check")


def dps_set_step_limit(tree: Tree, limit: int):
    """Caps the nodes one traversal may walk (0: the node count, the default).
    A diagnostic: a traversal reaching the cap stops and dps_check raises."""
    _check(load().dps_set_step_limit(tree.handle, int(limit)), "dps_set_step_limit")


def dps_set_memory_limit(nbytes: int):
    """Process-wide cap on the device bytes one build may hold (0: none)."""
    _check(load().dps_set_memory_limit(int(nbytes)), "dps_set_memory_limit")


def dps_destroy(tree: Tree):
    if tree._h is not None:
        load().dps_destroy(tree._h)
        tree._h = None


def dps_status_string(status: int) -> str:
    return load().dps_status_string(int(status)).decode()


def dps_last_error() -> str:
    return load().dps_last_error().decode(errors="replace")
