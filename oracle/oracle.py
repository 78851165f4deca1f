"""ctypes wrapper of the FP64 reference (test infrastructure only).

Inputs are the FP32 arrays both sides read; outputs are float64 NumPy arrays.
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dps_oracle.c")
# DPS_ORACLE_SANITIZE=1 selects a separate build with AddressSanitizer and
# UndefinedBehaviorSanitizer (the process must preload the ASan runtime)
_SANITIZE = os.environ.get("DPS_ORACLE_SANITIZE") == "1"
_LIB = os.path.join(_HERE, "libdps_oracle_san.so" if _SANITIZE else "libdps_oracle.so")
_lib = None

_f32p = np.ctypeslib.ndpointer(np.float32, flags="C_CONTIGUOUS")
_f64p = ct.POINTER(ct.c_double)


def build(force: bool = True) -> str:
    """Compile the reference with gcc (FP64, no floating-point contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        opt = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
               "-fno-omit-frame-pointer"] if _SANITIZE else ["-O2"]
        cmd = ["gcc", *opt, "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build(force=True)
    lib = ct.CDLL(_LIB)
    vp = ct.c_void_p
    lib.orc_rho.restype = ct.c_double
    lib.orc_rho.argtypes = [ct.c_double]
    lib.orc_psi.restype = ct.c_double
    lib.orc_psi.argtypes = [ct.c_double]
    for nm in ("orc_rho_series", "orc_psi_series", "orc_rho_closed", "orc_chi", "orc_chi_series"):
        getattr(lib, nm).restype = ct.c_double
        getattr(lib, nm).argtypes = [ct.c_double]
    lib.orc_radial_nu.restype = ct.c_double
    lib.orc_radial_nu.argtypes = [ct.c_double, ct.c_double]
    lib.orc_radial_eps.restype = None
    lib.orc_radial_eps.argtypes = [ct.c_double, ct.c_double, _f64p, _f64p]
    lib.orc_radial.restype = None
    lib.orc_radial.argtypes = [ct.c_double, ct.c_double, _f64p, _f64p]
    lib.orc_direct.restype = ct.c_int
    lib.orc_direct.argtypes = [vp, vp, vp, vp, ct.c_int64, ct.c_int, vp, ct.c_int64, ct.c_double,
                               vp, vp, vp, vp, ct.c_int]
    lib.orc_direct_adjoint.restype = ct.c_int
    lib.orc_direct_adjoint.argtypes = [vp, vp, vp, vp, ct.c_int64, ct.c_int, vp, ct.c_int64,
                                       ct.c_double, vp, vp, vp, vp, vp, vp, ct.c_int]
    lib.orc_tree_build.restype = vp
    lib.orc_tree_build.argtypes = [vp, vp, vp, ct.c_int64, ct.c_int]
    lib.orc_tree_free.restype = None
    lib.orc_tree_free.argtypes = [vp]
    lib.orc_tree_set_attrs.restype = ct.c_int
    lib.orc_tree_set_attrs.argtypes = [vp, vp, ct.c_int]
    lib.orc_tree_set_kind.restype = ct.c_int
    lib.orc_tree_set_kind.argtypes = [vp, ct.c_int]
    lib.orc_direct_mono.restype = ct.c_int
    lib.orc_direct_mono.argtypes = [vp, vp, vp, ct.c_int64, ct.c_int, vp, ct.c_int64, ct.c_double,
                                    vp, vp, vp, vp, ct.c_int]
    lib.orc_direct_mono_adjoint.restype = ct.c_int
    lib.orc_direct_mono_adjoint.argtypes = [vp, vp, vp, ct.c_int64, ct.c_int, vp, ct.c_int64, ct.c_double,
                                            vp, vp, vp, ct.c_int]
    lib.orc_round_bf16.restype = ct.c_double
    lib.orc_round_bf16.argtypes = [ct.c_float]
    lib.orc_tree_set_storage.restype = ct.c_int
    lib.orc_tree_set_storage.argtypes = [vp, ct.c_int, ct.c_int]
    lib.orc_tree_set_scale.restype = ct.c_int
    lib.orc_tree_set_scale.argtypes = [vp, ct.c_int]
    lib.orc_tree_export_stored.restype = ct.c_int
    lib.orc_tree_export_stored.argtypes = [vp, vp, vp]
    lib.orc_tree_num_nodes.restype = ct.c_int64
    lib.orc_tree_num_nodes.argtypes = [vp]
    lib.orc_tree_depth.restype = ct.c_int
    lib.orc_tree_depth.argtypes = [vp]
    lib.orc_tree_export.restype = ct.c_int
    lib.orc_tree_export.argtypes = [vp] * 10
    lib.orc_bh_query.restype = ct.c_int
    lib.orc_bh_query.argtypes = [vp, vp, ct.c_int64, ct.c_float, ct.c_double, vp, vp, vp, vp, vp,
                                 ct.c_int]
    lib.orc_bh_adjoint.restype = ct.c_int
    lib.orc_bh_adjoint.argtypes = [vp, vp, ct.c_int64, ct.c_float, ct.c_double, vp, vp, vp, vp,
                                   vp, vp, vp, vp, vp, vp, ct.c_int]
    _lib = lib
    return lib


def _c32(a, shape_last=None):
    a = np.ascontiguousarray(a, dtype=np.float32)
    if shape_last is not None and (a.ndim != 2 or a.shape[1] != shape_last):
        raise ValueError(f"expected [n,{shape_last}] array, got {a.shape}")
    return a


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ct.c_void_p)


def rho(t): return load().orc_rho(float(t))
def psi(t): return load().orc_psi(float(t))
def rho_series(t): return load().orc_rho_series(float(t))
def psi_series(t): return load().orc_psi_series(float(t))
def rho_closed(t): return load().orc_rho_closed(float(t))
def chi(t): return load().orc_chi(float(t))
def chi_series(t): return load().orc_chi_series(float(t))


def radial_nu(r, eps):
    """nu = chi(r/eps)/(4 pi r^7), the Hessian's radial factor."""
    return load().orc_radial_nu(float(r), float(eps))


def radial_eps(r, eps):
    """(d kappa / d eps, d lambda / d eps)."""
    k, l = ct.c_double(), ct.c_double()
    load().orc_radial_eps(float(r), float(eps), ct.byref(k), ct.byref(l))
    return k.value, l.value


def radial(r, eps):
    """(kappa, lambda) = (rho(r/eps)/(4 pi r^3), psi(r/eps)/(4 pi r^5))."""
    k, l = ct.c_double(), ct.c_double()
    load().orc_radial(float(r), float(eps), ct.byref(k), ct.byref(l))
    return k.value, l.value


def round_bf16(v):
    """Nearest bfloat16 value (ties to even) of an FP32 value, as a float."""
    return load().orc_round_bf16(float(np.float32(v)))


STORAGE_MODES = {"exact": 0, "bf16": 1, "fp32": 2}


def direct(p, n, A, mu, x, eps, want_grad=True, nthreads=0):
    """FP64 direct sum.  Returns dict f[Q,C], g[Q,C,3], sf[Q,C], sg[Q,C]."""
    lib = load()
    p, n, x = _c32(p, 3), _c32(n, 3), _c32(x, 3)
    A = _c32(A).reshape(-1)
    mu = _c32(mu)
    if mu.ndim == 1:
        mu = mu[:, None]
    M, C, Q = p.shape[0], mu.shape[1], x.shape[0]
    f = np.zeros((Q, C)); sf = np.zeros((Q, C)); sg = np.zeros((Q, C))
    g = np.zeros((Q, C, 3)) if want_grad else None
    rc = lib.orc_direct(_ptr(p), _ptr(n), _ptr(A), _ptr(mu), M, C, _ptr(x), Q, float(eps),
                        _ptr(f), _ptr(g), _ptr(sf), _ptr(sg), int(nthreads))
    if rc:
        raise ValueError("orc_direct rejected its arguments")
    return {"f": f, "g": g, "sf": sf, "sg": sg}


def direct_adjoint(p, n, A, mu, x, eps, df, nthreads=0, dg=None, extra=False):
    """Exact transpose of ``direct`` (values and, with dg[Q,C,3], gradients):
    returns (dmu[M,C], dx[Q,3]), or with extra=True (dmu, dx, dn[M,3], deps)
    including the derivatives in the normals and in eps.  df may be None when
    dg is given."""
    lib = load()
    p, n, x = _c32(p, 3), _c32(n, 3), _c32(x, 3)
    A = _c32(A).reshape(-1)
    mu = _c32(mu)
    if mu.ndim == 1:
        mu = mu[:, None]
    M, C, Q = p.shape[0], mu.shape[1], x.shape[0]
    df = None if df is None else _c32(df).reshape(Q, C)
    dg = None if dg is None else _c32(dg).reshape(Q, C, 3)
    dmu = np.zeros((M, C)); dx = np.zeros((Q, 3))
    dn = np.zeros((M, 3)) if extra else None
    deps = np.zeros(1) if extra else None
    rc = lib.orc_direct_adjoint(_ptr(p), _ptr(n), _ptr(A), _ptr(mu), M, C, _ptr(x), Q, float(eps),
                                _ptr(df), _ptr(dg), _ptr(dmu), _ptr(dx), _ptr(dn), _ptr(deps), int(nthreads))
    if rc:
        raise ValueError("orc_direct_adjoint rejected its arguments")
    return (dmu, dx, dn, float(deps[0])) if extra else (dmu, dx)


def direct_mono(p, A, mu, x, eps, want_grad=True, nthreads=0):
    """FP64 direct sum of the monopole kernel rho(r/eps)/(4 pi r^2) (appearance
    channels, foreshortening skipped).  Returns dict f, g, sf, sg."""
    lib = load()
    p, x = _c32(p, 3), _c32(x, 3)
    A = _c32(A).reshape(-1)
    mu = _c32(mu)
    if mu.ndim == 1:
        mu = mu[:, None]
    M, C, Q = p.shape[0], mu.shape[1], x.shape[0]
    f = np.zeros((Q, C)); sf = np.zeros((Q, C)); sg = np.zeros((Q, C))
    g = np.zeros((Q, C, 3)) if want_grad else None
    rc = lib.orc_direct_mono(_ptr(p), _ptr(A), _ptr(mu), M, C, _ptr(x), Q, float(eps), _ptr(f), _ptr(g),
                             _ptr(sf), _ptr(sg), int(nthreads))
    if rc:
        raise ValueError("orc_direct_mono rejected its arguments")
    return {"f": f, "g": g, "sf": sf, "sg": sg}


def direct_mono_adjoint(p, A, mu, x, eps, df, nthreads=0):
    """Exact transpose of ``direct_mono``: returns (dmu[M,C], dx[Q,3])."""
    lib = load()
    p, x = _c32(p, 3), _c32(x, 3)
    A = _c32(A).reshape(-1)
    mu = _c32(mu)
    if mu.ndim == 1:
        mu = mu[:, None]
    M, C, Q = p.shape[0], mu.shape[1], x.shape[0]
    df = _c32(df).reshape(Q, C)
    dmu = np.zeros((M, C)); dx = np.zeros((Q, 3))
    rc = lib.orc_direct_mono_adjoint(_ptr(p), _ptr(A), _ptr(mu), M, C, _ptr(x), Q, float(eps), _ptr(df),
                                     _ptr(dmu), _ptr(dx), int(nthreads))
    if rc:
        raise ValueError("orc_direct_mono_adjoint rejected its arguments")
    return dmu, dx


class Tree:
    """Canonical octree + FP64 node dipoles + Barnes-Hut queries."""

    def __init__(self, p, n, A, mu=None, leaf_size=16, kind="dipole"):
        """kind: "dipole" (eq. dipole_sum) or "monopole" (appearance channels
        with the foreshortening term skipped: scalar moments sum A mu)."""
        lib = load()
        self._p = _c32(p, 3)
        self._n = _c32(n, 3)
        self._A = _c32(A).reshape(-1)
        self.M = self._p.shape[0]
        h = lib.orc_tree_build(_ptr(self._p), _ptr(self._n), _ptr(self._A), self.M, int(leaf_size))
        if not h:
            raise ValueError("orc_tree_build rejected its arguments")
        self._h = ct.c_void_p(h)
        self.N = int(lib.orc_tree_num_nodes(self._h))
        self.depth = int(lib.orc_tree_depth(self._h))
        self.C = 0
        if kind not in ("dipole", "monopole"):
            raise ValueError(kind)
        self.kind = kind
        if kind == "monopole":
            lib.orc_tree_set_kind(self._h, 1)
        if mu is not None:
            self.set_attrs(mu)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.orc_tree_free(h)
            self._h = None

    def set_attrs(self, mu):
        mu = _c32(mu)
        if mu.ndim == 1:
            mu = mu[:, None]
        if mu.shape[0] != self.M:
            raise ValueError("attribute rows must match the point count")
        self.C = mu.shape[1]
        if load().orc_tree_set_attrs(self._h, _ptr(mu), self.C):
            raise ValueError("orc_tree_set_attrs rejected its arguments")

    def set_storage(self, mode="exact", fp32_levels=-1):
        """Evaluate from values rounded as a store holds them: "exact" (FP64
        moments, the default), "fp32" (moments rounded once to FP32) or
        "bf16" (attributes and moments rounded to bfloat16, moments through
        FP32; nodes of level <= fp32_levels keep the FP32 rounding).  Applies
        to later queries and adjoints, and survives set_attrs."""
        if load().orc_tree_set_storage(self._h, STORAGE_MODES[mode], int(fp32_levels)):
            raise ValueError("orc_tree_set_storage rejected its arguments")

    def set_scale(self, mode="mass"):
        """Error scale of a node's far-field term in sf, sg, sdx and friends:
        "mass" (the sum of its points' absolute dipoles, the default) or
        "moment" (the magnitude of its own moment |D_t|, stricter where the
        moment cancels)."""
        if load().orc_tree_set_scale(self._h, {"mass": 0, "moment": 1}[mode]):
            raise ValueError("orc_tree_set_scale rejected its arguments")

    def export_stored(self):
        """(moments [N,C,3], sorted attributes [M,C]) as the sums read them."""
        Ds = np.zeros((self.N, self.C, 3))
        mus = np.zeros((self.M, self.C))
        if load().orc_tree_export_stored(self._h, _ptr(Ds), _ptr(mus)):
            raise ValueError("no attributes set")
        return Ds, mus

    def export(self):
        M, N, C = self.M, self.N, self.C
        out = {
            "codes_in": np.zeros(M, np.uint64), "codes": np.zeros(M, np.uint64),
            "perm": np.zeros(M, np.uint32), "nodes": np.zeros((N, 6), np.int32),
            "geom": np.zeros((N, 4), np.float32), "area": np.zeros(N),
            "D": np.zeros((N, C, 3)) if C else None, "bounds": np.zeros(5),
            "leaf_of": np.zeros(M, np.int32),
        }
        load().orc_tree_export(self._h, *[_ptr(out[k]) for k in
                                          ("codes_in", "codes", "perm", "nodes", "geom", "area",
                                           "D", "bounds", "leaf_of")])
        return out

    def query(self, x, beta, eps, want_grad=True, nthreads=0):
        """Barnes-Hut forward.  Returns dict f, g, sf, sg, counts[Q,4]
        (visited nodes, far-field nodes, leaves opened, near points)."""
        x = _c32(x, 3)
        Q, C = x.shape[0], self.C
        f = np.zeros((Q, C)); sf = np.zeros((Q, C)); sg = np.zeros((Q, C))
        g = np.zeros((Q, C, 3)) if want_grad else None
        counts = np.zeros((Q, 4), np.int32)
        rc = load().orc_bh_query(self._h, _ptr(x), Q, float(beta), float(eps), _ptr(f), _ptr(g),
                                 _ptr(sf), _ptr(sg), _ptr(counts), int(nthreads))
        if rc:
            raise ValueError("orc_bh_query rejected its arguments")
        return {"f": f, "g": g, "sf": sf, "sg": sg, "counts": counts}

    def adjoint(self, x, beta, eps, df, nthreads=0, dg=None, extra=False):
        """Barnes-Hut adjoint for value cotangents df[Q,C] and/or gradient
        cotangents dg[Q,C,3] (df may be None when dg is given).  Returns dict
        dmu[M,C] (caller order), dx[Q,3], sdmu[M,C], sdx[Q] (absolute scales
        for error normalisation); with extra=True also dn[M,3] (normals,
        caller order), sdn[M], deps and sdeps (the global eps)."""
        x = _c32(x, 3)
        Q, C, M = x.shape[0], self.C, self.M
        df = None if df is None else _c32(df).reshape(Q, C)
        dg = None if dg is None else _c32(dg).reshape(Q, C, 3)
        dmu = np.zeros((M, C)); dx = np.zeros((Q, 3))
        sdmu = np.zeros((M, C)); sdx = np.zeros(Q)
        dn = np.zeros((M, 3)) if extra else None
        sdn = np.zeros(M) if extra else None
        deps = np.zeros(1) if extra else None
        sdeps = np.zeros(1) if extra else None
        rc = load().orc_bh_adjoint(self._h, _ptr(x), Q, float(beta), float(eps), _ptr(df), _ptr(dg),
                                   _ptr(dmu), _ptr(dx), _ptr(dn), _ptr(deps), _ptr(sdmu), _ptr(sdx), _ptr(sdn),
                                   _ptr(sdeps), int(nthreads))
        if rc:
            raise ValueError("orc_bh_adjoint rejected its arguments")
        out = {"dmu": dmu, "dx": dx, "sdmu": sdmu, "sdx": sdx}
        if extra:
            out.update(dn=dn, sdn=sdn, deps=float(deps[0]), sdeps=float(sdeps[0]))
        return out
