"""FP64 CPU oracle for demons registration: ctypes binding of demons_oracle.c.

TEST INFRASTRUCTURE ONLY.  Imported by the tests, by the package smoke check
and by the benchmark's CPU-baseline leg; the product path never imports it.
The C source shares no code with the HIP library.

Arrays are numpy float64, C-contiguous: volumes [nz, ny, nx] (x fastest),
fields [3, nz, ny, nx] with components (x, y, z) in voxel units.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "demons_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

PASSIVE, EVOLVED, ACTIVE, DOUBLE, INVERSE_CONSISTENT = 0, 1, 2, 3, 4
VARIANTS = {"passive": PASSIVE, "evolved": EVOLVED, "active": ACTIVE, "double": DOUBLE,
            "inverse_consistent": INVERSE_CONSISTENT}
OK, EINVAL, ENOMEM, ENUMERIC = 0, -1, -2, -4
DEFAULT_COMPOSE_ITERS = 10


class OracleError(RuntimeError):
    pass


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (-O2, OpenMP) next to the source."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", "-std=c11", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC, "-lm"],
                       check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        i64 = ctypes.c_int64
        L.orc_max_threads.restype = ctypes.c_int
        L.orc_set_threads.argtypes = [ctypes.c_int]
        L.orc_trilerp.restype = ctypes.c_double
        L.orc_trilerp.argtypes = [dp, i64, i64, i64, ctypes.c_double, ctypes.c_double, ctypes.c_double]
        L.orc_warp.argtypes = [dp, dp, i64, i64, i64, ctypes.c_double, dp]
        L.orc_gradient.argtypes = [dp, i64, i64, i64, dp]
        L.orc_gauss_weights.argtypes = [ctypes.c_double, ctypes.c_int, dp]
        L.orc_smooth.argtypes = [dp, ctypes.c_int, i64, i64, i64, ctypes.c_double, ctypes.c_int, dp]
        L.orc_restrict.argtypes = [dp, i64, i64, i64, dp]
        L.orc_prolong.argtypes = [dp, i64, i64, i64, dp, i64, i64, i64]
        L.orc_force.argtypes = [ctypes.c_int, ctypes.c_double, dp, dp, dp, i64, i64, i64, dp, dp]
        L.orc_iterate.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int, dp, dp, i64, i64,
                                  i64, dp, ctypes.c_int, ctypes.c_double, dp]
        L.orc_compose.argtypes = [dp, i64, i64, i64, ctypes.c_int, dp]
        L.orc_register.argtypes = [dp, dp, i64, i64, i64, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                   ctypes.c_int, ctypes.c_int, ip, ctypes.c_double, ctypes.c_int, dp, dp, ip]
        L.orc_register_ex.argtypes = [dp, dp, i64, i64, i64, dp, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                      ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_int, ip,
                                      ctypes.c_double, ctypes.c_int, dp, dp, ip]
        L.orc_smooth3.argtypes = [dp, ctypes.c_int, i64, i64, i64, dp, ip, dp]
        L.orc_iterate_mm.argtypes = [ctypes.c_int, ctypes.c_double, dp, ip, dp, dp, i64, i64, i64, dp, dp,
                                     ctypes.c_int, ctypes.c_double, dp]
        _lib = L
    return _lib


def max_threads() -> int:
    """OpenMP threads the oracle's element-wise loops use."""
    return int(lib().orc_max_threads())


def set_threads(n: int) -> None:
    """Run the oracle's element-wise loops on n threads from now on (its sums
    are serial, so results do not depend on it)."""
    lib().orc_set_threads(int(n))


def _p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _vol(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.ndim != 3:
        raise ValueError("volume must be [nz, ny, nx]")
    return a


def _field(a, shape3):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.shape != (3,) + tuple(shape3):
        raise ValueError(f"field must be [3, nz, ny, nx], got {a.shape}")
    return a


def _dims(a):
    nz, ny, nx = a.shape[-3:]
    return nx, ny, nz


def default_radius(sigma: float) -> int:
    return int(np.ceil(3.0 * sigma))


def trilerp(I, px, py, pz):
    I = _vol(I)
    return lib().orc_trilerp(_p(I), *_dims(I), float(px), float(py), float(pz))


def warp(I, v, sign=1.0):
    I = _vol(I)
    v = _field(v, I.shape)
    out = np.empty_like(I)
    lib().orc_warp(_p(I), _p(v), *_dims(I), float(sign), _p(out))
    return out


def gradient(I):
    I = _vol(I)
    out = np.empty((3,) + I.shape)
    lib().orc_gradient(_p(I), *_dims(I), _p(out))
    return out


def gauss_weights(sigma, radius):
    w = np.empty(2 * radius + 1)
    lib().orc_gauss_weights(float(sigma), int(radius), _p(w))
    return w


def smooth(a, sigma, radius=None):
    """Gaussian smoothing of a volume [nz,ny,nx] or of a stack [c,nz,ny,nx]."""
    radius = default_radius(sigma) if radius is None else int(radius)
    a = np.ascontiguousarray(a, dtype=np.float64)
    stack = a if a.ndim == 4 else a[None]
    out = np.empty_like(stack)
    rc = lib().orc_smooth(_p(stack), stack.shape[0], *_dims(stack), float(sigma), radius, _p(out))
    if rc != OK:
        raise OracleError(rc)
    return out if a.ndim == 4 else out[0]


def smooth3(a, sigma3, radius3):
    """Per-axis Gaussian smoothing (sigma and radius per axis x, y, z) of a
    volume or a stack."""
    a = np.ascontiguousarray(a, dtype=np.float64)
    stack = a if a.ndim == 4 else a[None]
    out = np.empty_like(stack)
    sg = np.ascontiguousarray(sigma3, dtype=np.float64)
    rd = (ctypes.c_int * 3)(*[int(r) for r in radius3])
    rc = lib().orc_smooth3(_p(stack), stack.shape[0], *_dims(stack), _p(sg), rd, _p(out))
    if rc != OK:
        raise OracleError(rc)
    return out if a.ndim == 4 else out[0]


def iterate_mm(variant, S, M, v_mm, iters, sigma3, radius3, h_mm, alpha=1.0, eps=0.0):
    """iterate() in physical units: field in mm, voxel size h_mm, per-axis
    Gaussian widths sigma3 (voxels) and radii radius3."""
    S = _vol(S)
    M = _vol(M)
    v = np.array(_field(v_mm, S.shape), copy=True)
    hist = np.zeros((max(iters, 1), 4))
    sg = np.ascontiguousarray(sigma3, dtype=np.float64)
    hh = np.ascontiguousarray(h_mm, dtype=np.float64)
    rd = (ctypes.c_int * 3)(*[int(r) for r in radius3])
    n = lib().orc_iterate_mm(int(variant), float(alpha), _p(sg), rd, _p(S), _p(M), *_dims(S), _p(hh), _p(v),
                             int(iters), float(eps), _p(hist))
    if n < 0:
        raise OracleError(n)
    return v, hist[:n]


def coarse_shape(shape3):
    """[nz, ny, nx] -> ceil(n / 2) per dimension."""
    return tuple((n + 1) // 2 for n in shape3)


def restrict(I):
    I = _vol(I)
    out = np.empty(coarse_shape(I.shape))
    lib().orc_restrict(_p(I), *_dims(I), _p(out))
    return out


def prolong(vc, fine_shape3):
    vc = np.ascontiguousarray(vc, dtype=np.float64)
    out = np.empty((3,) + tuple(fine_shape3))
    nz, ny, nx = fine_shape3
    lib().orc_prolong(_p(vc), *_dims(vc), _p(out), nx, ny, nz)
    return out


def force(variant, S, M, v, alpha=1.0):
    """u = v + dr (Eqs 1-6) and (sum|dr|, sum|v|, sum D^2)."""
    S = _vol(S)
    M = _vol(M)
    v = _field(v, S.shape)
    u = np.empty_like(v)
    sums = np.empty(3)
    rc = lib().orc_force(int(variant), float(alpha), _p(S), _p(M), _p(v), *_dims(S), _p(u), _p(sums))
    if rc != OK:
        raise OracleError(rc)
    return u, sums


def iterate(variant, S, M, v, iters, sigma, radius=None, alpha=1.0, eps=0.0):
    """Run `iters` iterations at one level; returns (field, history[n,4])."""
    radius = default_radius(sigma) if radius is None else int(radius)
    S = _vol(S)
    M = _vol(M)
    v = np.array(_field(v, S.shape), copy=True)
    hist = np.zeros((max(iters, 1), 4))
    n = lib().orc_iterate(int(variant), float(alpha), float(sigma), radius, _p(S), _p(M), *_dims(S), _p(v),
                          int(iters), float(eps), _p(hist))
    if n < 0:
        raise OracleError(n)
    return v, hist[:n]


def compose(h, K=DEFAULT_COMPOSE_ITERS):
    h = np.ascontiguousarray(h, dtype=np.float64)
    out = np.empty_like(h)
    lib().orc_compose(_p(h), *_dims(h), int(K), _p(out))
    return out


def register(S, M, variant, iters, sigma, radius=None, alpha=1.0, eps=0.0, compose_iters=DEFAULT_COMPOSE_ITERS,
             raise_on_error=True, spacing=None, physical=False, image_sigma=0.0):
    """Multi-scale registration.  iters lists levels coarse -> fine.

    spacing: None or the voxel sizes (x, y, z) in mm; physical=True works in
    mm (sigma and image_sigma in mm); image_sigma > 0 pre-smooths every
    level's images.  radius None (or <= 0) selects ceil(3 sigma) per axis.

    Returns (field [3,nz,ny,nx] in voxels, history [sum(iters_run), 4],
    iters_run list, rc).
    """
    radius = 0 if radius is None else int(radius)
    S = _vol(S)
    M = _vol(M)
    if S.shape != M.shape:
        raise ValueError("S and M differ in shape")
    iters = [int(i) for i in iters]
    levels = len(iters)
    it = (ctypes.c_int * max(levels, 1))(*iters)
    run = (ctypes.c_int * max(levels, 1))()
    field = np.zeros((3,) + S.shape)
    hist = np.zeros((max(sum(iters), 1), 4))
    sp = np.ascontiguousarray(spacing, dtype=np.float64) if spacing is not None else None
    rc = lib().orc_register_ex(_p(S), _p(M), *_dims(S), _p(sp) if sp is not None else None, int(bool(physical)),
                               float(image_sigma), int(variant), float(alpha), float(sigma), radius, levels, it,
                               float(eps), int(compose_iters), _p(field), _p(hist), run)
    if rc != OK and raise_on_error:
        raise OracleError(rc)
    runs = list(run)[:levels]
    return field, hist[:sum(runs)], runs, rc
