"""ctypes binding of libdemons.so (include/demons.h), same names as the C ABI.

Argument marshalling only: every step of the registration runs in the HIP
kernels of libdemons.so.  Tensors are torch CUDA (HIP) float32 tensors,
contiguous, on the handle's device: volumes [nz, ny, nx], fields
[3, nz, ny, nx] in voxel units.  If the shared library is missing this module
raises; there is no other code path.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdemons.so")

DIR_OK, DIR_EINVAL, DIR_ENOMEM, DIR_EDEVICE, DIR_ENUMERIC, DIR_EBUSY = 0, -1, -2, -3, -4, -5
DIR_NOALLOC_SCRATCH_BYTES = 128 * 1024 * 1024   # include/demons.h
DIR_PASSIVE, DIR_EVOLVED_PASSIVE, DIR_ACTIVE, DIR_DOUBLE, DIR_INVERSE_CONSISTENT = 0, 1, 2, 3, 4
DIR_MAX_LEVELS = 8
DIR_MAX_RADIUS = 16
DIR_MAX_BATCH = 8
DIR_STORE_F32, DIR_STORE_F16, DIR_STORE_BF16 = 0, 1, 2
DIR_UNITS_VOXELS, DIR_UNITS_MM = 0, 1
UNITS = {"voxels": DIR_UNITS_VOXELS, "mm": DIR_UNITS_MM}
STORAGE = {"f32": DIR_STORE_F32, "f16": DIR_STORE_F16, "bf16": DIR_STORE_BF16}
VARIANTS = {"passive": DIR_PASSIVE, "evolved": DIR_EVOLVED_PASSIVE, "active": DIR_ACTIVE, "double": DIR_DOUBLE,
            "inverse_consistent": DIR_INVERSE_CONSISTENT}


class DemonsError(RuntimeError):
    def __init__(self, code, where=""):
        self.code = int(code)
        msg = f"{where}: {_strerror(self.code)} ({self.code})"
        detail = _last_error()
        if detail:
            msg += f" [{detail}]"
        super().__init__(msg)


class dir_params(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_int32), ("variant", ctypes.c_int32), ("alpha", ctypes.c_double),
                ("sigma", ctypes.c_double), ("radius", ctypes.c_int32), ("levels", ctypes.c_int32),
                ("iters", ctypes.c_int32 * DIR_MAX_LEVELS), ("eps", ctypes.c_double),
                ("compose_iters", ctypes.c_int32), ("storage", ctypes.c_int32), ("units", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("image_sigma", ctypes.c_double)]


class dir_stats(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_int32), ("levels", ctypes.c_int32),
                ("iters_run", ctypes.c_int32 * DIR_MAX_LEVELS), ("mse_final", ctypes.c_double),
                ("relnorm_final", ctypes.c_double), ("history", ctypes.POINTER(ctypes.c_double)),
                ("history_capacity", ctypes.c_int32), ("history_len", ctypes.c_int32)]


_lib = None


def lib():
    """Load libdemons.so; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise DemonsError(DIR_EDEVICE, f"{LIB_PATH} missing; build it with python -m paper_0909_0928_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
        L.dir_abi_version.restype = i32
        L.dir_strerror.restype = ctypes.c_char_p
        L.dir_strerror.argtypes = [i32]
        L.dir_last_error_message.restype = ctypes.c_char_p
        L.dir_create.argtypes = [ctypes.POINTER(vp), i32, vp]
        L.dir_set_stream.argtypes = [vp, vp]
        L.dir_destroy.argtypes = [vp]
        L.dir_synchronize.argtypes = [vp]
        L.dir_register.argtypes = [vp, vp, vp, i32, i32, i32, ctypes.POINTER(f64), ctypes.POINTER(dir_params), vp,
                                   ctypes.POINTER(dir_stats)]
        L.dir_warp.argtypes = [vp, vp, vp, i32, i32, i32, vp]
        L.dir_gradient.argtypes = [vp, vp, i32, i32, i32, vp]
        L.dir_smooth.argtypes = [vp, vp, i32, i32, i32, i32, f64, i32, vp]
        L.dir_restrict.argtypes = [vp, vp, i32, i32, i32, vp]
        L.dir_prolong.argtypes = [vp, vp, i32, i32, i32, vp, i32, i32, i32]
        L.dir_force.argtypes = [vp, i32, f64, vp, vp, vp, i32, i32, i32, vp, ctypes.POINTER(f64)]
        L.dir_step.argtypes = [vp, i32, f64, vp, vp, vp, i32, i32, i32, f64, i32, vp, ctypes.POINTER(f64)]
        L.dir_step_stored.argtypes = [vp, i32, i32, f64, vp, vp, vp, i32, i32, i32, f64, i32, vp, ctypes.POINTER(f64)]
        L.dir_step_noalloc.argtypes = [vp, i32, f64, vp, vp, vp, i32, i32, i32, f64, i32, vp, ctypes.POINTER(f64)]
        L.dir_register_async.argtypes = [vp, vp, vp, i32, i32, i32, vp, vp, vp]
        L.dir_register_batch.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, vp]
        L.dir_register_batch_async.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp]
        L.dir_pool_set_max_batch.argtypes = [vp, i32]
        L.dir_autotune.argtypes = [vp, i32, i32, i32, vp, i32, vp]
        L.dir_autotune_clear.argtypes = []
        L.dir_autotune_clear.restype = None
        L.dir_wait.argtypes = [vp, vp]
        L.dir_set_graphs.argtypes = [vp, i32]
        L.dir_similarity.argtypes = [vp, vp, vp, vp, i32, i32, i32, ctypes.POINTER(f64), ctypes.POINTER(f64)]
        u64, i64 = ctypes.c_uint64, ctypes.c_int64
        L.dir_workspace_bytes.argtypes = [i32, i32, i32, vp, ctypes.POINTER(u64)]
        L.dir_pool_create.argtypes = [ctypes.POINTER(vp), i32, i32, u64]
        L.dir_pool_destroy.argtypes = [vp]
        L.dir_pool_submit.argtypes = [vp, vp, vp, i32, i32, i32, vp, vp, vp, ctypes.POINTER(i64)]
        L.dir_pool_progress.argtypes = [vp]
        L.dir_pool_poll.argtypes = [vp, i64, vp, ctypes.POINTER(i32)]
        L.dir_pool_wait.argtypes = [vp, i64, vp]
        L.dir_pool_stats.argtypes = [vp, ctypes.POINTER(u64), ctypes.POINTER(u64), ctypes.POINTER(i32),
                                     ctypes.POINTER(i32)]
        L.dir_compose.argtypes = [vp, vp, i32, i32, i32, i32, vp]
        L.dir_timing_count.restype = i32
        L.dir_timing_name.restype = ctypes.c_char_p
        L.dir_timing_name.argtypes = [i32]
        L.dir_timing_enable.argtypes = [vp, ctypes.c_uint64]
        L.dir_timing_read.argtypes = [vp, i32, ctypes.POINTER(f64), ctypes.POINTER(ctypes.c_int64)]
        L.dir_timing_read_level.argtypes = [vp, i32, i32, ctypes.POINTER(f64), ctypes.POINTER(ctypes.c_int64)]
        for name in ("dir_create", "dir_set_stream", "dir_destroy", "dir_synchronize", "dir_register", "dir_warp",
                     "dir_gradient", "dir_smooth", "dir_restrict", "dir_prolong", "dir_force", "dir_step", "dir_compose",
                     "dir_register_async", "dir_register_batch", "dir_register_batch_async", "dir_wait",
                     "dir_pool_set_max_batch", "dir_autotune", "dir_set_graphs", "dir_step_stored", "dir_similarity",
                     "dir_step_noalloc",
                     "dir_workspace_bytes", "dir_pool_create", "dir_pool_destroy", "dir_pool_submit",
                     "dir_pool_progress", "dir_pool_poll", "dir_pool_wait", "dir_pool_stats",
                     "dir_timing_enable", "dir_timing_read", "dir_timing_read_level"):
            getattr(L, name).restype = i32
        _lib = L
    return _lib


def _strerror(code):
    try:
        return lib().dir_strerror(int(code)).decode()
    except Exception:
        return "error"


def _last_error():
    try:
        return lib().dir_last_error_message().decode()
    except Exception:
        return ""


def _check(rc, where):
    if rc != DIR_OK:
        raise DemonsError(rc, where)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _dev_f32(t, name, ndim):
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float32 or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous float32 tensor on the GPU")
    if t.dim() != ndim:
        raise ValueError(f"{name} must have {ndim} dimensions, got {tuple(t.shape)}")
    return t


def _dims(vol):
    nz, ny, nx = vol.shape[-3:]
    return int(nx), int(ny), int(nz)


def _stream_ptr(stream, device):
    if stream is None:
        stream = torch.cuda.current_stream(device)
    if isinstance(stream, torch.cuda.Stream):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(int(stream))


class Handle:
    """Owns one dir_handle; use as a context manager or call dir_destroy."""

    def __init__(self, ptr, device, stream=None):
        self.ptr = ptr
        self.device = device
        self.stream = stream      # torch stream the handle enqueues on (None: the current one at creation)
        self.inflight = None      # tensors and stats buffer of a registration not yet collected

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        dir_destroy(self)

    def __del__(self):
        try:
            if self.ptr:
                lib().dir_destroy(self.ptr)
                self.ptr = ctypes.c_void_p()
        except Exception:
            pass

    @property
    def _as_param_(self):
        return self.ptr


def dir_abi_version():
    return lib().dir_abi_version()


def dir_strerror(code):
    return _strerror(code)


def dir_create(device=0, stream=None):
    h = ctypes.c_void_p()
    if stream is None:
        stream = torch.cuda.current_stream(device)
    _check(lib().dir_create(ctypes.byref(h), int(device), _stream_ptr(stream, device)), "dir_create")
    return Handle(h, device, stream if isinstance(stream, torch.cuda.Stream) else None)


def dir_set_stream(h, stream):
    if stream is None:
        stream = torch.cuda.current_stream(h.device)
    _check(lib().dir_set_stream(h.ptr, _stream_ptr(stream, h.device)), "dir_set_stream")
    h.stream = stream if isinstance(stream, torch.cuda.Stream) else None


def dir_destroy(h):
    if h is not None and h.ptr:
        rc = lib().dir_destroy(h.ptr)
        h.ptr = ctypes.c_void_p()
        _check(rc, "dir_destroy")


def dir_set_graphs(h, enable):
    _check(lib().dir_set_graphs(h.ptr, int(bool(enable))), "dir_set_graphs")


def dir_synchronize(h):
    _check(lib().dir_synchronize(h.ptr), "dir_synchronize")


def make_params(variant, iters, sigma, radius=0, alpha=1.0, eps=0.0, compose_iters=-1, storage="f32", units="voxels",
                image_sigma=0.0):
    """dir_params; `iters` lists the levels coarsest first.  units "mm"
    (sigma and image_sigma in mm) needs spacing_mm in the registration call."""
    if isinstance(variant, str):
        variant = VARIANTS[variant]
    iters = [int(i) for i in iters]
    if not 1 <= len(iters) <= DIR_MAX_LEVELS:
        raise ValueError("1..8 levels")
    p = dir_params()
    p.struct_size = ctypes.sizeof(dir_params)
    p.variant = int(variant)
    p.alpha = float(alpha)
    p.sigma = float(sigma)
    p.radius = int(radius)
    p.levels = len(iters)
    for k, n in enumerate(iters):
        p.iters[k] = n
    p.eps = float(eps)
    p.compose_iters = int(compose_iters)
    p.storage = STORAGE[storage] if isinstance(storage, str) else int(storage)
    p.units = UNITS[units] if isinstance(units, str) else int(units)
    p.image_sigma = float(image_sigma)
    return p


def _register_args(static, moving, params, field_out, spacing_mm):
    _dev_f32(static, "static", 3)
    _dev_f32(moving, "moving", 3)
    if static.shape != moving.shape:
        raise ValueError("static and moving differ in shape")
    if field_out is None:
        field_out = torch.empty((3,) + tuple(static.shape), dtype=torch.float32, device=static.device)
    _dev_f32(field_out, "field_out", 4)
    sp = (ctypes.c_double * 3)(*spacing_mm) if spacing_mm is not None else None
    return field_out, sp


def _new_stats(params, history):
    st = dir_stats()
    st.struct_size = ctypes.sizeof(dir_stats)
    total = sum(params.iters[k] for k in range(params.levels))
    buf = (ctypes.c_double * max(4 * total, 4))() if history else None
    if history:
        st.history = ctypes.cast(buf, ctypes.POINTER(ctypes.c_double))
        st.history_capacity = total
    return st, buf


def _stats_dict(rc, st, buf):
    stats = {"rc": rc, "levels": st.levels, "iters_run": list(st.iters_run)[:st.levels],
             "mse_final": st.mse_final, "relnorm_final": st.relnorm_final, "history": None}
    if buf is not None:
        stats["history"] = [tuple(buf[4 * i:4 * i + 4]) for i in range(st.history_len)]
    return stats


def dir_register(h, static, moving, params, field_out=None, spacing_mm=None, history=True):
    """Register `moving` onto `static`; returns (field [3,nz,ny,nx], stats dict)."""
    field_out, sp = _register_args(static, moving, params, field_out, spacing_mm)
    nx, ny, nz = _dims(static)
    st, buf = _new_stats(params, history)
    rc = lib().dir_register(h.ptr, _ptr(static), _ptr(moving), nx, ny, nz, sp, ctypes.byref(params),
                            _ptr(field_out), ctypes.byref(st))
    stats = _stats_dict(rc, st, buf)
    if rc != DIR_OK:
        raise DemonsError(rc, "dir_register")
    return field_out, stats


def _batch_args(h, statics, movings, params, field_outs, spacing_mm, history):
    count = len(statics)
    if not 1 <= count <= DIR_MAX_BATCH or len(movings) != count or len(params) != count:
        raise ValueError(f"1..{DIR_MAX_BATCH} registrations, with one moving image and one dir_params each")
    if field_outs is None:
        field_outs = [None] * count
    if spacing_mm is not None and len(spacing_mm) != count:
        raise ValueError("spacing_mm: one (x, y, z) triple per registration")
    outs, dims = [], []
    for k in range(count):
        o, _ = _register_args(statics[k], movings[k], params[k], field_outs[k], None)
        outs.append(o)
        dims.extend(_dims(statics[k]))
    sp = (ctypes.c_double * (3 * count))(*[float(v) for t in spacing_mm for v in t]) if spacing_mm is not None \
        else None
    if h.stream is not None and h.stream != torch.cuda.current_stream(h.device):
        h.stream.wait_stream(torch.cuda.current_stream(h.device))
    ptrs = lambda ts: (ctypes.c_void_p * count)(*[t.data_ptr() for t in ts])
    parr = (dir_params * count)(*params)
    sts, bufs = [], []
    for p in params:
        st, buf = _new_stats(p, history)
        sts.append(st)
        bufs.append(buf)
    sarr = (dir_stats * count)(*sts)
    args = (h.ptr, count, ptrs(statics), ptrs(movings), (ctypes.c_int32 * (3 * count))(*dims), sp, parr, ptrs(outs))
    return args, outs, sarr, bufs


def dir_register_batch(h, statics, movings, params, field_outs=None, spacing_mm=None, history=True):
    """Lockstep batch of len(statics) registrations (at most DIR_MAX_BATCH),
    of any sizes; `params` is a list of dir_params that agree in levels,
    iterations, sigma, radius and storage; `spacing_mm` is None or one triple
    per registration.  Returns a list of (field, stats dict), each field
    bitwise the one dir_register computes."""
    args, outs, sarr, bufs = _batch_args(h, statics, movings, params, field_outs, spacing_mm, history)
    rc = lib().dir_register_batch(*args, sarr)
    res = [(outs[k], _stats_dict(rc, sarr[k], bufs[k])) for k in range(len(outs))]
    if rc != DIR_OK:
        raise DemonsError(rc, "dir_register_batch")
    return res


def dir_register_batch_async(h, statics, movings, params, field_outs=None, spacing_mm=None, history=True):
    """dir_register_batch without the wait; dir_wait(h) returns its list of
    (field, stats dict)."""
    args, outs, sarr, bufs = _batch_args(h, statics, movings, params, field_outs, spacing_mm, history)
    _check(lib().dir_register_batch_async(*args), "dir_register_batch_async")
    h.inflight = ("batch", (statics, movings, params), outs, sarr, bufs)
    return outs


def dir_autotune(h, shape_zyx, params, count=1):
    """Time the smoothing kernel's z-chunk depths at every pyramid level of a
    volume of shape (nz, ny, nx) for launches of `count` registrations and
    keep the fastest (process-wide); returns them, finest level first."""
    nz, ny, nx = shape_zyx
    depths = (ctypes.c_int32 * params.levels)()
    _check(lib().dir_autotune(h.ptr, int(nx), int(ny), int(nz), ctypes.byref(params), int(count), depths),
           "dir_autotune")
    return list(depths)


def dir_autotune_clear():
    lib().dir_autotune_clear()


def dir_register_async(h, static, moving, params, field_out=None, spacing_mm=None, history=True):
    """Enqueue a registration on the handle's stream and return at once; the
    field is complete when dir_wait(h) returns.  The handle's stream first
    waits for the caller's current stream (where the inputs were made)."""
    field_out, sp = _register_args(static, moving, params, field_out, spacing_mm)
    nx, ny, nz = _dims(static)
    if h.stream is not None and h.stream != torch.cuda.current_stream(h.device):
        h.stream.wait_stream(torch.cuda.current_stream(h.device))
    rc = lib().dir_register_async(h.ptr, _ptr(static), _ptr(moving), nx, ny, nz, sp, ctypes.byref(params),
                                  _ptr(field_out))
    _check(rc, "dir_register_async")
    st, buf = _new_stats(params, history)
    h.inflight = (static, moving, field_out, params, st, buf)
    return field_out


def dir_wait(h):
    """Collect the registration enqueued by dir_register_async: (field, stats)."""
    if h.inflight is None:
        raise DemonsError(DIR_EINVAL, "dir_wait: nothing in flight")
    if h.inflight[0] == "batch":
        _, _, outs, sarr, bufs = h.inflight
        rc = lib().dir_wait(h.ptr, sarr)
        h.inflight = None
        res = [(outs[k], _stats_dict(rc, sarr[k], bufs[k])) for k in range(len(outs))]
        if rc != DIR_OK:
            raise DemonsError(rc, "dir_wait")
        return res
    _, _, field_out, _, st, buf = h.inflight
    rc = lib().dir_wait(h.ptr, ctypes.byref(st))
    h.inflight = None
    stats = _stats_dict(rc, st, buf)
    if rc != DIR_OK:
        raise DemonsError(rc, "dir_wait")
    return field_out, stats


def dir_warp(h, vol, field, out=None):
    _dev_f32(vol, "vol", 3)
    _dev_f32(field, "field", 4)
    if field.shape[1:] != vol.shape or field.shape[0] != 3:
        raise ValueError("field must be [3] + vol.shape")
    out = torch.empty_like(vol) if out is None else _dev_f32(out, "out", 3)
    _check(lib().dir_warp(h.ptr, _ptr(vol), _ptr(field), *_dims(vol), _ptr(out)), "dir_warp")
    return out


def dir_gradient(h, img, out=None):
    _dev_f32(img, "img", 3)
    out = torch.empty((3,) + tuple(img.shape), dtype=torch.float32, device=img.device) if out is None else out
    _dev_f32(out, "out", 4)
    _check(lib().dir_gradient(h.ptr, _ptr(img), *_dims(img), _ptr(out)), "dir_gradient")
    return out


def dir_smooth(h, x, sigma, radius=0, out=None):
    """Smooth a volume [nz,ny,nx] or a stack [c,nz,ny,nx] (c <= 3)."""
    if x.dim() == 3:
        ncomp = 1
        _dev_f32(x, "x", 3)
    else:
        _dev_f32(x, "x", 4)
        ncomp = x.shape[0]
    out = torch.empty_like(x) if out is None else out
    _dev_f32(out, "out", x.dim())
    _check(lib().dir_smooth(h.ptr, _ptr(x), ncomp, *_dims(x), float(sigma), int(radius), _ptr(out)), "dir_smooth")
    return out


def coarse_shape(shape3):
    return tuple((int(n) + 1) // 2 for n in shape3)


def dir_restrict(h, x, out=None):
    _dev_f32(x, "x", 3)
    out = torch.empty(coarse_shape(x.shape), dtype=torch.float32, device=x.device) if out is None else out
    _dev_f32(out, "out", 3)
    _check(lib().dir_restrict(h.ptr, _ptr(x), *_dims(x), _ptr(out)), "dir_restrict")
    return out


def dir_prolong(h, coarse, fine_shape3, out=None):
    _dev_f32(coarse, "coarse", 4)
    fz, fy, fx = (int(n) for n in fine_shape3)
    out = torch.empty((3, fz, fy, fx), dtype=torch.float32, device=coarse.device) if out is None else out
    _dev_f32(out, "out", 4)
    _check(lib().dir_prolong(h.ptr, _ptr(coarse), *_dims(coarse), _ptr(out), fx, fy, fz), "dir_prolong")
    return out


def dir_force(h, variant, alpha, static, moving, field, out=None):
    """u = v + dr (Eqs 1-6) and the FP64 sums (sum|dr|, sum|v|, sum D^2)."""
    if isinstance(variant, str):
        variant = VARIANTS[variant]
    _dev_f32(static, "static", 3)
    _dev_f32(moving, "moving", 3)
    _dev_f32(field, "field", 4)
    out = torch.empty_like(field) if out is None else _dev_f32(out, "out", 4)
    sums = (ctypes.c_double * 3)()
    _check(lib().dir_force(h.ptr, int(variant), float(alpha), _ptr(static), _ptr(moving), _ptr(field),
                           *_dims(static), _ptr(out), sums), "dir_force")
    return out, tuple(sums)


def dir_step(h, variant, alpha, static, moving, field, sigma, radius=0, out=None):
    """One iteration as inside dir_register: G_sigma * (v + dr), and the sums."""
    if isinstance(variant, str):
        variant = VARIANTS[variant]
    _dev_f32(static, "static", 3)
    _dev_f32(moving, "moving", 3)
    _dev_f32(field, "field", 4)
    out = torch.empty_like(field) if out is None else _dev_f32(out, "out", 4)
    sums = (ctypes.c_double * 3)()
    _check(lib().dir_step(h.ptr, int(variant), float(alpha), _ptr(static), _ptr(moving), _ptr(field),
                          *_dims(static), float(sigma), int(radius), _ptr(out), sums), "dir_step")
    return out, tuple(sums)


def dir_step_stored(h, storage, variant, alpha, static, moving, field, sigma, radius=0, out=None):
    """dir_step with images and field held in `storage` ("f32", "f16", "bf16")."""
    if isinstance(variant, str):
        variant = VARIANTS[variant]
    st = STORAGE[storage] if isinstance(storage, str) else int(storage)
    _dev_f32(static, "static", 3)
    _dev_f32(moving, "moving", 3)
    _dev_f32(field, "field", 4)
    out = torch.empty_like(field) if out is None else _dev_f32(out, "out", 4)
    sums = (ctypes.c_double * 3)()
    _check(lib().dir_step_stored(h.ptr, st, int(variant), float(alpha), _ptr(static), _ptr(moving), _ptr(field),
                                 *_dims(static), float(sigma), int(radius), _ptr(out), sums), "dir_step_stored")
    return out, tuple(sums)


def dir_step_noalloc(h, variant, alpha, static, moving, field, sigma, radius=0, out=None):
    """dir_step with its intermediates in the library's fixed scratch array
    (no allocation inside the call; `out` is allocated here when None)."""
    if isinstance(variant, str):
        variant = VARIANTS[variant]
    _dev_f32(static, "static", 3)
    _dev_f32(moving, "moving", 3)
    _dev_f32(field, "field", 4)
    out = torch.empty_like(field) if out is None else _dev_f32(out, "out", 4)
    sums = (ctypes.c_double * 3)()
    _check(lib().dir_step_noalloc(h.ptr, int(variant), float(alpha), _ptr(static), _ptr(moving), _ptr(field),
                                  *_dims(static), float(sigma), int(radius), _ptr(out), sums), "dir_step_noalloc")
    return out, tuple(sums)


def dir_similarity(h, static, moving, field=None):
    """(mse, cc) of static and moving deformed by field (None: undeformed)."""
    _dev_f32(static, "static", 3)
    _dev_f32(moving, "moving", 3)
    if field is not None:
        _dev_f32(field, "field", 4)
    mse, cc = ctypes.c_double(), ctypes.c_double()
    _check(lib().dir_similarity(h.ptr, _ptr(static), _ptr(moving), _ptr(field) if field is not None else None,
                                *_dims(static), ctypes.byref(mse), ctypes.byref(cc)), "dir_similarity")
    return mse.value, cc.value


def dir_compose(h, half, K=-1, out=None):
    _dev_f32(half, "half", 4)
    out = torch.empty_like(half) if out is None else _dev_f32(out, "out", 4)
    _check(lib().dir_compose(h.ptr, _ptr(half), *_dims(half), int(K), _ptr(out)), "dir_compose")
    return out


def dir_timing_names():
    L = lib()
    return [L.dir_timing_name(k).decode() for k in range(L.dir_timing_count())]


def dir_timing_enable(h, kernels=()):
    """Time the named kernels (or indices) from now on; () stops timing."""
    names = dir_timing_names()
    mask = 0
    for k in kernels:
        mask |= 1 << (names.index(k) if isinstance(k, str) else int(k))
    _check(lib().dir_timing_enable(h.ptr, ctypes.c_uint64(mask)), "dir_timing_enable")


def dir_timing_read(h, kernel, level=None):
    """(device ms, launches) of a timed kernel; `level` (0 = finest) restricts
    the totals to one pyramid level."""
    names = dir_timing_names()
    k = names.index(kernel) if isinstance(kernel, str) else int(kernel)
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    if level is None:
        _check(lib().dir_timing_read(h.ptr, k, ctypes.byref(ms), ctypes.byref(n)), "dir_timing_read")
    else:
        _check(lib().dir_timing_read_level(h.ptr, k, int(level), ctypes.byref(ms), ctypes.byref(n)),
               "dir_timing_read_level")
    return ms.value, n.value


def dir_workspace_bytes(shape_zyx, params):
    """Device bytes a handle allocates for a registration of this shape [nz, ny, nx]."""
    nz, ny, nx = shape_zyx
    b = ctypes.c_uint64()
    _check(lib().dir_workspace_bytes(int(nx), int(ny), int(nz), ctypes.byref(params), ctypes.byref(b)),
           "dir_workspace_bytes")
    return b.value


class Pool:
    """dir_pool: registrations of any size admitted by workspace budget onto
    `slots` streams, up to `max_batch` compatible ones per slot as a lockstep
    batch.  submit() keeps the request's tensors alive until its result is
    taken by poll() or wait()."""

    def __init__(self, slots=4, max_bytes=0, device=0, max_batch=1):
        self.ptr = ctypes.c_void_p()
        _check(lib().dir_pool_create(ctypes.byref(self.ptr), int(device), int(slots), ctypes.c_uint64(max_bytes)),
               "dir_pool_create")
        if max_batch != 1:
            rc = lib().dir_pool_set_max_batch(self.ptr, int(max_batch))
            if rc != DIR_OK:
                lib().dir_pool_destroy(self.ptr)
                self.ptr = ctypes.c_void_p()
                raise DemonsError(rc, "dir_pool_set_max_batch")
        self.device = device
        self._live = {}

    def submit(self, static, moving, params, field_out=None, spacing_mm=None):
        field_out, sp = _register_args(static, moving, params, field_out, spacing_mm)
        nx, ny, nz = _dims(static)
        t = ctypes.c_int64()
        _check(lib().dir_pool_submit(self.ptr, _ptr(static), _ptr(moving), nx, ny, nz, sp, ctypes.byref(params),
                                     _ptr(field_out), ctypes.byref(t)), "dir_pool_submit")
        self._live[t.value] = (static, moving, field_out, params)
        return t.value

    def _stats(self):
        st = dir_stats()
        st.struct_size = ctypes.sizeof(dir_stats)
        return st

    def poll(self, ticket):
        """None while running or queued, else (field, stats dict)."""
        st = self._stats()
        done = ctypes.c_int32()
        rc = lib().dir_pool_poll(self.ptr, int(ticket), ctypes.byref(st), ctypes.byref(done))
        if not done.value:
            _check(rc, "dir_pool_poll")
            return None
        live = self._live.pop(ticket, None)
        if rc != DIR_OK:
            raise DemonsError(rc, "dir_pool_poll")
        return live[2], _stats_dict(rc, st, None)

    def wait(self, ticket):
        st = self._stats()
        rc = lib().dir_pool_wait(self.ptr, int(ticket), ctypes.byref(st))
        live = self._live.pop(ticket, None)
        if rc != DIR_OK:
            raise DemonsError(rc, "dir_pool_wait")
        return live[2], _stats_dict(rc, st, None)

    def progress(self):
        _check(lib().dir_pool_progress(self.ptr), "dir_pool_progress")

    def stats(self):
        held, peak = ctypes.c_uint64(), ctypes.c_uint64()
        run, q = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().dir_pool_stats(self.ptr, ctypes.byref(held), ctypes.byref(peak), ctypes.byref(run),
                                    ctypes.byref(q)), "dir_pool_stats")
        return {"held_bytes": held.value, "peak_bytes": peak.value, "peak_running": run.value, "queued": q.value}

    def close(self):
        if self.ptr:
            lib().dir_pool_destroy(self.ptr)
            self.ptr = ctypes.c_void_p()
            self._live.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
