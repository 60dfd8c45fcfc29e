"""Seeded synthetic 4DCT-shaped inputs for demons registration.

This module only draws inputs: a static CT-like phantom S, a moving image M made
by deforming S with a known smooth random field, and the ground-truth
displacement that registers M back onto S.  It contains none of the
registration arithmetic (no trilinear resampling, gradients, forces or
smoothing), so the HIP path and the FP64 oracle can both consume it without
sharing any of the method's code.

The shapes and intensities stand in for the paper's clinical data set
(Sec 3.1, Table 1: thoracic 4DCT, 256x256x94-112 voxels, 0.97-1.16 x 2.5 mm,
lungs inside the body).  That data set is not available here; everything below
is drawn from ``numpy.random.default_rng(seed)`` in a fixed order (blobs, then
field, then noise).

Array layout: volumes are ``[nz][ny][nx]`` float64 (x fastest); vector fields
are ``[3][nz][ny][nx]`` with components (x, y, z), in voxel units.

Warp convention shared by every consumer: the registered field ``v`` satisfies
``M(x - v(x)) ~= S(x)``.
"""
from __future__ import annotations

import dataclasses
import math
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

BACKGROUND_HU = -1000.0
BODY_HU = 0.0
LUNG_HU = -800.0
EDGE_SCALE_VOX = 0.5          # logistic edge scale of the ellipsoids, in voxels
N_BLOBS = 20
N_FIELD_BUMPS = 8
LIPSCHITZ_LIMIT = 0.8
REDRAW_SEED_STEP = 10 ** 6
MAX_REDRAWS = 100
MIN_WIDTH_AXIS = 16           # axes shorter than this do not set the field's width
SLAB_VOXELS = 1 << 21         # analytic volumes are evaluated in z slabs of at most this many voxels


@dataclasses.dataclass
class Phantom:
    shape: tuple            # (nx, ny, nz)
    seed: int
    max_u: float
    spacing_mm: tuple
    static: np.ndarray      # [nz, ny, nx] float64
    moving: np.ndarray      # [nz, ny, nx] float64
    field_g: np.ndarray     # [3, nz, ny, nx] forward field g used to build M
    body: np.ndarray        # bool mask [nz, ny, nx]
    lung: np.ndarray        # bool mask [nz, ny, nx]
    redraws: int
    lipschitz: float
    _params: dict = dataclasses.field(repr=False, default_factory=dict)

    # -- analytic pieces (no registration arithmetic) ---------------------
    def static_at(self, px, py, pz):
        return _static_analytic(self._params, px, py, pz)

    def g_at(self, px, py, pz):
        return _field_analytic(self._params, px, py, pz)

    def ground_truth(self, px=None, py=None, pz=None, tol=1e-12, max_steps=60):
        """Solve v*(x) = g(x - v*(x)) by fixed-point steps from v = g(x).

        With M(y) = S(y + g(y)), the field v* makes M(x - v*(x)) = S(x)
        exactly (noise aside).  The map is a contraction because the
        Lipschitz constant of g is kept below 0.8.  Returns (v, residual)
        with v of shape [3, ...] matching the points (whole grid by default).
        """
        if px is None:
            nx, ny, nz = self.shape
            pz, py, px = np.meshgrid(np.arange(nz, dtype=np.float64),
                                     np.arange(ny, dtype=np.float64),
                                     np.arange(nx, dtype=np.float64), indexing="ij")
        px = np.asarray(px, np.float64)
        py = np.asarray(py, np.float64)
        pz = np.asarray(pz, np.float64)
        v = np.stack(self.g_at(px, py, pz))
        for _ in range(max_steps):
            nv = np.stack(self.g_at(px - v[0], py - v[1], pz - v[2]))
            step = float(np.max(np.abs(nv - v))) if nv.size else 0.0
            v = nv
            if step < tol:
                break
        res = np.stack(self.g_at(px - v[0], py - v[1], pz - v[2])) - v
        return v, float(np.max(np.abs(res))) if res.size else 0.0


def _by_slabs(fn, px, py, pz, ncomp=0, workers=None):
    """fn(px, py, pz) evaluated over z slabs of the coordinate grids, on
    threads (numpy's element-wise loops release the interpreter lock).  The
    slabs depend only on the grid's shape, so the values do not depend on the
    number of threads.  fn returns one array of the slab's shape, or (ncomp > 0)
    a tuple of ncomp of them, stacked on a new first axis."""
    nz = px.shape[0]
    per = max(1, SLAB_VOXELS // max(1, px[0].size))
    out = np.empty(((ncomp,) if ncomp else ()) + px.shape)

    def run(z0):
        sl = slice(z0, z0 + per)
        r = fn(px[sl], py[sl], pz[sl])
        if ncomp:
            for c in range(ncomp):
                out[c, sl] = r[c]
        else:
            out[sl] = r

    starts = range(0, nz, per)
    workers = workers or min(16, os.cpu_count() or 1)
    if len(starts) == 1 or workers == 1:
        for z0 in starts:
            run(z0)
    else:
        with ThreadPoolExecutor(max_workers=min(workers, len(starts))) as ex:
            list(ex.map(run, starts))
    return out


def _grid(shape):
    nx, ny, nz = shape
    return np.meshgrid(np.arange(nz, dtype=np.float64),
                       np.arange(ny, dtype=np.float64),
                       np.arange(nx, dtype=np.float64), indexing="ij")


def _soft_inside(px, py, pz, centre, semi):
    """Smooth indicator of an ellipsoid: ~1 inside, ~0 outside.

    The edge is a logistic in an approximate signed distance (normalised
    radius minus one, times the smallest semi-axis), scale EDGE_SCALE_VOX.
    """
    r = np.sqrt(((px - centre[0]) / semi[0]) ** 2 + ((py - centre[1]) / semi[1]) ** 2
                + ((pz - centre[2]) / semi[2]) ** 2)
    d = (r - 1.0) * min(semi)
    return 0.5 * (1.0 - np.tanh(0.5 * d / EDGE_SCALE_VOX))


def _static_analytic(p, px, py, pz):
    val = BACKGROUND_HU + (BODY_HU - BACKGROUND_HU) * _soft_inside(px, py, pz, p["body_c"], p["body_a"])
    for c in p["lung_c"]:
        val = val + (LUNG_HU - BODY_HU) * _soft_inside(px, py, pz, c, p["lung_a"])
    for (c, amp, sb) in p["blobs"]:
        val = val + amp * np.exp(-((px - c[0]) ** 2 + (py - c[1]) ** 2 + (pz - c[2]) ** 2) / (2.0 * sb * sb))
    return val


def _field_analytic(p, px, py, pz):
    gx = np.zeros(np.shape(px))
    gy = np.zeros(np.shape(px))
    gz = np.zeros(np.shape(px))
    s2 = 2.0 * p["s"] ** 2
    for (c, a) in p["bumps"]:
        e = p["A"] * np.exp(-((px - c[0]) ** 2 + (py - c[1]) ** 2 + (pz - c[2]) ** 2) / s2)
        gx = gx + a[0] * e
        gy = gy + a[1] * e
        gz = gz + a[2] * e
    return gx, gy, gz


def _max_jacobian_frobenius(g):
    """Largest Frobenius norm of the finite-difference Jacobian of g on the grid."""
    fro2 = np.zeros(g.shape[1:])
    for comp in range(3):
        for axis in range(3):
            if g.shape[1 + axis] < 2:
                continue
            d = np.gradient(g[comp], axis=axis)
            fro2 += d * d
    return float(np.sqrt(fro2.max()))


def make_phantom(shape, seed, max_u, spacing_mm=(1.0, 1.0, 1.0), noise_hu=10.0) -> Phantom:
    """Build one seeded static/moving pair.

    shape      (nx, ny, nz) voxels.
    max_u      the largest |g| on the grid, in voxels (met exactly).
    noise_hu   standard deviation of the Gaussian noise added to M.
    """
    nx, ny, nz = (int(s) for s in shape)
    n = np.array([nx, ny, nz], np.float64)
    centre = (n - 1.0) / 2.0
    body_a = (0.45 * nx, 0.35 * ny, 0.45 * nz)
    lung_a = (0.14 * nx, 0.22 * ny, 0.38 * nz)
    lung_c = (centre + np.array([0.20 * nx, 0.0, 0.0]), centre - np.array([0.20 * nx, 0.0, 0.0]))

    rng = np.random.default_rng(seed)
    # 1) blobs: centres uniform inside the body ellipsoid (rejection), amplitude, width
    blobs = []
    while len(blobs) < N_BLOBS:
        c = rng.uniform(centre - np.array(body_a), centre + np.array(body_a))
        if np.sum(((c - centre) / np.array(body_a)) ** 2) > 1.0:
            continue
        amp = rng.uniform(-300.0, 300.0)
        sb = rng.uniform(2.0, 5.0)
        blobs.append((c, amp, sb))

    # 2) smooth random field, redrawn while too steep
    redraws = 0
    field_rng = rng
    pz, py, px = _grid((nx, ny, nz))
    # bump width: 0.3 x the shortest axis, ignoring thin axes of a slab-like volume
    long_axes = [d for d in (nx, ny, nz) if d >= MIN_WIDTH_AXIS]
    width = 0.3 * float(min(long_axes) if long_axes else max(nx, ny, nz))
    while True:
        bumps = []
        for _ in range(N_FIELD_BUMPS):
            c = field_rng.uniform(np.zeros(3), n - 1.0)
            a = field_rng.normal(size=3)
            bumps.append((c, a))
        params = {"s": width, "A": 1.0, "bumps": bumps}
        g = _by_slabs(lambda x, y, z: _field_analytic(params, x, y, z), px, py, pz, ncomp=3)
        gmax = float(np.sqrt((g * g).sum(axis=0)).max())
        params["A"] = max_u / gmax if gmax > 0 else 0.0
        g = g * params["A"]
        lip = _max_jacobian_frobenius(g)
        if lip < LIPSCHITZ_LIMIT:
            break
        redraws += 1
        if redraws > MAX_REDRAWS:
            raise ValueError(f"no field with Lipschitz constant < {LIPSCHITZ_LIMIT} for shape {shape}, "
                             f"max_u {max_u}")
        field_rng = np.random.default_rng(seed + REDRAW_SEED_STEP * redraws)

    full = {"body_c": centre, "body_a": body_a, "lung_c": lung_c, "lung_a": lung_a, "blobs": blobs}
    full.update(params)

    static = _by_slabs(lambda x, y, z: _static_analytic(full, x, y, z), px, py, pz)
    qx, qy, qz = px + g[0], py + g[1], pz + g[2]
    moving = _by_slabs(lambda x, y, z: _static_analytic(full, x, y, z), qx, qy, qz)
    del qx, qy, qz
    # 3) noise, drawn from the generator that drew the field
    moving = moving + field_rng.normal(0.0, noise_hu, size=moving.shape)

    body = _by_slabs(lambda x, y, z: _soft_inside(x, y, z, centre, body_a), px, py, pz) > 0.5
    lung = np.zeros_like(body)
    for c in lung_c:
        lung |= _by_slabs(lambda x, y, z: _soft_inside(x, y, z, c, lung_a), px, py, pz) > 0.5
    return Phantom(shape=(nx, ny, nz), seed=seed, max_u=float(max_u), spacing_mm=tuple(spacing_mm),
                   static=static, moving=moving, field_g=g, body=body, lung=lung,
                   redraws=redraws, lipschitz=lip, _params=full)


def smooth_translation_pair(shape, t, seed=0, n_blobs=40, width=(2.5, 4.0)):
    """A smooth textured image S (sum of Gaussian blobs) and M(y) = S(y + t).

    Registering M onto S must give v = t in the interior.  Used to check
    recovery of a known sub-voxel translation.
    """
    nx, ny, nz = shape
    rng = np.random.default_rng(seed)
    pz, py, px = _grid(shape)
    n = np.array([nx, ny, nz], np.float64)
    blobs = [(rng.uniform(0.1 * (n - 1), 0.9 * (n - 1)), rng.uniform(200.0, 600.0) * rng.choice([-1, 1]),
              rng.uniform(*width)) for _ in range(n_blobs)]

    def f(qx, qy, qz):
        val = np.zeros(np.shape(qx))
        for c, amp, sb in blobs:
            val = val + amp * np.exp(-((qx - c[0]) ** 2 + (qy - c[1]) ** 2 + (qz - c[2]) ** 2) / (2 * sb * sb))
        return val

    return f(px, py, pz), f(px + t[0], py + t[1], pz + t[2])


def random_volume(shape, seed, scale=100.0):
    """Plain seeded noise volume [nz, ny, nx] (for per-step parity inputs)."""
    nx, ny, nz = shape
    return np.random.default_rng(seed).normal(0.0, scale, size=(nz, ny, nx))


def random_field(shape, seed, amp=2.0):
    """Seeded smooth-ish random displacement field [3, nz, ny, nx] with |v| <~ amp.

    Built from a few random sinusoids so that it is smooth but not aligned
    with the grid.
    """
    nx, ny, nz = shape
    rng = np.random.default_rng(seed)
    pz, py, px = _grid(shape)
    out = np.zeros((3, nz, ny, nx))
    for comp in range(3):
        for _ in range(3):
            k = rng.uniform(-0.4, 0.4, size=3)
            ph = rng.uniform(0, 2 * math.pi)
            out[comp] += np.sin(k[0] * px + k[1] * py + k[2] * pz + ph)
    return out * (amp / 3.0)


# Workloads of the benchmark and the parity tests (sizes in voxels, x fastest).
CONFIG_SMALL = dict(shape=(64, 64, 32), seed=1, max_u=3.0, spacing_mm=(1.0, 1.0, 1.0))
CONFIG_FULL = dict(shape=(256, 256, 100), seed=2, max_u=15.0, spacing_mm=(1.1, 1.1, 2.5))


def noise_volume_f32(shape, seed, scale=100.0):
    """Seeded FP32 noise volume [nz, ny, nx], drawn directly in FP32 so that
    volumes of hundreds of millions of voxels stay cheap to build and hold."""
    nx, ny, nz = shape
    out = np.random.default_rng(seed).standard_normal(size=(nz, ny, nx), dtype=np.float32)
    out *= np.float32(scale)
    return out


def separable_field_f32(shape, seed, amp=2.0):
    """Seeded smooth FP32 field [3, nz, ny, nx] with |v_c| <= amp per component:
    each component is a sum of one sinusoid per axis, (f_z + f_y) + f_x in
    FP32, so a crop of it is a plain slice of the stored array and its
    slope stays below 0.4 * amp / 3 per voxel."""
    nx, ny, nz = shape
    rng = np.random.default_rng(seed)
    out = np.empty((3, nz, ny, nx), dtype=np.float32)
    for c in range(3):
        axes = []
        for n in (nz, ny, nx):
            k = rng.uniform(0.05, 0.4)
            ph = rng.uniform(0.0, 2.0 * math.pi)
            axes.append((np.float32(amp / 3.0) * np.sin(k * np.arange(n) + ph)).astype(np.float32))
        fz, fy, fx = axes
        np.add(fz[:, None, None] + fy[None, :, None], fx[None, None, :], out=out[c])
    return out
