"""The HIP path at the largest volume the ABI accepts, against the FP64 oracle.

993 x 1057 x 341 = 357,913,941 voxels is exactly the limit (a three-component
FP32 field just under 4 GiB), and every axis is ragged: x spans a full and a
481-voxel 512-wide force tile, y ends in a one-row smoothing tile, z in a
five-plane chunk.  The oracle cannot run a volume this size, so outputs are
checked at sampled voxels, each against the oracle run on a crop around it:
the crop reaches every input the sampled output depends on (smoothing radius,
stencil, trilinear neighbours and the largest displacement), and where it
meets the volume boundary it keeps that boundary, so clamping is the same.
Full-volume FP64 sums that have a plain definition (sum |v|, and the
intensity error of the undeformed pair) are checked in full.
"""
import math
import sys

import numpy as np
import pytest
import torch

import oracle as O
from paper_0909_0928_amd import phantom as P

pytestmark = [pytest.mark.gpu, pytest.mark.slow,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

REL_TOL = 1e-5
NX, NY, NZ = 993, 1057, 341
SHAPE = (NZ, NY, NX)
AMP = 2.5               # |v_c| <= AMP for the separable field
SIGMA, RADIUS = 1.5, 5


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _rel(a, b, base):
    return np.linalg.norm((a - b).ravel()) / np.linalg.norm((b - base).ravel())


def _elem(a, b, base):
    """Worst sampled element's error relative to max|b - base| (the per-element
    bound beside the normwise one)."""
    return float(np.abs(a - b).max()) / float(np.abs(b - base).max())


def _samples():
    """Corners, the far end of each ragged tile and seeded interior points (z, y, x)."""
    pts = [(z, y, x) for z in (0, NZ - 1) for y in (0, NY - 1) for x in (0, NX - 1)]
    pts += [(NZ - 1, NY - 1, NX - 2), (NZ - 3, NY - 1, 511), (NZ - 5, NY - 2, 512), (336, 1056, 480),
            (170, 1040, 992), (4, 16, 600)]
    rng = np.random.default_rng(9001)
    pts += [tuple(int(rng.integers(0, n)) for n in SHAPE) for _ in range(10)]
    return pts


SAMPLES = _samples()


def _crop(p, m):
    sl = tuple(slice(max(0, c - m), min(n, c + m + 1)) for c, n in zip(p, SHAPE))
    loc = tuple(c - s.start for c, s in zip(p, sl))
    return sl, loc


def _pick(t):
    """Field values [3, k] of a device field at the samples."""
    idx = [torch.tensor([p[a] for p in SAMPLES], device=t.device) for a in range(3)]
    return t[:, idx[0], idx[1], idx[2]].double().cpu().numpy()


@pytest.fixture(scope="module")
def big():
    _say(f"max-size inputs {NX}x{NY}x{NZ}: building on the host")
    S = P.noise_volume_f32((NX, NY, NZ), 31, scale=150.0)
    M = P.noise_volume_f32((NX, NY, NZ), 32, scale=150.0)
    v = P.separable_field_f32((NX, NY, NZ), 33, amp=AMP)
    assert S.size == 357_913_941
    dS, dM, dv = (torch.from_numpy(a).cuda() for a in (S, M, v))
    torch.cuda.synchronize()
    yield S, M, v, dS, dM, dv
    del dS, dM, dv
    torch.cuda.empty_cache()


@pytest.fixture(scope="module")
def B():
    from paper_0909_0928_amd import binding
    return binding


@pytest.fixture(scope="module")
def h(B):
    handle = B.dir_create(0)
    yield handle
    B.dir_destroy(handle)


_NORM_SUM = {}


def _sum_norm_v(v):
    """sum over voxels of |v(x)|, in FP64 (computed once per field)."""
    if id(v) not in _NORM_SUM:
        total = 0.0
        for z0 in range(0, NZ, 16):
            s = v[:, z0:z0 + 16].astype(np.float64)
            total += float(np.sqrt((s * s).sum(axis=0)).sum())
        _NORM_SUM[id(v)] = total
    return _NORM_SUM[id(v)]


def test_max_size_warp(B, h, big):
    S, M, v, dS, dM, dv = big
    _say("max-size dir_warp")
    got = B.dir_warp(h, dM, dv)
    torch.cuda.synchronize()
    m = math.ceil(AMP) + 2
    ref = []
    for p in SAMPLES:
        sl, loc = _crop(p, m)
        ref.append(O.warp(M[sl].astype(np.float64), v[(slice(None),) + sl].astype(np.float64))[loc])
    idx = [torch.tensor([p[a] for p in SAMPLES], device="cuda") for a in range(3)]
    g = got[idx[0], idx[1], idx[2]].double().cpu().numpy()
    del got
    ref = np.array(ref)
    assert _rel(g, ref, np.zeros_like(ref)) < REL_TOL
    assert _elem(g, ref, np.zeros_like(ref)) <= 10 * REL_TOL


@pytest.mark.parametrize("variant,alpha", [("passive", 1.0), ("evolved", 1.0), ("active", 1.0), ("double", 0.4),
                                           ("inverse_consistent", 1.0), ("passive", 0.4)])
def test_max_size_step(B, h, big, variant, alpha):
    """One iteration G * (v + dr) as the registration runs it (force, x pass,
    pre-warp where the variant has one, y/z passes with the sums reducer)."""
    S, M, v, dS, dM, dv = big
    _say(f"max-size dir_step {variant} alpha {alpha}")
    out, sums = B.dir_step(h, variant, alpha, dS, dM, dv, SIGMA, RADIUS)
    torch.cuda.synchronize()
    got = _pick(out)
    del out
    m = RADIUS + math.ceil(AMP) + 3
    ref, base = [], []
    for p in SAMPLES:
        sl, loc = _crop(p, m)
        vc = v[(slice(None),) + sl].astype(np.float64)
        u, _ = O.force(O.VARIANTS[variant], S[sl].astype(np.float64), M[sl].astype(np.float64), vc, alpha=alpha)
        ref.append(O.smooth(u, SIGMA, RADIUS)[(slice(None),) + loc])
        base.append(vc[(slice(None),) + loc])
    ref, base = np.array(ref).T, np.array(base).T
    assert _rel(got, ref, base) < REL_TOL
    assert _elem(got, ref, base) <= 10 * REL_TOL
    assert all(math.isfinite(s) and s > 0 for s in sums)
    assert abs(sums[1] - _sum_norm_v(v)) <= REL_TOL * sums[1]


def test_max_size_compose(B, h, big):
    S, M, v, dS, dM, dv = big
    _say("max-size dir_compose K 10")
    half = (dv * 0.5).contiguous()
    got = _pick(B.dir_compose(h, half, 10))
    del half
    hv = v * np.float32(0.5)  # the same (exact) FP32 products as on the device
    m = math.ceil(AMP / 2) + 3
    ref = []
    for p in SAMPLES:
        sl, loc = _crop(p, m)
        ref.append(O.compose(hv[(slice(None),) + sl].astype(np.float64), 10)[(slice(None),) + loc])
    ref = np.array(ref).T
    assert _rel(got, ref, np.zeros_like(ref)) < REL_TOL
    assert _elem(got, ref, np.zeros_like(ref)) <= 10 * REL_TOL


def test_max_size_register(B, h, big):
    """A one-level, two-iteration registration: bitwise the two steps it is
    made of, the first history entry's intensity error equal to the plain
    mean of (M - S)^2, and sampled voxels equal to the oracle's iterations."""
    S, M, v, dS, dM, dv = big
    _say("max-size dir_register passive 1 level 2 iterations")
    f, stats = B.dir_register(h, dS, dM, B.make_params("passive", [2], sigma=SIGMA, radius=RADIUS))
    torch.cuda.synchronize()
    got = _pick(f)
    _say("max-size dir_step x2 from a zero field")
    w = torch.zeros_like(f)
    for _ in range(2):
        w, _ = B.dir_step(h, "passive", 1.0, dS, dM, w, SIGMA, RADIUS)
    torch.cuda.synchronize()
    assert torch.equal(f, w)
    del f, w
    torch.cuda.empty_cache()

    sse = 0.0
    for z0 in range(0, NZ, 16):
        d = M[z0:z0 + 16].astype(np.float64) - S[z0:z0 + 16]
        sse += float((d * d).sum())
    mse0 = stats["history"][0][2]
    assert abs(mse0 - sse / S.size) <= 1e-12 * mse0
    assert stats["history"][0][1] == 0.0  # sum |v| of the zero start field

    # passive, alpha 1: |dr| <= 1/2, and smoothing keeps the bound, so the
    # second iteration gathers within one voxel
    m = (RADIUS + 3) + (RADIUS + 1 + 3)
    ref = []
    for p in SAMPLES:
        sl, loc = _crop(p, m)
        Sc, Mc = S[sl].astype(np.float64), M[sl].astype(np.float64)
        vc, _ = O.iterate(O.VARIANTS["passive"], Sc, Mc, np.zeros((3,) + Sc.shape), 2, SIGMA, RADIUS)
        ref.append(vc[(slice(None),) + loc])
    ref = np.array(ref).T
    assert _rel(got, ref, np.zeros_like(ref)) < REL_TOL
    assert _elem(got, ref, np.zeros_like(ref)) <= 10 * REL_TOL


UNIT_ROUNDOFF = {"f16": 2.0 ** -11, "bf16": 2.0 ** -8}


def _round_f32(a, fmt):
    """FP32 array rounded to the 16-bit format (nearest even), back in FP32,
    slab by slab: what the kernels hold after their storage conversion."""
    out = np.empty_like(a)
    flat_in, flat_out = a.reshape(-1, a.shape[-1]), out.reshape(-1, a.shape[-1])
    step = 1 << 16
    for r0 in range(0, flat_in.shape[0], step):
        x = flat_in[r0:r0 + step]
        if fmt == "f16":
            flat_out[r0:r0 + step] = x.astype(np.float16).astype(np.float32)
        else:  # bfloat16: upper 16 bits of binary32, ties to even (finite inputs)
            u = x.view(np.uint32)
            u = (u + np.uint32(0x7FFF) + ((u >> np.uint32(16)) & np.uint32(1))) & np.uint32(0xFFFF0000)
            flat_out[r0:r0 + step] = u.view(np.float32)
    return out


@pytest.mark.parametrize("fmt", ["f16", "bf16"])
@pytest.mark.parametrize("variant", ["passive", "inverse_consistent"])
def test_max_size_step_stored(B, h, big, fmt, variant):
    """16-bit storage at the largest size: the oracle gets the same
    16-bit-representable inputs, so the step agrees to the rounding of the two
    stored intermediates (x-smoothed u and the output)."""
    S, M, v, _, _, _ = big
    _say(f"max-size dir_step_stored {fmt} {variant}: rounding inputs on the host")
    Sr, Mr, vr = (_round_f32(a, fmt) for a in (S, M, v))
    dS, dM, dv = (torch.from_numpy(a).cuda() for a in (Sr, Mr, vr))
    _say(f"max-size dir_step_stored {fmt} {variant}")
    out, sums = B.dir_step_stored(h, fmt, variant, 1.0, dS, dM, dv, SIGMA, RADIUS)
    torch.cuda.synchronize()
    got = _pick(out)
    del out, dS, dM, dv
    torch.cuda.empty_cache()
    m = RADIUS + math.ceil(AMP) + 3
    ref = []
    for p in SAMPLES:
        sl, loc = _crop(p, m)
        u, _ = O.force(O.VARIANTS[variant], Sr[sl].astype(np.float64), Mr[sl].astype(np.float64),
                       vr[(slice(None),) + sl].astype(np.float64))
        ref.append(O.smooth(u, SIGMA, RADIUS)[(slice(None),) + loc])
    ref = np.array(ref).T
    assert _rel(got, ref, np.zeros_like(ref)) <= 2.5 * UNIT_ROUNDOFF[fmt]
    assert _elem(got, ref, np.zeros_like(ref)) <= 4 * UNIT_ROUNDOFF[fmt]
    assert all(math.isfinite(s) and s > 0 for s in sums)
    total = 0.0
    for z0 in range(0, NZ, 16):
        s = vr[:, z0:z0 + 16].astype(np.float64)
        total += float(np.sqrt((s * s).sum(axis=0)).sum())
    assert abs(sums[1] - total) <= REL_TOL * total
