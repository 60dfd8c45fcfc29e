"""Registrations with images and fields stored in 16-bit formats (FP32
arithmetic, FP64 sums), against the FP64 oracle and the FP32 path.

Per step, the oracle gets the same 16-bit-representable inputs the kernels
see, so the field must agree to the rounding of the two stored intermediates
(x-smoothed u and the output): 2 unit roundoffs plus FP32 slack; the FP64
sums (|dr|, |v|, D^2) to the FP32 bound where D is formed inside the force
kernel, and to D's storage rounding where it comes from the pre-warp.
End to end the rounding of the field every iteration is a perturbation of
the iteration; the result is compared with the FP32 path and with the
ground truth, and the error against the oracle is printed."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_0909_0928_amd import phantom as P

gpu = [pytest.mark.gpu, pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]


def on_gpu(f):
    for m in gpu:
        f = m(f)
    return f

UNIT_ROUNDOFF = {"f16": 2.0 ** -11, "bf16": 2.0 ** -8}


@pytest.fixture(scope="module")
def B():
    from paper_0909_0928_amd import binding
    return binding


@pytest.fixture(scope="module")
def h(B):
    handle = B.dir_create(0)
    yield handle
    B.dir_destroy(handle)


def round_to(a, fmt):
    """Round float64 values to the storage format (nearest even), back as float64."""
    a = np.asarray(a, dtype=np.float64)
    if fmt == "f16":
        return a.astype(np.float16).astype(np.float64)
    if fmt == "bf16":
        u = np.ascontiguousarray(a.astype(np.float32)).view(np.uint32).astype(np.uint64)
        u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
        return u.astype(np.uint32).view(np.float32).astype(np.float64)
    return a.astype(np.float32).astype(np.float64)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, dtype=np.float32))).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def rel(a, b):
    return np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel())


def worst(a, b):
    """Largest element error relative to max|b| (the per-element bound beside
    the normwise one)."""
    return float(np.abs(a - b).max()) / float(np.abs(b).max())


def test_round_to_matches_definition():
    # bfloat16 keeps the upper 16 bits of binary32, ties to even
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 1.0 + 2 ** -9, 1.0 + 3 * 2 ** -9, -1000.5])
    assert list(round_to(x, "bf16")) == [1.0, 1.0, 1.0 + 2 ** -6, 1.0, 1.0 + 2 ** -7, -1000.0]
    assert round_to(np.array([1.0 + 2 ** -11]), "f16")[0] == 1.0


@on_gpu
@pytest.mark.parametrize("fmt", ["f16", "bf16"])
@pytest.mark.parametrize("shape3", [(11, 13, 17), (9, 33, 65), (3, 4, 530)])
@pytest.mark.parametrize("variant", ["passive", "evolved", "active", "double", "inverse_consistent"])
def test_step_stored(B, h, fmt, shape3, variant):
    nz, ny, nx = shape3
    ph = P.make_phantom((nx, ny, nz), seed=31, max_u=2.0)
    S, M = round_to(ph.static, fmt), round_to(ph.moving, fmt)
    v = round_to(P.random_field((nx, ny, nz), 32, amp=2.0), fmt)
    alpha = 0.4 if variant == "double" else 1.0
    out, sums = B.dir_step_stored(h, fmt, variant, alpha, dev(S), dev(M), dev(v), 1.5, 5)
    u_ref, sums_ref = O.force(O.VARIANTS[variant], S, M, v, alpha=alpha)
    ref = O.smooth(u_ref, 1.5, 5)
    got = host(out)
    assert rel(got, ref) <= 2.5 * UNIT_ROUNDOFF[fmt]
    # per element: the two stored roundings of at most max|ref| each
    assert worst(got, ref) <= 4 * UNIT_ROUNDOFF[fmt]
    # Passive and evolved form D from the stored images inside the force
    # kernel: their sums see exactly the oracle's inputs.  The other variants
    # read D back from the pre-warp, stored in the format: D's
    # relative rounding bounds the force's (|d ln dr / d ln D| <= 1), hence 2u.
    tol = 1e-5 if variant in ("passive", "evolved") else 2.0 * UNIT_ROUNDOFF[fmt]
    for k in range(3):
        assert abs(sums[k] - sums_ref[k]) <= tol * abs(sums_ref[k]) + 1e-12


@on_gpu
def test_step_stored_f32_is_dir_step(B, h):
    ph = P.make_phantom((40, 24, 12), seed=33, max_u=2.0)
    v = P.random_field((40, 24, 12), 34, amp=2.0)
    a, sa = B.dir_step(h, "inverse_consistent", 1.0, dev(ph.static), dev(ph.moving), dev(v), 1.5, 5)
    b, sb = B.dir_step_stored(h, "f32", "inverse_consistent", 1.0, dev(ph.static), dev(ph.moving), dev(v), 1.5, 5)
    assert torch.equal(a, b) and sa == sb


@pytest.fixture(scope="module")
def small_pair():
    ph = P.make_phantom((64, 64, 32), seed=1, max_u=3.0)
    return ph


@on_gpu
@pytest.mark.parametrize("variant", ["passive", "inverse_consistent"])
def test_end_to_end_storage(B, h, small_pair, variant):
    ph = small_pair
    S, M = dev(ph.static), dev(ph.moving)
    iters = [50] if variant == "passive" else [30, 20]
    f32, _ = B.dir_register(h, S, M, B.make_params(variant, iters, sigma=1.0, radius=3))
    f32 = host(f32)
    S64, M64 = ph.static.astype(np.float32).astype(np.float64), ph.moving.astype(np.float32).astype(np.float64)
    body = ph.body
    z, y, x = np.nonzero(body)
    vt, _ = ph.ground_truth(x.astype(float), y.astype(float), z.astype(float))

    def gt_err(f):
        return float(np.sqrt(((f[:, body] - vt) ** 2).sum(axis=0)).mean())

    def rms(a, b, mask=None):
        d = ((a - b) ** 2).sum(axis=0)
        return float(np.sqrt((d[mask] if mask is not None else d).mean()))

    e32 = gt_err(f32)
    print(f"\n{variant}: FP32 GT error {e32:.4f} vox")
    for fmt in ("f16", "bf16"):
        f, stats = B.dir_register(h, S, M, B.make_params(variant, iters, sigma=1.0, radius=3, storage=fmt))
        f = host(f)
        # the oracle on the images rounded to the format: separates the
        # quantisation of the inputs from the storage of fields and D/P
        ref_q, _, _, _ = O.register(round_to(S64, fmt), round_to(M64, fmt), O.VARIANTS[variant], iters,
                                    sigma=1.0, radius=3)
        e = gt_err(f)
        print(f"{variant} {fmt}: GT error {e:.4f} vox ({e - e32:+.4f}); RMS vs FP32 all {rms(f, f32):.4f} "
              f"body {rms(f, f32, body):.4f}; RMS vs oracle on rounded images all {rms(f, ref_q):.4f} "
              f"body {rms(f, ref_q, body):.4f}")
        assert np.isfinite(f).all()
        assert e - e32 <= 0.05                      # ground-truth error degrades by at most 0.05 voxel
        # inside the body the stored fields (and D) move the result from the
        # oracle on the same rounded images by the format's rounding, not more
        # (measured: f16 <= 0.009, bf16 <= 0.05 voxel RMS)
        assert rms(f, ref_q, body) <= (0.02 if fmt == "f16" else 0.1)


# The y/z smoothing of 16-bit fields with even nx runs two columns per lane
# (one 4-byte access per column pair) when a launch has at least 1,024
# workgroups of 128 columns x 16 rows x 4 planes per component.
# 256 x 128 x 96 gives 2 * 8 * 24 * 3 = 1152 such workgroups.
TWO_COLUMN_SHAPE = (96, 128, 256)   # nz, ny, nx


@on_gpu
@pytest.mark.parametrize("fmt", ["f16", "bf16"])
@pytest.mark.parametrize("variant", ["passive", "inverse_consistent"])
def test_step_stored_two_column_smoothing(B, h, fmt, variant):
    """The two-column 16-bit smoothing against the oracle (force + smoothing on
    the same rounded inputs), normwise and per element."""
    nz, ny, nx = TWO_COLUMN_SHAPE
    ph = P.make_phantom((nx, ny, nz), seed=35, max_u=3.0)
    S, M = round_to(ph.static, fmt), round_to(ph.moving, fmt)
    v = round_to(P.random_field((nx, ny, nz), 36, amp=2.5), fmt)
    out, sums = B.dir_step_stored(h, fmt, variant, 1.0, dev(S), dev(M), dev(v), 1.5, 5)
    u_ref, sums_ref = O.force(O.VARIANTS[variant], S, M, v)
    ref = O.smooth(u_ref, 1.5, 5)
    got = host(out)
    assert rel(got, ref) <= 2.5 * UNIT_ROUNDOFF[fmt]
    assert worst(got, ref) <= 4 * UNIT_ROUNDOFF[fmt]
    tol = 1e-5 if variant == "passive" else 2.0 * UNIT_ROUNDOFF[fmt]
    for k in range(3):
        assert abs(sums[k] - sums_ref[k]) <= tol * abs(sums_ref[k]) + 1e-12


@on_gpu
@pytest.mark.parametrize("fmt", ["f16", "bf16"])
def test_two_column_smoothing_equals_one_column(B, h, fmt):
    """Bitwise: a registration of the two-column shape alone (its smoothing
    launches take two columns per lane) against the same registration in a
    lockstep batch with an odd-nx companion of the same z-chunk depth (4), whose
    shared launches then take one column per lane for both."""
    B.dir_autotune_clear()   # untuned depths: 4 for both registrations
    nz, ny, nx = TWO_COLUMN_SHAPE
    a = P.make_phantom((nx, ny, nz), seed=37, max_u=3.0)
    b = P.make_phantom((255, 128, 24), seed=38, max_u=3.0)
    p = B.make_params("inverse_consistent", [3], sigma=1.5, radius=5, storage=fmt)
    q = B.make_params("passive", [3], sigma=1.5, radius=5, storage=fmt)
    alone, st_alone = B.dir_register(h, dev(a.static), dev(a.moving), p)
    res = B.dir_register_batch(h, [dev(a.static), dev(b.static)], [dev(a.moving), dev(b.moving)], [p, q])
    (in_batch, st_batch), _ = res
    assert torch.equal(alone, in_batch)
    assert np.array_equal(np.array(st_alone["history"]), np.array(st_batch["history"]), equal_nan=True)
