"""HIP path vs the FP64 oracle, through the C ABI.

Both sides get identical FP32-representable inputs (the oracle reads them as
float64).  Per-step outputs must agree to a normwise relative error of 1e-5;
whole registrations to an RMS field difference of 0.01 voxel.
"""
import sys

import numpy as np
import pytest
import torch

import oracle as O
from paper_0909_0928_amd import phantom as P

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

REL_TOL = 1e-5          # per-step normwise relative error
RMS_TOL_VOX = 0.01      # end-to-end field RMS difference, voxels


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def B():
    from paper_0909_0928_amd import binding
    return binding


@pytest.fixture(scope="module")
def h(B):
    handle = B.dir_create(0)
    yield handle
    B.dir_destroy(handle)


def f32(a):
    return np.asarray(a, dtype=np.float32)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(f32(a))).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def rel(a, b):
    nb = np.linalg.norm(b.ravel())
    return np.linalg.norm((a - b).ravel()) / (nb if nb > 0 else 1.0)


def assert_close(a, b, tol=REL_TOL, elem=10 * REL_TOL, extra=None):
    """Normwise relative error below tol, and every element within elem of
    max|b| (plus extra[i], a per-element rounding bound where one is derived
    for the operation): a wrong border plane or tile edge can hide under the
    norm of a large volume, not under the per-element bound."""
    r = rel(a, b)
    scale = float(np.abs(b).max()) if b.size else 0.0
    s = scale if scale > 0 else 1.0
    err = np.abs(a - b)
    if extra is not None:
        err = np.maximum(err - extra, 0.0)
    m = float(err.max()) / s if b.size else 0.0
    assert r < tol and m <= elem, f"normwise {r:.2e} (bound {tol:.0e}), worst element {m:.2e} of max|ref| " \
                                  f"beyond its rounding bound (bound {elem:.0e})"


U32 = 2.0 ** -24   # unit roundoff of FP32


def ic_force_rounding_bound(S, M, v, alpha=1.0):
    """Per voxel, a first-order bound on how far the inverse-consistent force
    (Eq 6) moves when the kernels' FP32 intermediates P = Im + Is and
    D = Im - Is are each rounded once (relative U32) before the central
    difference of P is taken.  P sits near twice the image intensity
    (about -2000 HU in air), so a gradient component (P[i+1] - P[i-1]) / 2
    moves by up to U32 (|P[i+1]| + |P[i-1]|) / 2, which is large against a
    gradient of a few thousandths.  With den = alpha^2 D^2 + |g|^2 and
    f = D g / den, |df| <= 3 (|D| |dg| + |g| |dD|) / den.  Doubled for the
    second-order terms and the FP32 arithmetic of the force itself."""
    Im = O.warp(M, v)
    Is = O.warp(S, v, sign=-1.0)
    Pp, D = Im + Is, Im - Is
    g = O.gradient(Pp)
    dg2 = np.zeros_like(Pp)
    for axis in range(3):
        n = Pp.shape[axis]
        hi = np.take(np.abs(Pp), np.minimum(np.arange(n) + 1, n - 1), axis=axis)
        lo = np.take(np.abs(Pp), np.maximum(np.arange(n) - 1, 0), axis=axis)
        dg2 += (U32 * (hi + lo) / 2) ** 2
    den = alpha * alpha * D * D + (g * g).sum(axis=0)
    gn = np.sqrt((g * g).sum(axis=0))
    b = np.where(den > 1e-9, 3 * (np.abs(D) * np.sqrt(dg2) + gn * U32 * np.abs(D)) / np.where(den > 1e-9, den, 1.0),
                 0.0)
    return 2 * b[None]


def rms_vox(a, b):
    return float(np.sqrt(((a - b) ** 2).sum(axis=0).mean()))


SHAPES = [(11, 13, 17), (9, 33, 65), (5, 4, 70), (1, 7, 9), (3, 1, 130), (16, 64, 64)]


def _img(shape3, seed):
    return f32(P.random_volume((shape3[2], shape3[1], shape3[0]), seed, scale=150.0)).astype(np.float64)


def _fld(shape3, seed, amp=2.5):
    return f32(P.random_field((shape3[2], shape3[1], shape3[0]), seed, amp=amp)).astype(np.float64)


# --------------------------------------------------------------------------
# per step
# --------------------------------------------------------------------------
@pytest.mark.parametrize("shape3", SHAPES)
def test_warp(B, h, shape3):
    I, v = _img(shape3, 1), _fld(shape3, 2, amp=4.0)
    got = host(B.dir_warp(h, dev(I), dev(v)))
    assert_close(got, O.warp(I, v))


@pytest.mark.parametrize("shape3", SHAPES)
def test_gradient(B, h, shape3):
    I = _img(shape3, 3)
    got = host(B.dir_gradient(h, dev(I)))
    assert_close(got, O.gradient(I))


@pytest.mark.parametrize("shape3", SHAPES)
@pytest.mark.parametrize("sigma,radius", [(1.0, 3), (1.5, 5), (0.8, 1), (2.0, 16), (1.0, 0)])
def test_smooth(B, h, shape3, sigma, radius):
    u = np.stack([_img(shape3, 4 + c) for c in range(3)])
    got = host(B.dir_smooth(h, dev(u), sigma, radius))
    R = radius if radius > 0 else O.default_radius(sigma)
    assert_close(got, O.smooth(u, sigma, R))
    one = host(B.dir_smooth(h, dev(u[0]), sigma, radius))
    assert_close(one, O.smooth(u[0], sigma, R))


@pytest.mark.parametrize("shape3", SHAPES)
def test_restrict(B, h, shape3):
    I = _img(shape3, 7)
    got = host(B.dir_restrict(h, dev(I)))
    assert_close(got, O.restrict(I))


@pytest.mark.parametrize("coarse,fine", [((6, 7, 9), (11, 13, 17)), ((3, 17, 33), (5, 33, 65)), ((1, 4, 35), (1, 7, 70)),
                                         ((8, 32, 32), (16, 64, 64))])
def test_prolong(B, h, coarse, fine):
    vc = _fld(coarse, 8)
    got = host(B.dir_prolong(h, dev(vc), fine))
    assert_close(got, O.prolong(vc, fine))


@pytest.mark.parametrize("shape3", [(11, 13, 17), (9, 33, 65), (3, 4, 530)])
@pytest.mark.parametrize("with_field", [True, False])
def test_similarity(B, h, shape3, with_field):
    """MSE and correlation coefficient of S and M(x - v): the definitions on the
    oracle's FP64 deformed image."""
    S, M = _img(shape3, 60), f32(_img(shape3, 61) + 0.5 * _img(shape3, 60)).astype(np.float64)
    v = _fld(shape3, 62, amp=3.0) if with_field else None
    mse, cc = B.dir_similarity(h, dev(S), dev(M), dev(v) if with_field else None)
    Im = O.warp(M, v) if with_field else M
    assert abs(mse - ((Im - S) ** 2).mean()) <= 1e-9 * ((Im - S) ** 2).mean()
    assert abs(cc - np.corrcoef(Im.ravel(), S.ravel())[0, 1]) <= 1e-9
    same_mse, same_cc = B.dir_similarity(h, dev(S), dev(S), None)
    assert same_mse == 0.0 and abs(same_cc - 1.0) <= 1e-12


def _pair(shape3, seed, amp=2.0):
    """Phantom-like static/moving images and a moderate field, FP32-exact."""
    nz, ny, nx = shape3
    ph = P.make_phantom((nx, ny, nz), seed=seed, max_u=amp)
    v = _fld(shape3, seed + 100, amp=amp)
    return f32(ph.static).astype(np.float64), f32(ph.moving).astype(np.float64), v


ALL = ["passive", "evolved", "active", "double", "inverse_consistent"]


@pytest.mark.parametrize("shape3", [(11, 13, 17), (9, 33, 65), (20, 40, 72)])
@pytest.mark.parametrize("variant", ALL)
@pytest.mark.parametrize("alpha", [1.0, 0.4, 2.0])
def test_force(B, h, shape3, variant, alpha):
    S, M, v = _pair(shape3, 11)
    u_gpu, sums_gpu = B.dir_force(h, variant, alpha, dev(S), dev(M), dev(v))
    u_ref, sums_ref = O.force(O.VARIANTS[variant], S, M, v, alpha=alpha)
    assert_close(host(u_gpu) - v, u_ref - v)
    for k in range(3):
        assert abs(sums_gpu[k] - sums_ref[k]) <= REL_TOL * abs(sums_ref[k]) + 1e-12


@pytest.mark.parametrize("shape3", [(1, 1, 1), (1, 1, 2), (2, 1, 1), (1, 2, 1)])
@pytest.mark.parametrize("variant", ALL)
def test_degenerate_volumes(B, h, shape3, variant):
    """One- and two-voxel volumes: every sample clamped onto the border, the
    trilinear gathers at the volume's first element and its last."""
    S, M = _img(shape3, 80), _img(shape3, 81)
    v = _fld(shape3, 82)
    u_gpu, sums_gpu = B.dir_force(h, variant, 1.0, dev(S), dev(M), dev(v))
    u_ref, sums_ref = O.force(O.VARIANTS[variant], S, M, v)
    assert_close(host(u_gpu) - v, u_ref - v)
    for k in range(3):
        assert abs(sums_gpu[k] - sums_ref[k]) <= REL_TOL * abs(sums_ref[k]) + 1e-12
    out, _ = B.dir_step(h, variant, 1.0, dev(S), dev(M), dev(v), 1.5, 5)
    # the update is often zero here (no gradient along a one-voxel axis), so
    # the error is taken relative to the field itself
    assert_close(host(out), O.smooth(u_ref, 1.5, 5))
    mse, _ = B.dir_similarity(h, dev(S), dev(M), dev(v))
    d = O.warp(M, v) - S
    assert abs(mse - float((d * d).mean())) <= 1e-9 * float((d * d).mean())


STEP_SHAPES = [(11, 13, 17), (9, 33, 65), (20, 40, 72), (7, 30, 129), (2, 3, 300), (1, 2, 257), (3, 4, 530), (1, 3, 1100)]


@pytest.mark.parametrize("shape3", STEP_SHAPES)
@pytest.mark.parametrize("variant", ALL)
@pytest.mark.parametrize("sigma,radius", [(1.0, 3), (1.5, 5)])
def test_step(B, h, shape3, variant, sigma, radius):
    """One iteration exactly as the registration runs it: G * (v + dr)."""
    S, M, v = _pair(shape3, 13)
    alpha = 0.4 if variant == "double" else 1.0
    out, sums_gpu = B.dir_step(h, variant, alpha, dev(S), dev(M), dev(v), sigma, radius)
    u_ref, sums_ref = O.force(O.VARIANTS[variant], S, M, v, alpha=alpha)
    ref = O.smooth(u_ref, sigma, radius)
    assert_close(host(out) - v, ref - v)
    for k in range(3):
        assert abs(sums_gpu[k] - sums_ref[k]) <= REL_TOL * abs(sums_ref[k]) + 1e-12


# (nz, ny, nx): force workgroups of two row steps (the stencil values carried
# from one step to the next) with a one-plane last z chunk, on 512-, 256- and
# three 512-voxel tiles (inner-halo points, which carry nothing)
CARRY_SHAPES = [(37, 200, 300), (61, 160, 130), (23, 64, 1030)]


@pytest.mark.parametrize("shape3", CARRY_SHAPES)
@pytest.mark.parametrize("variant,alpha", [("active", 1.0), ("double", 0.4), ("inverse_consistent", 1.0)])
def test_step_carried_stencils(B, h, shape3, variant, alpha):
    """One iteration of the forces whose z-stencil values a lane carries
    between row steps, against the oracle (field and sums)."""
    S, M, v = _pair(shape3, 15)
    out, sums_gpu = B.dir_step(h, variant, alpha, dev(S), dev(M), dev(v), 1.5, 5)
    u_ref, sums_ref = O.force(O.VARIANTS[variant], S, M, v, alpha=alpha)
    ref = O.smooth(u_ref, 1.5, 5)
    extra = None
    if variant == "inverse_consistent":
        extra = O.smooth(ic_force_rounding_bound(S, M, v, alpha), 1.5, 5)
    assert_close(host(out) - v, ref - v, extra=extra)
    for k in range(3):
        assert abs(sums_gpu[k] - sums_ref[k]) <= REL_TOL * abs(sums_ref[k]) + 1e-12


@pytest.mark.parametrize("shape3", [(3, 4, 5), (2, 3, 40), (1, 2, 257)])
@pytest.mark.parametrize("variant", ["passive", "inverse_consistent"])
def test_step_widest_radius(B, h, shape3, variant):
    """R = 16 (the largest): halos wider than short rows, and a one-voxel last tile."""
    S, M, v = _pair(shape3, 14)
    out, sums_gpu = B.dir_step(h, variant, 1.0, dev(S), dev(M), dev(v), 4.0, 16)
    u_ref, sums_ref = O.force(O.VARIANTS[variant], S, M, v, alpha=1.0)
    ref = O.smooth(u_ref, 4.0, 16)
    assert_close(host(out) - v, ref - v)
    for k in range(3):
        assert abs(sums_gpu[k] - sums_ref[k]) <= REL_TOL * abs(sums_ref[k]) + 1e-12


@pytest.mark.parametrize("variant", ALL)
@pytest.mark.parametrize("shape3", [(12, 30, 41), (5, 9, 300)])
def test_register_equals_iterated_step(B, h, variant, shape3):
    """A one-level registration is bitwise the iteration of dir_step from a zero
    field (and, for IC, its composition): the same kernels, launch
    configurations and reduction order inside and outside a registration."""
    S, M, _ = _pair(shape3, 70)
    alpha = 0.4 if variant == "double" else 1.0
    iters = 6
    f, _ = B.dir_register(h, dev(S), dev(M), B.make_params(variant, [iters], sigma=1.5, radius=5, alpha=alpha))
    v = torch.zeros((3,) + tuple(S.shape), dtype=torch.float32, device="cuda")
    for _ in range(iters):
        v, _ = B.dir_step(h, variant, alpha, dev(S), dev(M), v, 1.5, 5)
    if variant == "inverse_consistent":
        v = B.dir_compose(h, v)
    assert torch.equal(f, v)


@pytest.mark.parametrize("shape3", [(11, 13, 17), (9, 33, 65)])
@pytest.mark.parametrize("K", [0, 1, 10])
def test_compose(B, h, shape3, K):
    hf = _fld(shape3, 12, amp=0.8)
    got = host(B.dir_compose(h, dev(hf), K))
    assert_close(got, O.compose(hf, K))


# --------------------------------------------------------------------------
# full-size steps, in the launch configuration the benchmark times
# --------------------------------------------------------------------------
@pytest.fixture(scope="module")
def full_pair():
    nz, ny, nx = 100, 256, 256
    ph = P.make_phantom((nx, ny, nz), seed=2, max_u=15.0, spacing_mm=(1.1, 1.1, 2.5))
    v = f32(ph.field_g * 0.8).astype(np.float64)
    return f32(ph.static).astype(np.float64), f32(ph.moving).astype(np.float64), v


@pytest.mark.slow
def test_full_size_warp_smooth(B, h, full_pair):
    S, M, v = full_pair
    _say("full-size warp 256x256x100")
    assert_close(host(B.dir_warp(h, dev(M), dev(v))), O.warp(M, v))
    _say("full-size smooth 256x256x100 sigma 1.5 R 5")
    assert_close(host(B.dir_smooth(h, dev(v), 1.5, 5)), O.smooth(v, 1.5, 5))


@pytest.mark.slow
@pytest.mark.parametrize("variant", ALL)
def test_full_size_step(B, h, full_pair, variant):
    S, M, v = full_pair
    _say(f"full-size step {variant} 256x256x100 sigma 1.5 R 5")
    out, sums_gpu = B.dir_step(h, variant, 1.0, dev(S), dev(M), dev(v), 1.5, 5)
    u_ref, sums_ref = O.force(O.VARIANTS[variant], S, M, v)
    ref = O.smooth(u_ref, 1.5, 5)
    assert_close(host(out) - v, ref - v)
    for k in range(3):
        assert abs(sums_gpu[k] - sums_ref[k]) <= REL_TOL * abs(sums_ref[k])


@pytest.mark.slow
@pytest.mark.parametrize("variant", ALL)
def test_full_size_force(B, h, full_pair, variant):
    S, M, v = full_pair
    _say(f"full-size force {variant} 256x256x100")
    u_gpu, sums_gpu = B.dir_force(h, variant, 1.0, dev(S), dev(M), dev(v))
    u_ref, sums_ref = O.force(O.VARIANTS[variant], S, M, v)
    # the inverse-consistent force at this size has voxels where the FP32
    # storage of P alone moves it by 2.4e-4 of max|f| (measured on the CPU
    # with P and D rounded in FP64 arithmetic): those get their derived bound
    extra = ic_force_rounding_bound(S, M, v) if variant == "inverse_consistent" else None
    assert_close(host(u_gpu) - v, u_ref - v, extra=extra)
    for k in range(3):
        assert abs(sums_gpu[k] - sums_ref[k]) <= REL_TOL * abs(sums_ref[k])


# --------------------------------------------------------------------------
# whole registrations
# --------------------------------------------------------------------------
def test_small_config_passive_end_to_end(B, h):
    """64x64x32, passive, 1 level, 50 iterations, sigma 1, R 3."""
    ph = P.make_phantom(**P.CONFIG_SMALL)
    S, M = f32(ph.static).astype(np.float64), f32(ph.moving).astype(np.float64)
    params = B.make_params("passive", [50], sigma=1.0, radius=3)
    field, stats = B.dir_register(h, dev(S), dev(M), params)
    ref, hist, runs, rc = O.register(S, M, O.PASSIVE, [50], sigma=1.0, radius=3)
    got = host(field)
    d = rms_vox(got, ref)
    vt, _ = ph.ground_truth()
    err_gpu = float(np.sqrt(((got - vt) ** 2).sum(axis=0))[ph.body].mean())
    err_ref = float(np.sqrt(((ref - vt) ** 2).sum(axis=0))[ph.body].mean())
    _say(f"small passive: rms(gpu-oracle)={d:.2e} vox; mean GT error gpu {err_gpu:.4f} oracle {err_ref:.4f} vox")
    assert d <= RMS_TOL_VOX
    assert abs(err_gpu - err_ref) <= 0.01
    assert stats["iters_run"] == [50]
    hg = np.array(stats["history"])
    # the first iterations agree to FP32 accuracy; later ones drift apart by
    # the rounding envelope of the iteration (about 5e-3 voxel RMS here)
    assert np.allclose(hg[:5, :3], hist[:5, :3], rtol=1e-5, atol=1e-9)
    assert np.allclose(hg[:, :3], hist[:, :3], rtol=2e-2, atol=1e-9)


# Settings whose result moves by well under 0.01 voxel RMS when the inputs are
# perturbed at FP32 rounding level: GPU and oracle must agree to 0.01 voxel.
WELL_CONDITIONED = [("passive", 1.0), ("evolved", 1.0), ("active", 1.0), ("double", 1.0), ("active", 0.4),
                    ("double", 2.0), ("inverse_consistent", 1.0)]
# Settings where the oracle itself moves by 0.015-0.04 voxel RMS under such
# perturbations (alpha = 0.4 lets noise-driven steps of up to 1.25 voxels
# through): the GPU must lie inside that rounding envelope.
ILL_CONDITIONED = [("passive", 0.4), ("double", 0.4)]
ITERS_SMALL = [20, 10, 5]


@pytest.fixture(scope="module")
def multilevel_pair():
    nz, ny, nx = 27, 75, 90
    ph = P.make_phantom((nx, ny, nz), seed=21, max_u=5.0, spacing_mm=(1.1, 1.1, 2.5))
    return ph, f32(ph.static).astype(np.float64), f32(ph.moving).astype(np.float64)


@pytest.mark.parametrize("variant,alpha", WELL_CONDITIONED)
def test_multilevel_end_to_end(B, h, multilevel_pair, variant, alpha):
    """A reduced 3-level case with the full-size construction (ragged dims)."""
    ph, S, M = multilevel_pair
    params = B.make_params(variant, ITERS_SMALL, sigma=1.5, alpha=alpha)
    field, stats = B.dir_register(h, dev(S), dev(M), params)
    ref, hist, runs, rc = O.register(S, M, O.VARIANTS[variant], ITERS_SMALL, sigma=1.5, alpha=alpha)
    d = rms_vox(host(field), ref)
    _say(f"{variant} alpha={alpha}: rms(gpu-oracle)={d:.2e} vox")
    assert d <= RMS_TOL_VOX
    assert stats["iters_run"] == ITERS_SMALL
    # Coarse levels start from FP32-stored restricted images, whose rounding
    # (~3e-5 HU) reaches the force through voxels with a near-zero intensity
    # difference: the first sums agree to ~5e-5 rather than to 1e-7.
    hg = np.array(stats["history"])
    assert np.allclose(hg[:3, :3], hist[:3, :3], rtol=1e-3, atol=1e-9)


@pytest.mark.parametrize("variant,alpha", ILL_CONDITIONED)
def test_multilevel_within_rounding_envelope(B, h, multilevel_pair, variant, alpha):
    ph, S, M = multilevel_pair
    params = B.make_params(variant, ITERS_SMALL, sigma=1.5, alpha=alpha)
    got = host(B.dir_register(h, dev(S), dev(M), params)[0])
    ref, _, _, _ = O.register(S, M, O.VARIANTS[variant], ITERS_SMALL, sigma=1.5, alpha=alpha)
    rng = np.random.default_rng(99)
    Sp = S * (1 + rng.uniform(-6e-8, 6e-8, S.shape))
    Mp = M * (1 + rng.uniform(-6e-8, 6e-8, M.shape))
    pert, _, _, _ = O.register(Sp, Mp, O.VARIANTS[variant], ITERS_SMALL, sigma=1.5, alpha=alpha)
    env = rms_vox(pert, ref)
    d = rms_vox(got, ref)
    vt, _ = ph.ground_truth()
    e_gpu = float(np.sqrt(((got - vt) ** 2).sum(axis=0))[ph.body].mean())
    e_ref = float(np.sqrt(((ref - vt) ** 2).sum(axis=0))[ph.body].mean())
    _say(f"{variant} alpha={alpha}: rms(gpu-oracle)={d:.2e}, oracle envelope {env:.2e}, "
         f"GT error gpu {e_gpu:.4f} oracle {e_ref:.4f} vox")
    assert d <= max(RMS_TOL_VOX, 3.0 * env)
    assert abs(e_gpu - e_ref) <= 0.01


@pytest.mark.parametrize("variant", ALL)
def test_zero_update_when_images_match(B, h, variant):
    S = _img((9, 20, 33), 30)
    params = B.make_params(variant, [3, 4], sigma=1.0)
    field, stats = B.dir_register(h, dev(S), dev(S), params)
    assert torch.count_nonzero(field).item() == 0


def test_bitwise_reproducible(B, h):
    S, M, _ = _pair((12, 40, 48), 40)
    params = B.make_params("inverse_consistent", [6, 6], sigma=1.0)
    f1, s1 = B.dir_register(h, dev(S), dev(M), params)
    f2, s2 = B.dir_register(h, dev(S), dev(M), params)
    assert torch.equal(f1, f2)
    assert s1["history"] == s2["history"] or np.array_equal(np.array(s1["history"]), np.array(s2["history"]),
                                                            equal_nan=True)


def test_timing_per_level_and_unchanged_results(B, h):
    """Timed launches (dispatch-stamped events) give the same field, and the
    per-level counts follow the iteration schedule."""
    S, M, _ = _pair((12, 40, 48), 41)
    params = B.make_params("active", [6, 4], sigma=1.0)
    f0, _ = B.dir_register(h, dev(S), dev(M), params)
    B.dir_timing_enable(h, ["force", "smooth_yz", "warp", "restrict"])
    try:
        f1, _ = B.dir_register(h, dev(S), dev(M), params)
        reads = {k: (B.dir_timing_read(h, k), B.dir_timing_read(h, k, level=0), B.dir_timing_read(h, k, level=1))
                 for k in ("force", "smooth_yz", "warp", "restrict", "compose")}
    finally:
        B.dir_timing_enable(h, ())
    assert torch.equal(f0, f1)
    for k, counts in (("force", (10, 4, 6)), ("smooth_yz", (10, 4, 6)), ("warp", (10, 4, 6))):
        (ms, n), (ms0, n0), (ms1, n1) = reads[k]
        assert (n, n0, n1) == counts, k
        assert ms > 0 and ms0 > 0 and ms1 > 0 and abs(ms - ms0 - ms1) <= 1e-9 * max(ms, 1.0), k
    assert reads["restrict"][0][1] == 2 and reads["restrict"][2][1] == 2   # S and M into level 1
    assert reads["compose"][0] == (0.0, 0)                                   # not enabled
    with pytest.raises(B.DemonsError):
        B.dir_timing_read(h, "force", level=8)


def test_stopping_rule(B, h):
    t = (0.6, -0.4, 0.5)
    S, M = P.smooth_translation_pair((20, 20, 20), t, seed=4)
    S, M = f32(S).astype(np.float64), f32(M).astype(np.float64)
    eps = 2e-3
    params = B.make_params("passive", [80], sigma=1.0, radius=3, eps=eps)
    field, stats = B.dir_register(h, dev(S), dev(M), params)
    _, hist, runs, _ = O.register(S, M, O.PASSIVE, [80], sigma=1.0, radius=3, eps=eps)
    l = np.array([e[3] for e in stats["history"]])
    n = stats["iters_run"][0]
    assert 10 < n < 80 and len(l) == n
    assert l[n - 11] - l[n - 1] <= eps                    # the rule fired at the last iteration
    assert all(not (l[k - 10] - l[k] <= eps) for k in range(10, n - 1))
    assert abs(n - runs[0]) <= 1                          # FP32 vs FP64 may move the stall by one


def test_invalid_arguments(B, h):
    S = dev(_img((4, 5, 6), 50))
    out = torch.empty((3, 4, 5, 6), device="cuda")
    L = B.lib()
    p = B.make_params("passive", [2], sigma=1.0)
    import ctypes
    ptr = lambda t: ctypes.c_void_p(t.data_ptr())
    assert L.dir_register(h.ptr, ptr(S), ptr(S), 6, 5, 4, None, ctypes.byref(p), None, None) == B.DIR_EINVAL
    assert L.dir_register(h.ptr, ptr(S), ptr(S), 0, 5, 4, None, ctypes.byref(p), ptr(out), None) == B.DIR_EINVAL
    for field, value in (("alpha", 0.0), ("sigma", -1.0), ("levels", 0), ("levels", 9), ("variant", 7),
                         ("radius", 17), ("eps", -1.0), ("storage", 3), ("storage", -1), ("struct_size", 8)):
        q = B.make_params("passive", [2], sigma=1.0)
        setattr(q, field, value)
        assert L.dir_register(h.ptr, ptr(S), ptr(S), 6, 5, 4, None, ctypes.byref(q), ptr(out), None) == B.DIR_EINVAL
    q = B.make_params("passive", [2], sigma=1.0)
    q.iters[0] = -1
    assert L.dir_register(h.ptr, ptr(S), ptr(S), 6, 5, 4, None, ctypes.byref(q), ptr(out), None) == B.DIR_EINVAL
    bad = (ctypes.c_double * 3)(1.0, 0.0, 1.0)
    assert L.dir_register(h.ptr, ptr(S), ptr(S), 6, 5, 4, bad, ctypes.byref(p), ptr(out), None) == B.DIR_EINVAL
    with pytest.raises(B.DemonsError):
        B.dir_smooth(h, dev(np.zeros((3, 4, 5, 6))), 1.0, 17)
    big = 2 ** 31 // 3 // (1024 * 1024) + 1
    assert L.dir_warp(h.ptr, ptr(S), ptr(out), 1024, 1024, big, ptr(S)) == B.DIR_EINVAL


def test_nan_input_reports_numeric_error(B, h):
    S, M, _ = _pair((9, 20, 33), 41)
    M = M.copy()
    M[3, 4, 5] = np.nan
    params = B.make_params("passive", [3], sigma=1.0)
    with pytest.raises(B.DemonsError) as ei:
        B.dir_register(h, dev(S), dev(M), params)
    assert ei.value.code == B.DIR_ENUMERIC


@pytest.mark.parametrize("alpha,n_stop", [(1.0, 15), (0.4, 20)])
def test_stopping_rule_closed_form(B, h, alpha, n_stop):
    """The stopping rule and every history column on the decoupled ramp, whose
    relative norm l(n) has a closed form (a smoothing so narrow that its FP32
    taps are exactly 1 and 0): the level stops after iteration n_stop."""
    from closed_forms import decoupled_ramp, decoupled_ramp_history, stop_eps
    nx, ny, nz, t, cap = 12, 3, 2, 0.75, 40
    S, M = decoupled_ramp(nx, ny, nz, t)
    expect = decoupled_ramp_history(nx, ny, nz, t, alpha, cap)
    eps = stop_eps(expect[:, 3], n_stop)
    params = B.make_params("passive", [cap], sigma=0.05, radius=1, alpha=alpha, eps=eps)
    _, stats = B.dir_register(h, dev(S), dev(M), params)
    assert stats["iters_run"] == [n_stop + 1]
    hg = np.array(stats["history"])
    np.testing.assert_allclose(hg[:, :3], expect[:n_stop + 1, :3], rtol=1e-5, atol=0)
    np.testing.assert_allclose(hg[1:, 3], expect[1:n_stop + 1, 3], rtol=1e-5)
