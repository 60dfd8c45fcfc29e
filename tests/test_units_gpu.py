"""Physical units (DIR_UNITS_MM) and image pre-smoothing (image_sigma) of the
HIP path against the FP64 oracle, through the C ABI.

The oracle writes the physical mode in millimetres (field, gradients, norms)
while the kernels run it on the voxel grid with a metric; both must give the
same registration.  One iteration from a zero field is held to the per-step
bound (normwise 1e-5 on the field, 1e-5 on the FP64 sums of the history),
a few iterations on a nonzero field to the same bound on the increment, and
whole multi-level registrations to the end-to-end bound (RMS 0.01 voxel).
"""
import sys

import numpy as np
import pytest
import torch

import oracle as O
from paper_0909_0928_amd import phantom as P

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

REL_TOL = 1e-5
RMS_TOL_VOX = 0.01
ALL = ["passive", "evolved", "active", "double", "inverse_consistent"]
SPACING = (1.1, 1.1, 2.5)      # x, y, z voxel sizes of the paper's CT (Table 1)


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


def f64(a):
    return np.asarray(a, np.float32).astype(np.float64)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, np.float32))).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def rel(a, b):
    nb = np.linalg.norm(b.ravel())
    return np.linalg.norm((a - b).ravel()) / (nb if nb > 0 else 1.0)


def rms_vox(a, b):
    return float(np.sqrt(((a - b) ** 2).sum(axis=0).mean()))


@pytest.fixture(scope="module")
def pair():
    ph = P.make_phantom((45, 38, 21), seed=41, max_u=3.0, spacing_mm=SPACING)
    return ph, f64(ph.static), f64(ph.moving)


def _both(B, h, S, M, variant, iters, sigma, alpha=1.0, units="mm", spacing=SPACING, image_sigma=0.0,
          storage="f32"):
    params = B.make_params(variant, iters, sigma=sigma, alpha=alpha, units=units, image_sigma=image_sigma,
                           storage=storage)
    field, stats = B.dir_register(h, dev(S), dev(M), params, spacing_mm=spacing)
    ref, hist, runs, rc = O.register(S, M, O.VARIANTS[variant], iters, sigma=sigma, alpha=alpha, spacing=spacing,
                                     physical=(units == "mm"), image_sigma=image_sigma)
    assert stats["iters_run"] == list(iters) == runs
    return host(field), np.array(stats["history"]), ref, hist


@pytest.mark.parametrize("variant", ALL)
def test_mm_first_iteration(B, h, pair, variant):
    """One iteration from a zero field: anisotropic Gaussian (sigma 1.5 mm is
    1.36 voxels in x and y and 0.6 in z, radii 5, 5, 2), metric force and the
    mm norms of the sums."""
    _, S, M = pair
    alpha = 0.4 if variant == "double" else 1.0
    got, hg, ref, hist = _both(B, h, S, M, variant, [1], 1.5, alpha=alpha)
    r = rel(got, ref)
    _say(f"mm first iteration {variant}: normwise {r:.2e}")
    assert r < REL_TOL
    assert float(np.abs(got - ref).max()) <= 10 * REL_TOL * float(np.abs(ref).max())
    assert np.allclose(hg[0, :3], hist[0, :3], rtol=REL_TOL, atol=0)


@pytest.mark.parametrize("variant", ALL)
def test_mm_iterations_on_a_nonzero_field(B, h, pair, variant):
    """Three iterations: from the second on the field is nonzero, so the
    warp, the deformed-image gradients and |v| in mm are all exercised."""
    _, S, M = pair
    got, hg, ref, hist = _both(B, h, S, M, variant, [3], 1.5)
    r = rel(got, ref)
    _say(f"mm three iterations {variant}: normwise {r:.2e}")
    assert r < 3 * REL_TOL
    assert np.allclose(hg[:, :3], hist[:, :3], rtol=3 * REL_TOL, atol=0)
    assert np.all(hg[1:, 1] > 0)


@pytest.mark.parametrize("variant", ALL)
def test_mm_multilevel_end_to_end(B, h, pair, variant):
    """Three levels (voxels 1.1 x 1.1 x 2.5 mm, then twice and four times
    that), field carried between levels as a length."""
    ph, S, M = pair
    got, hg, ref, hist = _both(B, h, S, M, variant, [10, 6, 4], 2.0)
    d = rms_vox(got, ref)
    _say(f"mm 3-level {variant}: rms(gpu-oracle)={d:.2e} vox")
    assert d <= RMS_TOL_VOX
    assert np.allclose(hg[:3, :3], hist[:3, :3], rtol=1e-3, atol=1e-9)


WIDE = [(100, 40, 8), (200, 36, 6), (300, 32, 6)]  # force tiles 128, 256 and 512 voxels wide


@pytest.mark.parametrize("shape", WIDE)
@pytest.mark.parametrize("variant", ["passive", "active", "inverse_consistent"])
@pytest.mark.parametrize("units,sigma", [("mm", 1.5), ("voxels", 2.0)])
def test_wide_rows_runtime_radius(B, h, variant, shape, units, sigma):
    """The force kernels that take the smoothing radius at run time (every
    physical-units registration; sigma 2 voxels, radius 6, in voxel units) on
    rows wider than the other tests reach: tiles of 128, 256 and 512 voxels
    (two per thread), three iterations against the oracle."""
    ph = P.make_phantom(shape, seed=43, max_u=2.5, spacing_mm=SPACING)
    S, M = f64(ph.static), f64(ph.moving)
    got, hg, ref, hist = _both(B, h, S, M, variant, [3], sigma, units=units)
    r = rel(got, ref)
    _say(f"wide rows {shape} {variant} {units}: normwise {r:.2e}")
    assert r < 3 * REL_TOL
    assert float(np.abs(got - ref).max()) <= 30 * REL_TOL * float(np.abs(ref).max())
    assert np.allclose(hg[:, :3], hist[:, :3], rtol=3 * REL_TOL, atol=0)


def test_mm_unit_spacing_equals_voxel_units(B, h, pair):
    """With 1 mm voxels both units give the same registration (to rounding:
    the physical kernels take the metric as arguments)."""
    _, S, M = pair
    p_vox = B.make_params("inverse_consistent", [5, 5], sigma=1.5)
    p_mm = B.make_params("inverse_consistent", [5, 5], sigma=1.5, units="mm")
    a = host(B.dir_register(h, dev(S), dev(M), p_vox, spacing_mm=(1.0, 1.0, 1.0))[0])
    b = host(B.dir_register(h, dev(S), dev(M), p_mm, spacing_mm=(1.0, 1.0, 1.0))[0])
    assert rel(b, a) < REL_TOL


def smoothing_envelope(S, M, variant, units, image_sigma, seed=1):
    """How far the oracle's first iteration moves when its pre-smoothed images
    carry the error an FP32 smoothing may make: each image value scaled by
    1 + U(-g, g) with g = 3 (2R + 1) 2^-24, the worst-case relative error of
    three passes of 2R + 1 non-negative FP32 taps (a sum of n products of one
    sign loses at most n unit roundoffs; rounding the result to FP32 adds half
    of one).  Where the images are smooth, D = M(x - v) - S cancels to a few
    HU against -1000, so the passive force amplifies this far more than the
    per-step bound assumes for identical inputs."""
    mm = units == "mm"
    hh = SPACING if mm else (1.0, 1.0, 1.0)
    si = [image_sigma / x for x in hh]
    ri = [int(np.ceil(3 * q)) for q in si]
    g = 3 * (2 * max(ri) + 1) * 2.0 ** -24
    rng = np.random.default_rng(seed)
    Ss = O.smooth3(S, si, ri) * (1 + rng.uniform(-g, g, S.shape))
    Ms = O.smooth3(M, si, ri) * (1 + rng.uniform(-g, g, M.shape))
    ref = O.register(S, M, O.VARIANTS[variant], [1], sigma=1.5, spacing=SPACING, physical=mm,
                     image_sigma=image_sigma)[0]
    pert = O.register(Ss, Ms, O.VARIANTS[variant], [1], sigma=1.5, spacing=SPACING, physical=mm)[0]
    return rel(pert, ref)


@pytest.mark.parametrize("variant", ["passive", "active", "inverse_consistent"])
@pytest.mark.parametrize("units", ["voxels", "mm"])
def test_presmoothing_first_iteration(B, h, pair, variant, units):
    """image_sigma 1.2 (voxels, or mm: 1.09 voxels in x and y, 0.48 in z)
    smooths S and M before the first iteration.  The kernels store the
    smoothed images in FP32, so the force no longer sees the oracle's inputs:
    the bound is the oracle's own movement under the smoothing's FP32 error
    (1.6e-4 to 2.3e-4 for active and inverse-consistent, 1.4e-3 to 4.5e-3
    for passive, whose force cancels most; the GPU measured 1e-5 to 1.4e-4).
    Measured on the CPU: smoothing z with the y taps moves the result by 0.27
    to 0.31, a radius one short by 2.8e-3 to 3.7e-3 (caught by the active and
    inverse-consistent cases), M left unsmoothed by 0.6."""
    _, S, M = pair
    got, hg, ref, hist = _both(B, h, S, M, variant, [1], 1.5, units=units, image_sigma=1.2)
    r = rel(got, ref)
    env = smoothing_envelope(S, M, variant, units, 1.2)
    _say(f"pre-smoothed first iteration {variant} {units}: normwise {r:.2e}, smoothing envelope {env:.2e}")
    assert r <= max(REL_TOL, env)
    assert abs(hg[0, 2] - hist[0, 2]) <= 1e-3 * hist[0, 2]


@pytest.mark.parametrize("variant", ["passive", "double", "inverse_consistent"])
@pytest.mark.parametrize("units", ["voxels", "mm"])
def test_presmoothing_multilevel_end_to_end(B, h, pair, variant, units):
    """Every level's images smoothed, each restricted from the unsmoothed
    finer level."""
    _, S, M = pair
    got, hg, ref, hist = _both(B, h, S, M, variant, [8, 5, 3], 1.5, units=units, image_sigma=1.0)
    d = rms_vox(got, ref)
    _say(f"pre-smoothed 3-level {variant} {units}: rms(gpu-oracle)={d:.2e} vox")
    assert d <= RMS_TOL_VOX
    # smoothing changes the images: the run differs from the unsmoothed one
    plain = O.register(S, M, O.VARIANTS[variant], [8, 5, 3], sigma=1.5, spacing=SPACING,
                       physical=(units == "mm"))[0]
    assert rms_vox(ref, plain) > 10 * max(d, 1e-6)


@pytest.mark.parametrize("storage", ["f16", "bf16"])
def test_mm_presmoothing_16bit_storage(B, h, pair, storage):
    """Physical units and pre-smoothing with 16-bit storage: against the
    oracle on the same rounded images, over the body, to the storage study's
    bounds (0.02 voxel F16, 0.1 BF16)."""
    ph, S, M = pair
    rnd = (lambda a: torch.from_numpy(np.asarray(a, np.float32)).to(
        torch.float16 if storage == "f16" else torch.bfloat16).float().numpy().astype(np.float64))
    Sr, Mr = rnd(S), rnd(M)
    got, _, ref, _ = _both(B, h, Sr, Mr, "passive", [8, 5, 3], 1.5, image_sigma=1.0, storage=storage)
    d = float(np.sqrt(((got - ref) ** 2).sum(axis=0))[ph.body].mean())
    _say(f"mm pre-smoothed {storage}: body mean |gpu-oracle| {d:.2e} vox")
    assert d <= (0.02 if storage == "f16" else 0.1)


def test_mm_batch_equals_alone(B, h):
    """A lockstep batch of registrations in mm (shared spacing, mixed variants
    and sizes, one shared image) gives each field bitwise as alone."""
    shapes = [(40, 33, 18), (40, 33, 18), (31, 26, 15)]
    phs = [P.make_phantom(s, seed=50 + i, max_u=2.5, spacing_mm=SPACING) for i, s in enumerate(shapes)]
    S = [dev(f64(p.static)) for p in phs]
    M = [dev(f64(p.moving)) for p in phs]
    S[1] = S[0]                      # shared static image: one pyramid, one pre-smoothing
    variants = ["passive", "inverse_consistent", "double"]
    params = [B.make_params(v, [4, 3], sigma=1.5, units="mm", image_sigma=1.0) for v in variants]
    res = B.dir_register_batch(h, S, M, params, spacing_mm=[SPACING] * 3)
    for r in range(3):
        alone, st = B.dir_register(h, S[r], M[r], params[r], spacing_mm=SPACING)
        assert torch.equal(res[r][0], alone), variants[r]
        assert np.array_equal(np.array(res[r][1]["history"]), np.array(st["history"]), equal_nan=True)


def test_mm_invalid_arguments(B, h, pair):
    _, S, M = pair
    Sd, Md = dev(S), dev(M)
    p = B.make_params("passive", [2], sigma=1.5, units="mm")
    with pytest.raises(B.DemonsError) as e:
        B.dir_register(h, Sd, Md, p)                          # mm without spacing
    assert e.value.code == B.DIR_EINVAL
    p_wide = B.make_params("passive", [2], sigma=10.0, units="mm")  # 20 voxels at 0.5 mm: radius 60
    with pytest.raises(B.DemonsError):
        B.dir_register(h, Sd, Md, p_wide, spacing_mm=(0.5, 0.5, 0.5))
    with pytest.raises(B.DemonsError):
        B.dir_register(h, Sd, Md, B.make_params("passive", [2], sigma=1.5, image_sigma=-1.0))
    with pytest.raises(B.DemonsError):
        B.dir_register(h, Sd, Md, B.make_params("passive", [2], sigma=1.5, units=7))
    # a batch in mm needs one spacing
    with pytest.raises(B.DemonsError):
        B.dir_register_batch(h, [Sd, Sd], [Md, Md], [p, p], spacing_mm=[SPACING, (1.0, 1.0, 2.5)])


@pytest.mark.parametrize("variant", ["passive", "inverse_consistent"])
def test_mm_stopping_rule_matches_oracle(B, h, pair, variant):
    """The stopping rule on the mm norms: with eps set from the oracle's own
    relative-norm history, the GPU stops each level where the oracle does."""
    _, S, M = pair
    iters = [30, 30]
    _, hist, _, _ = O.register(S, M, O.VARIANTS[variant], iters, sigma=1.5, spacing=SPACING, physical=True)
    l = hist[iters[0]:, 3]                                  # finest level, l(n)
    drops = l[:-10] - l[10:]                                # l(n - 10) - l(n), n >= 10
    eps = float(np.sort(drops[np.isfinite(drops)])[len(drops) // 3]) * 1.0001
    params = B.make_params(variant, iters, sigma=1.5, units="mm", eps=eps)
    field, stats = B.dir_register(h, dev(S), dev(M), params, spacing_mm=SPACING)
    ref, hist_ref, runs, _ = O.register(S, M, O.VARIANTS[variant], iters, sigma=1.5, spacing=SPACING,
                                        physical=True, eps=eps)
    _say(f"mm stopping rule {variant}: eps {eps:.3e}, GPU runs {stats['iters_run']}, oracle {runs}")
    assert runs[1] < iters[1]                               # the rule fires on the finest level
    assert all(abs(a - b) <= 1 for a, b in zip(stats["iters_run"], runs))
    # the sums agree closely at the start; over 30 coarse iterations the
    # passive sums drift (the FP32 images' rounding reaches the force where D
    # is small), the mean D^2 stays close
    hg = np.array(stats["history"])
    n = min(len(hg), len(hist_ref))
    assert np.allclose(hg[:3, :3], hist_ref[:3, :3], rtol=1e-3, atol=1e-9)
    assert np.allclose(hg[:n, 2], hist_ref[:n, 2], rtol=1e-2, atol=0)


def test_mm_requests_batch_in_the_pool(B):
    """A pool with a batch limit admits compatible mm requests together (same
    spacing) and keeps requests with another spacing apart; every result is
    bitwise the lone registration's."""
    reqs = [((40, 33, 18), SPACING), ((31, 26, 15), SPACING), ((36, 30, 16), (1.0, 1.0, 2.0)),
            ((40, 33, 18), SPACING)]
    ins, alone = [], []
    hh = B.dir_create(0)
    try:
        for k, (shape, sp) in enumerate(reqs):
            ph = P.make_phantom(shape, seed=70 + k, max_u=2.5, spacing_mm=SPACING)
            Sd, Md = dev(f64(ph.static)), dev(f64(ph.moving))
            p = B.make_params(["passive", "inverse_consistent", "double", "active"][k], [4, 3], sigma=1.5,
                              units="mm", image_sigma=0.8)
            f, _ = B.dir_register(hh, Sd, Md, p, spacing_mm=sp)
            ins.append((Sd, Md, p, sp))
            alone.append(f.clone())
    finally:
        B.dir_destroy(hh)
    with B.Pool(slots=1, max_batch=4) as pool:
        Sb = dev(f64(P.make_phantom((160, 160, 80), seed=79, max_u=2.5).static))
        blocker = pool.submit(Sb, Sb.flip(0).contiguous(), B.make_params("passive", [30, 20], sigma=1.0))
        tickets = [pool.submit(S, M, p, spacing_mm=sp) for S, M, p, sp in ins]
        got = {t: pool.wait(t) for t in tickets}
        pool.wait(blocker)
    for k, t in enumerate(tickets):
        assert torch.equal(got[t][0], alone[k]), reqs[k]
