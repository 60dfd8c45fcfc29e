"""Lockstep batches (dir_register_batch): several registrations, of one size or
of several, run every iteration as one pre-warp, one force and one smoothing
launch (per tile class).
Each field, its iteration counts and its per-iteration history must be bitwise
those of the same registration run alone with dir_register (the kernels, their
arithmetic and the order of every sum are the same), and the batch must refuse
registrations that cannot run in lockstep."""
import ctypes

import numpy as np
import pytest
import torch

from paper_0909_0928_amd import phantom as P

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]


@pytest.fixture(scope="module")
def B():
    from paper_0909_0928_amd import binding
    return binding


@pytest.fixture(scope="module")
def h(B):
    hh = B.dir_create(0)
    yield hh
    B.dir_destroy(hh)


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, dtype=np.float32))).cuda()


def _pairs(shape, count, seed):
    out = []
    for k in range(count):
        ph = P.make_phantom(shape, seed=seed + k, max_u=2.5)
        out.append((_dev(ph.static), _dev(ph.moving)))
    return out


# the six force settings of the benchmark: every kind of pre-warp and a mixed force launch
SIX = [("passive", 1.0), ("active", 1.0), ("double", 1.0), ("passive", 0.4), ("inverse_consistent", 1.0),
       ("double", 0.4)]


def _alone(B, h, pairs, params):
    res = []
    for (S, M), p in zip(pairs, params):
        f, st = B.dir_register(h, S, M, p)
        res.append((f.clone(), st))
    return res


def _check_equal(batch, alone):
    for k, ((fb, sb), (fa, sa)) in enumerate(zip(batch, alone)):
        assert torch.equal(fb, fa), k
        assert sb["iters_run"] == sa["iters_run"], k
        # every FP64 sum bitwise (the relative norm is NaN while the field is zero)
        assert np.array_equal(np.array(sb["history"]), np.array(sa["history"]), equal_nan=True), k
        assert np.array_equal([sb["mse_final"], sb["relnorm_final"]], [sa["mse_final"], sa["relnorm_final"]],
                              equal_nan=True), k


# (shape xyz, iterations coarse to fine, storage): several force tiles, ragged edges in x, y and z
CASES = [((67, 45, 19), [6, 5, 4], "f32"),
         ((48, 40, 12), [5, 3], "f32"),
         ((130, 33, 21), [4, 3], "f32"),
         ((40, 36, 20), [5, 4], "f16"),
         ((36, 28, 14), [4, 4], "bf16")]


@pytest.mark.parametrize("shape,iters,storage", CASES)
def test_mixed_batch_equals_alone(B, h, shape, iters, storage):
    pairs = _pairs(shape, len(SIX), 700)
    params = [B.make_params(v, iters, sigma=1.0, alpha=a, storage=storage) for v, a in SIX]
    alone = _alone(B, h, pairs, params)
    for _ in range(2):  # the second call reuses the batch workspace
        batch = B.dir_register_batch(h, [S for S, _ in pairs], [M for _, M in pairs], params)
        _check_equal(batch, alone)


@pytest.mark.parametrize("variant", ["passive", "evolved", "active", "double", "inverse_consistent"])
def test_uniform_batch_equals_alone(B, h, variant):
    pairs = _pairs((45, 38, 17), 3, 750)
    params = [B.make_params(variant, [5, 4], sigma=1.5, alpha=a) for a in (1.0, 0.7, 0.4)]
    _check_equal(B.dir_register_batch(h, [S for S, _ in pairs], [M for _, M in pairs], params),
                 _alone(B, h, pairs, params))


def test_batch_of_one_and_of_the_limit(B, h):
    pairs = _pairs((33, 30, 11), B.DIR_MAX_BATCH, 780)
    params = [B.make_params(SIX[k % len(SIX)][0], [4, 3], sigma=1.0, alpha=SIX[k % len(SIX)][1])
              for k in range(B.DIR_MAX_BATCH)]
    alone = _alone(B, h, pairs, params)
    _check_equal(B.dir_register_batch(h, [pairs[0][0]], [pairs[0][1]], params[:1]), alone[:1])
    _check_equal(B.dir_register_batch(h, [S for S, _ in pairs], [M for _, M in pairs], params), alone)


# sizes that take every force tile width (64, 128, 256, 512 voxels) and
# different z-chunk depths of the smoothing
RAGGED = [(40, 36, 20), (100, 33, 17), (130, 45, 21), (300, 20, 9), (64, 64, 40), (257, 30, 12)]


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_ragged_batch_equals_alone(B, h, storage):
    pairs = []
    for k, shape in enumerate(RAGGED):
        pairs += _pairs(shape, 1, 860 + k)
    params = [B.make_params(v, [5, 4, 3], sigma=1.0, alpha=a, storage=storage) for v, a in SIX]
    alone = _alone(B, h, pairs, params)
    for _ in range(2):
        _check_equal(B.dir_register_batch(h, [S for S, _ in pairs], [M for _, M in pairs], params), alone)


def test_ragged_batch_of_uneven_ic_pairs(B, h):
    # the uneven inverse-consistent workload's shape mix, scaled down: x, y in
    # 64..128, z in 32..64, three levels
    rng = np.random.default_rng(11)
    shapes = [(int(rng.integers(64, 129)), int(rng.integers(64, 129)), int(rng.integers(32, 65))) for _ in range(8)]
    pairs = []
    for k, shape in enumerate(shapes):
        pairs += _pairs(shape, 1, 880 + k)
    params = [B.make_params("inverse_consistent", [6, 4, 3], sigma=1.5)] * len(shapes)
    alone = _alone(B, h, pairs, params)
    _check_equal(B.dir_register_batch(h, [S for S, _ in pairs], [M for _, M in pairs], params), alone)


def test_batch_stopping_rule_per_registration(B, h):
    # eps differs per registration: the stopped ones skip their remaining
    # iterations inside the batch, as a lone registration stops early
    pairs = _pairs((40, 32, 16), 4, 800)
    eps = [0.0, 1e-3, 1e-4, 0.5]
    params = [B.make_params("passive", [30, 25], sigma=1.0, eps=e) for e in eps]
    alone = _alone(B, h, pairs, params)
    assert any(st["iters_run"] != [30, 25] for _, st in alone)  # the rule fired somewhere
    _check_equal(B.dir_register_batch(h, [S for S, _ in pairs], [M for _, M in pairs], params), alone)


def test_batch_same_inputs_for_every_setting(B, h):
    # the benchmark's form: one pair registered under six settings
    (S, M), = _pairs((64, 48, 24), 1, 820)
    params = [B.make_params(v, [6, 4, 3], sigma=1.5, alpha=a) for v, a in SIX]
    alone = _alone(B, h, [(S, M)] * len(SIX), params)
    _check_equal(B.dir_register_batch(h, [S] * len(SIX), [M] * len(SIX), params), alone)


def test_batch_refuses_what_cannot_run_in_lockstep(B, h):
    pairs = _pairs((32, 24, 10), 2, 840)
    Ss, Ms = [S for S, _ in pairs], [M for _, M in pairs]
    p0 = B.make_params("passive", [4, 3], sigma=1.0)
    bad = [B.make_params("passive", [4, 2], sigma=1.0),             # other iterations
           B.make_params("passive", [4, 3], sigma=1.5),             # other sigma
           B.make_params("passive", [7], sigma=1.0),                # other levels
           B.make_params("passive", [4, 3], sigma=1.0, storage="f16")]
    for p1 in bad:
        with pytest.raises(B.DemonsError) as e:
            B.dir_register_batch(h, Ss, Ms, [p0, p1])
        assert e.value.code == B.DIR_EINVAL
    shared = torch.empty((3,) + tuple(Ss[0].shape), device="cuda")
    with pytest.raises(B.DemonsError) as e:                         # one output field for both
        B.dir_register_batch(h, Ss, Ms, [p0, p0], field_outs=[shared, shared])
    assert e.value.code == B.DIR_EINVAL
    # more than the batch limit, through the C ABI directly
    n = B.DIR_MAX_BATCH + 1
    arr = (ctypes.c_void_p * n)(*([Ss[0].data_ptr()] * n))
    outs = [torch.empty_like(shared) for _ in range(n)]
    parr = (B.dir_params * n)(*([p0] * n))
    dims = (ctypes.c_int32 * (3 * n))(*([32, 24, 10] * n))
    rc = B.lib().dir_register_batch(h.ptr, n, arr, arr, dims, None, parr,
                                    (ctypes.c_void_p * n)(*[o.data_ptr() for o in outs]), None)
    assert rc == B.DIR_EINVAL
    # the handle still works
    f, _ = B.dir_register(h, Ss[0], Ms[0], p0)
    assert torch.isfinite(f).all()


def test_batch_at_the_benchmark_size(B, h):
    # 256 x 256 x 100 with its three levels, in the launch configuration the
    # benchmark times: the six settings in one batch against each alone
    ph = P.make_phantom((256, 256, 100), seed=2, max_u=15.0)  # the benchmark's pair
    S, M = _dev(ph.static), _dev(ph.moving)
    params = [B.make_params(v, [100, 50, 25], sigma=1.5, alpha=a) for v, a in SIX]
    alone = _alone(B, h, [(S, M)] * len(SIX), params)
    _check_equal(B.dir_register_batch(h, [S] * len(SIX), [M] * len(SIX), params), alone)


def test_async_batch_equals_alone(B):
    # dir_register_batch_async on a handle with its own stream, collected by dir_wait
    pairs = _pairs((50, 42, 18), 3, 900)
    params = [B.make_params(v, [5, 4], sigma=1.0, alpha=a) for v, a in SIX[:3]]
    hs = B.dir_create(0, stream=torch.cuda.Stream())
    try:
        alone = _alone(B, hs, pairs, params)
        outs = B.dir_register_batch_async(hs, [S for S, _ in pairs], [M for _, M in pairs], params)
        with pytest.raises(B.DemonsError) as e:  # the handle is busy until dir_wait
            B.dir_register(hs, pairs[0][0], pairs[0][1], params[0])
        assert e.value.code == B.DIR_EBUSY
        res = B.dir_wait(hs)
        assert [f.data_ptr() for f, _ in res] == [o.data_ptr() for o in outs]
        _check_equal(res, alone)
    finally:
        B.dir_destroy(hs)


def test_non_finite_input_is_reported_per_registration(B, h):
    # a NaN voxel in one moving image makes that registration's sums
    # non-finite (DIR_ENUMERIC); the others of its batch are unaffected
    pairs = _pairs((36, 30, 14), 3, 920)
    bad = pairs[1][1].clone()
    bad[7, 11, 13] = float("nan")
    pairs[1] = (pairs[1][0], bad)
    params = [B.make_params(v, [4, 3], sigma=1.0, alpha=a) for v, a in SIX[:3]]
    with pytest.raises(B.DemonsError) as e:
        B.dir_register(h, pairs[1][0], pairs[1][1], params[1])
    assert e.value.code == B.DIR_ENUMERIC
    good = _alone(B, h, [pairs[0], pairs[2]], [params[0], params[2]])
    with pytest.raises(B.DemonsError) as e:
        B.dir_register_batch(h, [S for S, _ in pairs], [M for _, M in pairs], params)
    assert e.value.code == B.DIR_ENUMERIC
    # through a batching pool each ticket carries its own status
    (Sb, Mb), = _pairs((160, 160, 80), 1, 930)
    with B.Pool(slots=1, max_batch=3) as pool:
        # a long registration occupies the only slot, so the next three queue and are admitted together
        blocker = pool.submit(Sb, Mb, B.make_params("passive", [30, 20], sigma=1.0))
        tickets = [pool.submit(S, M, p) for (S, M), p in zip(pairs, params)]
        pool.wait(blocker)
        f0, _ = pool.wait(tickets[0])
        with pytest.raises(B.DemonsError) as e:
            pool.wait(tickets[1])
        assert e.value.code == B.DIR_ENUMERIC
        f2, _ = pool.wait(tickets[2])
        assert pool.stats()["peak_running"] == 3
    assert torch.equal(f0, good[0][0]) and torch.equal(f2, good[1][0])
    f, _ = B.dir_register(h, pairs[0][0], pairs[0][1], params[0])  # the handle still works
    assert torch.equal(f, good[0][0])


@pytest.mark.parametrize("storage,shapes,iters", [
    # FP32: each 82 MB level fits the cache three at a time, the four together do not
    ("f32", [(160, 160, 100), (150, 170, 96), (160, 160, 100), (144, 160, 104)], [4, 3, 2]),
    # the same with one level: no level in lockstep at all
    ("f32", [(160, 160, 100), (150, 170, 96), (160, 160, 100), (144, 160, 104)], [3]),
    # F16: each 105 MB level fits two at a time, the three together do not
    ("f16", [(256, 256, 100)] * 3, [4, 3, 2])])
def test_batch_levels_on_concurrent_streams(B, h, storage, shapes, iters):
    # the finest level does not run in lockstep; its registrations run on
    # several streams at once, and each result is still the lone one
    pairs = []
    for k, shape in enumerate(shapes):
        pairs += _pairs(shape, 1, 940 + k)
    params = [B.make_params(v, iters, sigma=1.5, alpha=a, storage=storage) for v, a in SIX[:len(shapes)]]
    alone = _alone(B, h, pairs, params)
    for _ in range(2):
        _check_equal(B.dir_register_batch(h, [S for S, _ in pairs], [M for _, M in pairs], params), alone)


def test_interleaved_lockstep_order_equals_alone(B, h):
    """Four FP32 registrations of 256x256x100 with different force variants
    and both pre-warp kinds: their 128x128x50 level runs in lockstep with at
    least 512 force and pre-warp workgroups per registration, so those
    launches take the order that interleaves the registrations over the XCDs;
    fields and every FP64 sum stay bitwise those of each registration alone."""
    pairs = _pairs((256, 256, 100), 2, 990)
    pairs = pairs + pairs
    names = [("passive", 1.0), ("inverse_consistent", 1.0), ("double", 0.4), ("active", 1.0)]
    params = [B.make_params(v, [4, 3, 1], sigma=1.5, alpha=a) for v, a in names]
    alone = _alone(B, h, pairs, params)
    _check_equal(B.dir_register_batch(h, [S for S, _ in pairs], [M for _, M in pairs], params), alone)


def test_batch_timing_counts_launches_per_tile_class_and_lane(B):
    # per-kernel timing on a batch: one force launch per tile class and
    # iteration on the lockstep level, one per registration and iteration on
    # the level run on concurrent streams; fields unchanged by the timing
    shapes = [(160, 160, 100), (100, 150, 96), (160, 160, 100), (150, 170, 96)]  # tile widths 256, 128, 256, 256
    pairs = []
    for k, shape in enumerate(shapes):
        pairs += _pairs(shape, 1, 960 + k)
    params = [B.make_params(v, [3, 2], sigma=1.0, alpha=a) for v, a in SIX[:4]]
    hs = B.dir_create(0, stream=torch.cuda.Stream())
    try:
        ref = B.dir_register_batch(hs, [S for S, _ in pairs], [M for _, M in pairs], params)
        ref = [(f.clone(), st) for f, st in ref]
        B.dir_timing_enable(hs, ["force", "smooth_yz", "restrict"])
        got = B.dir_register_batch(hs, [S for S, _ in pairs], [M for _, M in pairs], params)
        reads = {k: (B.dir_timing_read(hs, k, level=0), B.dir_timing_read(hs, k, level=1))
                 for k in ("force", "smooth_yz", "restrict")}
        B.dir_timing_enable(hs, ())
    finally:
        B.dir_destroy(hs)
    _check_equal(got, ref)
    # level 1 (80x80x50 and smaller, lockstep): x tiles of 128 for nx = 80 and of 64 for nx = 50: two force
    # launches per iteration; one smoothing launch (one z-chunk depth); level 0: 4 registrations x 2 iterations
    (ms0, n0), (ms1, n1) = reads["force"]
    assert n1 == 3 * 2 and n0 == 4 * 2 and ms0 > 0 and ms1 > 0
    (ys0, m0), (ys1, m1) = reads["smooth_yz"]
    assert m0 == 4 * 2 and m1 >= 3 and ys0 > 0
    assert reads["restrict"][1][1] == 2 * 4  # S and M of four registrations into level 1


def test_autotuned_smoothing_depth_leaves_results_unchanged(B, h):
    # the tuned z-chunk depth changes only which workgroup computes which
    # output: fields and histories are bitwise those of the fixed rule
    pairs = _pairs((96, 80, 40), 1, 980) * 6
    params = [B.make_params(v, [5, 4, 3], sigma=1.5, alpha=a) for v, a in SIX]
    B.dir_autotune_clear()
    try:
        before = B.dir_register_batch(h, [S for S, _ in pairs], [M for _, M in pairs], params)
        before = [(f.clone(), st) for f, st in before]
        alone = _alone(B, h, pairs[:1], params[:1])
        depths6 = B.dir_autotune(h, pairs[0][0].shape, params[0], count=6)
        depths1 = B.dir_autotune(h, pairs[0][0].shape, params[0], count=1)
        assert len(depths6) == 3 and all(d in (2, 4, 8) for d in depths6 + depths1)
        _check_equal(B.dir_register_batch(h, [S for S, _ in pairs], [M for _, M in pairs], params), before)
        _check_equal(_alone(B, h, pairs[:1], params[:1]), alone)
    finally:
        B.dir_autotune_clear()


@pytest.mark.parametrize("storage,shapes,iters", [
    ("f32", [(48, 40, 20)] * 6, [4, 3, 2]),               # every level in lockstep
    ("f32", [(256, 256, 100)] * 2, [3, 2, 1]),            # finest level one registration at a time
    ("f32", [(160, 160, 100)] * 3, [3, 2]),               # finest level on three lanes (side streams captured)
    ("f16", [(256, 256, 100)] * 3 + [(200, 180, 90)], [2, 2, 1]),
])
def test_graph_captured_batch_replays_equal_eager(B, storage, shapes, iters):
    """dir_set_graphs on: a batch (lockstep levels, and levels on side-stream
    lanes) is captured on first use and replayed; every replay, with eager
    work and synchronisations in between, gives each field and history bitwise
    as the eager batch; a changed parameter is captured anew."""
    pairs = []
    for k, shape in enumerate(shapes):
        pairs += _pairs(shape, 1, 300 + k)
    names = [SIX[k % len(SIX)] for k in range(len(shapes))]
    params = [B.make_params(v, iters, sigma=1.5, alpha=a, storage=storage) for v, a in names]
    S = [p[0] for p in pairs]
    M = [p[1] for p in pairs]
    s = torch.cuda.Stream()
    hg = B.dir_create(0, stream=s)
    try:
        eager = [(f.clone(), st) for f, st in B.dir_register_batch(hg, S, M, params)]
        B.dir_set_graphs(hg, True)
        outs = [torch.empty_like(f) for f, _ in eager]
        for rep in range(3):
            for o in outs:
                o.fill_(float("nan"))
            torch.cuda.synchronize()
            res = B.dir_register_batch(hg, S, M, params, field_outs=outs)
            _check_equal(res, eager)
            B.dir_warp(hg, S[0], outs[0])           # eager work on the handle's stream between replays
            (S[0] * 2.0).sum().item()               # and on the default stream
        changed = list(params)
        changed[0] = B.make_params(names[0][0], iters, sigma=1.5, alpha=0.7, storage=storage)
        res = B.dir_register_batch(hg, S, M, changed, field_outs=outs)
        B.dir_set_graphs(hg, False)
        ref = B.dir_register_batch(hg, S, M, changed)
        _check_equal(res, ref)
    finally:
        B.dir_destroy(hg)
