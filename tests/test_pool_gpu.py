"""The request pool (dir_pool_*): registrations of uneven sizes admitted by
workspace budget onto a few streams.  Every result must be bitwise the result
of dir_register alone on the same inputs, the workspace held must never
exceed the budget, and requests must overlap when the budget allows it."""
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


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, dtype=np.float32))).cuda()


# (shape xyz, variant, alpha, iterations coarse to fine, storage)
REQUESTS = [((48, 40, 12), "passive", 1.0, [8, 6], "f32"),
            ((96, 80, 40), "inverse_consistent", 1.0, [6, 4, 3], "f32"),
            ((33, 29, 17), "active", 1.0, [5, 4], "f16"),
            ((64, 64, 32), "double", 0.4, [6, 6, 3], "f32"),
            ((27, 45, 9), "evolved", 1.0, [7], "bf16"),
            ((80, 64, 24), "passive", 0.4, [4, 4], "f32"),
            ((40, 40, 24), "inverse_consistent", 1.0, [6, 5], "f16"),
            ((72, 56, 20), "active", 1.0, [5, 5], "f32")]


@pytest.fixture(scope="module")
def inputs():
    out = []
    for k, (shape, *_rest) in enumerate(REQUESTS):
        ph = P.make_phantom(shape, seed=500 + k, max_u=2.5)
        out.append((_dev(ph.static), _dev(ph.moving)))
    return out


def _params(B, req):
    _, variant, alpha, iters, st = req
    return B.make_params(variant, iters, sigma=1.0, alpha=alpha, storage=st)


@pytest.fixture(scope="module")
def alone(B, inputs):
    h = B.dir_create(0)
    try:
        res = []
        for (S, M), req in zip(inputs, REQUESTS):
            f, st = B.dir_register(h, S, M, _params(B, req))
            res.append((f.clone(), st["iters_run"]))
        return res
    finally:
        B.dir_destroy(h)


@pytest.mark.parametrize("slots,budget_factor", [(3, 1.5), (4, 0.0), (1, 1.0)])
def test_pool_results_equal_alone_and_budget_holds(B, inputs, alone, slots, budget_factor):
    needs = [B.dir_workspace_bytes(tuple(S.shape), _params(B, req)) for (S, _), req in zip(inputs, REQUESTS)]
    budget = int(budget_factor * max(needs))  # 0: no limit
    with B.Pool(slots=slots, max_bytes=budget) as pool:
        tickets = [pool.submit(S, M, _params(B, req)) for (S, M), req in zip(inputs, REQUESTS)]
        got = {}
        while len(got) < len(tickets):               # collect in whatever order they finish
            for t in tickets:
                if t not in got:
                    r = pool.poll(t)
                    if r is not None:
                        got[t] = r
        st = pool.stats()
    for k, t in enumerate(tickets):
        f, stats = got[t]
        assert torch.equal(f, alone[k][0]), REQUESTS[k]
        assert stats["iters_run"] == alone[k][1]
    if budget:
        assert st["peak_bytes"] <= budget
    assert 1 <= st["peak_running"] <= slots
    if slots > 1:
        assert st["peak_running"] >= 2                # requests overlapped on the device
    assert st["queued"] == 0


def test_pool_wait_poll_and_errors(B, inputs, alone):
    (S, M), req = inputs[1], REQUESTS[1]
    need = B.dir_workspace_bytes(tuple(S.shape), _params(B, req))
    with B.Pool(slots=2, max_bytes=need) as pool:
        t1 = pool.submit(S, M, _params(B, req))
        t2 = pool.submit(*inputs[3], _params(B, REQUESTS[3]))   # queued or running, within the budget
        f2, _ = pool.wait(t2)
        f1, _ = pool.wait(t1)
        assert torch.equal(f1, alone[1][0]) and torch.equal(f2, alone[3][0])
        with pytest.raises(B.DemonsError):
            pool.poll(t1)                                      # already taken
        with pytest.raises(B.DemonsError):
            pool.wait(12345)                                   # unknown
    with B.Pool(slots=1, max_bytes=need // 2) as pool:
        with pytest.raises(B.DemonsError) as e:
            pool.submit(S, M, _params(B, req))                 # needs more than the whole budget
        assert e.value.code == B.DIR_ENOMEM


# compatible schedules (levels, iterations, sigma, storage) at uneven sizes and
# every variant: a pool with a batch limit runs them as lockstep batches
COMPATIBLE = [((48, 40, 12), "passive", 1.0), ((96, 80, 40), "inverse_consistent", 1.0),
              ((33, 29, 17), "active", 1.0), ((64, 64, 32), "double", 0.4), ((27, 45, 9), "evolved", 1.0),
              ((80, 64, 24), "passive", 0.4), ((40, 40, 24), "inverse_consistent", 1.0),
              ((72, 56, 20), "active", 1.0), ((130, 36, 16), "double", 1.0)]


@pytest.fixture(scope="module")
def compatible(B):
    ins, alone = [], []
    h = B.dir_create(0)
    try:
        for k, (shape, variant, alpha) in enumerate(COMPATIBLE):
            ph = P.make_phantom(shape, seed=600 + k, max_u=2.5)
            S, M = _dev(ph.static), _dev(ph.moving)
            p = B.make_params(variant, [5, 4], sigma=1.0, alpha=alpha)
            f, st = B.dir_register(h, S, M, p)
            ins.append((S, M, p))
            alone.append((f.clone(), st["iters_run"]))
    finally:
        B.dir_destroy(h)
    return ins, alone


@pytest.mark.parametrize("slots,max_batch,budget_factor", [(1, 4, 0.0), (2, 8, 0.0), (3, 8, 2.5), (1, 8, 1.0)])
def test_pool_batches_equal_alone_and_budget_holds(B, compatible, slots, max_batch, budget_factor):
    ins, alone = compatible
    needs = [B.dir_workspace_bytes(tuple(S.shape), p) for S, _, p in ins]
    budget = int(budget_factor * max(needs))  # 0: no limit; 1.0: room for one registration only
    with B.Pool(slots=slots, max_bytes=budget, max_batch=max_batch) as pool:
        blockers = []
        if not budget:
            # long registrations occupy every slot first, so the compatible
            # requests queue behind them and are admitted in groups
            Sb = _dev(P.make_phantom((160, 160, 80), seed=699, max_u=2.5).static)
            Mb = Sb.flip(0).contiguous()
            blockers = [pool.submit(Sb, Mb, B.make_params("passive", [30, 20], sigma=1.0)) for _ in range(slots)]
        tickets = [pool.submit(S, M, p) for S, M, p in ins]
        got = {t: pool.wait(t) for t in reversed(tickets)}  # collect in an order other than submission
        for t in blockers:
            pool.wait(t)
        st = pool.stats()
    for k, t in enumerate(tickets):
        f, stats = got[t]
        assert torch.equal(f, alone[k][0]), COMPATIBLE[k]
        assert stats["iters_run"] == alone[k][1]
    if budget:
        assert st["peak_bytes"] <= budget
    if budget_factor == 0.0:
        assert st["peak_running"] >= 2  # requests ran as batches
    assert st["peak_running"] <= slots * max_batch
    assert st["queued"] == 0


def test_pool_rejects_a_bad_batch_limit(B):
    for bad in (0, B.DIR_MAX_BATCH + 1):
        with pytest.raises(B.DemonsError) as e:
            B.Pool(slots=1, max_batch=bad)
        assert e.value.code == B.DIR_EINVAL
