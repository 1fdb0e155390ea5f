"""GPU tests of the serving runtime: resident matrices, memory admission and
continuous batching. Every served result must equal, bitwise, the result of
applying the same updates one at a time with svdu_rank1_update (on the path
the server used), in release order, from the same initial factors."""
import numpy as np
import pytest
import torch

import synth_inputs as S

pytestmark = pytest.mark.gpu


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64).cuda()


SIZES = [(64, 64), (100, 100), (256, 256), (300, 300), (512, 512), (700, 700), (64, 64), (256, 256)]


def _setup(lib, server, sizes, seed=0):
    init = []
    for i, (m, n) in enumerate(sizes):
        P = S.make_problem(m, n, "uniform", seed=seed + i)
        U, s, V = dev(P.U), dev(P.sigma), dev(P.V)
        init.append((U.clone(), s.clone(), V.clone()))
        assert server.add_matrix(U, s, V) == i
    return init


def _requests(sizes, count, span, seed):
    rng = np.random.default_rng(seed)
    reqs = []
    t = 0.0
    for k in range(count):
        t += rng.exponential(span / count)
        i = int(rng.integers(0, len(sizes)))
        m, n = sizes[i]
        a = dev(rng.standard_normal(m) / np.sqrt(n))
        b = dev(rng.standard_normal(n) / np.sqrt(n))
        reqs.append((i, a, b, t))
    return reqs


def _replay(lib, init, reqs, fmm_min_n=0):
    cur = [tuple(t.clone() for t in x) for x in init]
    for i, a, b, _ in reqs:
        U, s, V = cur[i]
        path = lib.SVDU_PATH_FMM if (fmm_min_n and V.shape[0] >= fmm_min_n) else lib.SVDU_PATH_DIRECT
        Uo, so, Vo, _ = lib.rank1_update(U, s, V, a, b, path=path, want_defl=False)
        cur[i] = (Uo, so, Vo)
    return cur


@pytest.mark.parametrize("workers,fmm_min_n", [(1, 0), (3, 0), (3, 600)])
def test_served_results_equal_one_at_a_time(lib, workers, fmm_min_n):
    srv = lib.Server(arena_bytes=1 << 30, workers=workers, max_batch=16, fmm_min_n=fmm_min_n,
                     min_batch_cost=2e9)
    init = _setup(lib, srv, SIZES)
    reqs = _requests(SIZES, 60, span=0.05, seed=workers + fmm_min_n)
    # the first 20 are queued before the workers start (released at 0, so they
    # batch); the rest arrive while those run
    for k, (i, a, b, t) in enumerate(reqs):
        if k < 20:
            reqs[k] = (i, a, b, 0.0)
            srv.submit(i, a, b, 0.0)
    srv.start()
    for i, a, b, t in reqs[20:]:
        srv.submit(i, a, b, t)
    assert srv.drain(300.0) == lib.SVDU_OK
    done = sorted(srv.poll(), key=lambda c: c["id"])
    assert len(done) == len(reqs) and all(c["status"] == lib.SVDU_OK for c in done)
    assert max(c["batch"] for c in done) > 1          # batching happened
    # per matrix: updates ran in release order, one at a time
    for i in range(len(SIZES)):
        mine = [c for c in done if c["matrix"] == i]
        for p, q in zip(mine, mine[1:]):
            assert q["t_start"] >= p["t_done"] - 1e-9
    for c in done:
        assert c["t_start"] >= c["t_release"] - 1e-9 and c["t_done"] >= c["t_start"]
    ref = _replay(lib, init, reqs, fmm_min_n)
    for i in range(len(SIZES)):
        got = srv.current(i)
        for x, y in zip(ref[i], got):
            assert torch.equal(x, y), i
    srv.close()


def test_memory_admission_serialises_and_rejects(lib):
    """An arena that holds one large update at a time still serves everything
    (admission waits for memory); an update that can never fit fails alone."""
    sizes = [(512, 512), (512, 512), (600, 600), (64, 64), (2048, 2048)]
    need = lib.svdu_workspace_bytes(600, 600) + (1 << 16)
    srv = lib.Server(arena_bytes=int(need * 1.5), workers=3, max_batch=8, min_batch_cost=0.0)
    init = _setup(lib, srv, sizes, seed=50)
    reqs = [r for r in _requests(sizes, 30, span=0.01, seed=9)]
    srv.start()
    ids = [srv.submit(i, a, b, t) for i, a, b, t in reqs]
    assert srv.drain(300.0) == lib.SVDU_OK
    done = {c["id"]: c for c in srv.poll()}
    assert set(done) == set(ids)
    ok_reqs = []
    for rid, (i, a, b, t) in zip(ids, reqs):
        if sizes[i][0] == 2048:
            assert done[rid]["status"] == lib.SVDU_ENOMEM
        else:
            assert done[rid]["status"] == lib.SVDU_OK
            ok_reqs.append((i, a, b, t))
    ref = _replay(lib, init, ok_reqs)
    for i in range(len(sizes)):
        got = srv.current(i)
        for x, y in zip(ref[i], got):
            assert torch.equal(x, y), i
    srv.close()


def test_bad_request_fails_alone(lib):
    srv = lib.Server(arena_bytes=1 << 28, workers=2, max_batch=8, min_batch_cost=1e12)
    init = _setup(lib, srv, SIZES[:4], seed=70)
    srv.start()
    reqs = _requests(SIZES[:4], 12, span=0.0, seed=3)
    bad = 5
    a_bad = reqs[bad][1].clone()
    a_bad[0] = float("nan")
    reqs[bad] = (reqs[bad][0], a_bad, reqs[bad][2], reqs[bad][3])
    ids = [srv.submit(i, a, b, t) for i, a, b, t in reqs]
    assert srv.drain(120.0) == lib.SVDU_OK
    done = {c["id"]: c for c in srv.poll()}
    assert done[ids[bad]]["status"] == lib.SVDU_ENONFINITE
    assert all(done[r]["status"] == lib.SVDU_OK for k, r in enumerate(ids) if k != bad)
    # the failed update leaves its matrix unchanged; the others are applied in order
    ok = [r for k, r in enumerate(reqs) if k != bad]
    ref = _replay(lib, init, ok)
    for i in range(4):
        for x, y in zip(ref[i], srv.current(i)):
            assert torch.equal(x, y), i
    srv.close()
