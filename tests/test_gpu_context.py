"""GPU tests of contexts (svdu_create / svdu_destroy): each context holds its
own options, and two contexts used at the same time from two host threads
give, bitwise, the results each gives alone. A server keeps the options its
context had when it was created."""
import threading

import numpy as np
import pytest
import torch

import synth_inputs as S

pytestmark = pytest.mark.gpu


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64).cuda()


def _problem(seed, m=300, n=333):
    """Inputs whose updated matrix has planted close singular values (pairs at
    relative gaps 1e-9 and 1e-11), so that the refinement option changes the
    result bits: A^ is built first, then A = A^ - a b^T is decomposed on the
    host (LAPACK, a library routine used only to make inputs)."""
    rng = np.random.default_rng(seed)
    Uh, Vh = S.haar(m, rng), S.haar(n, rng)
    sh = np.sort(rng.uniform(0.5, 10.0, m))[::-1].copy()
    for k, g in enumerate((1e-9, 1e-11, 1e-9, 1e-11)):
        sh[8 * k + 2] = sh[8 * k + 1] * (1.0 - g)
    sh = np.sort(sh)[::-1].copy()
    a = rng.standard_normal(m) / np.sqrt(n)
    b = rng.standard_normal(n) / np.sqrt(n)
    A = (Uh * sh[None, :]) @ Vh[:, :m].T - np.outer(a, b)
    Ua, sa, Vta = np.linalg.svd(A, full_matrices=True)
    return [dev(Ua), dev(sa), dev(Vta.T), dev(a), dev(b)]


def _run(lib, ctx, args, stream, reps):
    outs = []
    with torch.cuda.stream(stream):
        for _ in range(reps):
            Uo, so, Vo, _ = lib.rank1_update(*args, ctx=ctx, stream=stream, want_defl=False)
            outs.append((Uo, so, Vo))
    stream.synchronize()
    return outs


def test_two_contexts_two_threads_bitwise(lib):
    ca, cb = lib.Context(), lib.Context()
    try:
        ca.set_option(lib.SVDU_OPT_REFINE, 1)
        ca.set_option(lib.SVDU_OPT_TILE_SHAPE, lib.SVDU_TILE_128x128)
        cb.set_option(lib.SVDU_OPT_REFINE, 0)
        cb.set_option(lib.SVDU_OPT_TILE_SHAPE, lib.SVDU_TILE_64x64)
        cb.set_option(lib.SVDU_OPT_PERSISTENT, 1)
        args = _problem(11)
        sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
        ref_a = _run(lib, ca, args, sa, 1)[0]
        ref_b = _run(lib, cb, args, sb, 1)[0]
        # the options differ in a way that shows in the bits (refinement on / off)
        assert not torch.equal(ref_a[0], ref_b[0])
        got = {}

        def worker(name, ctx, stream):
            got[name] = _run(lib, ctx, args, stream, 6)

        ta = threading.Thread(target=worker, args=("a", ca, sa))
        tb = threading.Thread(target=worker, args=("b", cb, sb))
        ta.start()
        tb.start()
        ta.join()
        tb.join()
        for name, ref in (("a", ref_a), ("b", ref_b)):
            assert len(got[name]) == 6
            for o in got[name]:
                for x, y in zip(o, ref):
                    assert torch.equal(x, y), name
    finally:
        ca.close()
        cb.close()


def test_timing_record_is_per_context(lib):
    ca, cb = lib.Context(), lib.Context()
    try:
        args = _problem(12)
        ca.set_option(lib.SVDU_OPT_TIMING, 1)
        lib.rank1_update(*args, ctx=ca, want_defl=False)
        lib.rank1_update(*args, ctx=cb, want_defl=False)
        lib.rank1_update(*args, ctx=ca, want_defl=False)
        ta = lib.timing_read(16, ctx=ca)
        tb = lib.timing_read(16, ctx=cb)
        assert len(ta) == 2 and len(tb) == 0
        assert all(t >= 0.0 for row in ta for t in row)
    finally:
        ca.close()
        cb.close()


def test_server_keeps_the_options_of_its_creation(lib):
    ctx = lib.Context()
    try:
        ctx.set_option(lib.SVDU_OPT_REFINE, 0)
        args = _problem(13)
        U, s, V, a, b = args
        ref = lib.rank1_update(U, s, V, a, b, ctx=ctx, want_defl=False)
        srv = lib.Server(arena_bytes=1 << 28, workers=2, max_batch=4, ctx=ctx)
        try:
            ids = [srv.add_matrix(U.clone(), s.clone(), V.clone()) for _ in range(3)]
            # changed after creation: the server must not see it
            ctx.set_option(lib.SVDU_OPT_REFINE, 1)
            srv.start()
            for i in ids:
                srv.submit(i, a, b, 0.0)
            ctx.set_option(lib.SVDU_OPT_SECULAR_MAXIT, 1)   # would fail every update if it reached the server
            assert srv.drain(120.0) == lib.SVDU_OK
            done = srv.poll()
            assert len(done) == 3 and all(c["status"] == lib.SVDU_OK for c in done)
            for i in ids:
                Uo, so, Vo = srv.current(i)
                assert torch.equal(Uo, ref[0]) and torch.equal(so, ref[1]) and torch.equal(Vo, ref[2])
        finally:
            srv.close()
    finally:
        ctx.close()


def _fmm_problem(seed, m, n):
    rng = np.random.default_rng(seed)
    return [S.haar_torch(m, seed=seed, device="cuda"), dev(S.sigma_uniform(m, 1e-3, 1.0, rng)),
            S.haar_torch(n, seed=seed + 1, device="cuda"), dev(rng.standard_normal(m) / np.sqrt(n)),
            dev(rng.standard_normal(n) / np.sqrt(n))]


def _run_fmm(lib, ctx, args, stream, reps):
    outs = []
    with torch.cuda.stream(stream):
        for _ in range(reps):
            Uo, so, Vo, _ = lib.rank1_update(*args, path=lib.SVDU_PATH_FMM, eps=1e-10, ctx=ctx, stream=stream,
                                             want_defl=False)
            outs.append((Uo, so, Vo))
    stream.synchronize()
    return outs


def test_fmm_path_two_contexts_two_threads_bitwise(lib):
    """The FMM path forks its right-hand products onto a second stream of the
    context and joins them back, and copies roots into the context's pinned
    memory: two contexts driving it at once from two threads, each on its own
    stream, give bitwise their single-thread results (order 3000, so the
    secular roots take the far-field form too)."""
    ca, cb = lib.Context(), lib.Context()
    try:
        pa, pb = _fmm_problem(31, 3000, 3000), _fmm_problem(41, 2500, 3100)
        sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
        ref_a = _run_fmm(lib, ca, pa, sa, 1)[0]
        ref_b = _run_fmm(lib, cb, pb, sb, 1)[0]
        # against the direct path of the same inputs
        for p, ref in ((pa, ref_a), (pb, ref_b)):
            Ud, sd, Vd, _ = lib.rank1_update(*p, want_defl=False)
            assert float((ref[1] - sd).abs().max()) <= 1e-13 * float(sd[0])
            assert float((ref[0] - Ud).abs().max()) <= 1e-9 and float((ref[2] - Vd).abs().max()) <= 1e-9
        got = {}

        def worker(name, ctx, args, stream):
            got[name] = _run_fmm(lib, ctx, args, stream, 3)

        ta = threading.Thread(target=worker, args=("a", ca, pa, sa))
        tb = threading.Thread(target=worker, args=("b", cb, pb, sb))
        ta.start()
        tb.start()
        ta.join()
        tb.join()
        for name, ref in (("a", ref_a), ("b", ref_b)):
            assert len(got[name]) == 3
            for o in got[name]:
                for x, y in zip(o, ref):
                    assert torch.equal(x, y), name
    finally:
        ca.close()
        cb.close()


def test_fmm_path_context_reused_across_orders(lib):
    """One context's pinned root buffer grows with the order; calls of
    different orders in a row match fresh contexts' results bitwise."""
    ctx = lib.Context()
    try:
        s = torch.cuda.current_stream()
        for m, seed in ((500, 51), (3000, 52), (500, 53)):
            p = _fmm_problem(seed, m, m)
            got = _run_fmm(lib, ctx, p, s, 1)[0]
            fresh = lib.Context()
            try:
                ref = _run_fmm(lib, fresh, p, s, 1)[0]
            finally:
                fresh.close()
            for x, y in zip(got, ref):
                assert torch.equal(x, y), m
    finally:
        ctx.close()


def test_fmm_path_error_exit_then_reuse(lib):
    """A non-finite input stops the FMM path before its products (the status
    word is read with the first level's roots); the call reports
    SVDU_ENONFINITE, and the same context's next call is bitwise a fresh
    context's."""
    ctx = lib.Context()
    try:
        p = _fmm_problem(61, 2300, 2300)
        bad = list(p)
        bad[3] = p[3].clone()
        bad[3][7] = float("nan")
        with pytest.raises(lib.SvduError) as e:
            lib.rank1_update(*bad, path=lib.SVDU_PATH_FMM, eps=1e-10, ctx=ctx, want_defl=False)
        assert e.value.code == lib.SVDU_ENONFINITE
        got = lib.rank1_update(*p, path=lib.SVDU_PATH_FMM, eps=1e-10, ctx=ctx, want_defl=False)
        fresh = lib.Context()
        try:
            ref = lib.rank1_update(*p, path=lib.SVDU_PATH_FMM, eps=1e-10, ctx=fresh, want_defl=False)
        finally:
            fresh.close()
        for x, y in zip(got[:3], ref[:3]):
            assert torch.equal(x, y)
    finally:
        ctx.close()
