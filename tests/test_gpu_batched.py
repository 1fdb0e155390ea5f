"""GPU tests of the batched form and of the product tile shapes.

A batched problem's result must be the same as the single-problem result of
the same inputs whatever else is in the batch, and the product kernels
accumulate every output in the same order for every tile shape and schedule,
so these comparisons are bitwise (torch.equal). Correctness itself is checked
against the CPU oracle on small members of each batch and by invariants
(reconstruction, orthogonality) on every member.
"""
import functools

import numpy as np
import pytest
import torch

import oracle as O
import synth_inputs as S

pytestmark = pytest.mark.gpu


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64).cuda()


def host(t):
    return t.detach().cpu().numpy()


def _items(problems):
    return [(dev(P.U), dev(P.sigma), dev(P.V), dev(P.a), dev(P.b)) for P in problems]


def _invariants(item, out):
    U, sig, V, a, b = item
    Ug, sg, Vg = out
    m = U.shape[0]
    Ah = (U * sig[None, :]) @ V[:, :m].T + torch.outer(a, b)
    recon = (torch.linalg.norm((Ug * sg[None, :]) @ Vg[:, :m].T - Ah) / torch.linalg.norm(Ah)).item()
    oU = torch.max(torch.abs(Ug.T @ Ug - torch.eye(m, dtype=torch.float64, device=U.device))).item()
    n = V.shape[0]
    oV = torch.max(torch.abs(Vg.T @ Vg - torch.eye(n, dtype=torch.float64, device=U.device))).item()
    return recon, oU, oV


MIXED = [(1, 1, "uniform", {}), (3, 7, "uniform", {}), (64, 64, "uniform", {}), (65, 130, "uniform", {}),
         (100, 173, "geometric", {}), (129, 129, "clustered", dict(zero_frac=0.05, zero_q=True)),
         (40, 40, "zero", {}), (257, 300, "uniform", {}), (16, 16, "uniform", {}), (200, 399, "uniform", {})]


def _mixed_problems(seed0=0):
    return [S.make_problem(m, n, kind, seed=seed0 + i, **kw) for i, (m, n, kind, kw) in enumerate(MIXED)]


@pytest.mark.parametrize("precision", [0, 1])
def test_batched_equals_single_bitwise(lib, precision):
    probs = _mixed_problems()
    items = _items(probs)
    singles = [lib.rank1_update(*it, precision=precision, want_defl=True) for it in items]
    b = lib.Batch(items, precision=precision, want_defl=True)
    b.launch()
    assert b.status() == [lib.SVDU_OK] * len(items)
    for i, (s, o, d) in enumerate(zip(singles, b.outs, b.defl)):
        for x, y in zip(s[:3], o):
            assert torch.equal(x, y), i
        assert torch.equal(s[3], d), i
    b.close()


def test_batched_mixes_lane_and_wave_item_kernels(lib):
    """Orders on both sides of 2048 in one batch: the secular, Loewner,
    column-norm and transposed-product launches then hold jobs that take one
    item per lane next to jobs that take one item per wave. Every problem must
    match its single-call result bitwise and reconstruct to 1e-12."""
    sizes = [(2100, 2100), (64, 2200), (300, 457), (1, 2049), (2049, 2049)]
    probs = [S.make_problem(m, n, "uniform", seed=90 + i) for i, (m, n) in enumerate(sizes)]
    items = _items(probs)
    singles = [lib.rank1_update(*it) for it in items]
    b = lib.Batch(items)
    b.launch()
    assert b.status() == [lib.SVDU_OK] * len(items)
    for i, (s, o) in enumerate(zip(singles, b.outs)):
        for x, y in zip(s[:3], o):
            assert torch.equal(x, y), i
        recon, oU, oV = _invariants(items[i], o)
        assert recon <= 1e-12 and oU <= 1e-12 and oV <= 1e-12, (i, recon, oU, oV)
    b.close()


def test_batched_graph_replays_and_persistent_schedule(lib):
    probs = _mixed_problems(seed0=20)
    items = _items(probs)
    ref = [lib.rank1_update(*it)[:3] for it in items]
    for persistent in (False, True):
        b = lib.Batch(items, persistent=persistent)
        for rep in range(3):
            for o in b.outs:           # clobber outputs between replays
                for t in o:
                    t.fill_(float("nan"))
            b.launch(use_graph=True)
            torch.cuda.synchronize()
            _ = torch.randn(1000, device="cuda").sum().item()   # unrelated eager work between replays
            assert b.status() == [lib.SVDU_OK] * len(items)
            for i, (r, o) in enumerate(zip(ref, b.outs)):
                for x, y in zip(r, o):
                    assert torch.equal(x, y), (persistent, rep, i)
        b.close()


def test_batched_new_inputs_between_graph_replays(lib):
    """Inputs may change between launches of a captured batch."""
    P1 = _mixed_problems(seed0=40)
    P2 = _mixed_problems(seed0=60)
    items = _items(P1)
    b = lib.Batch(items)
    b.launch(use_graph=True)
    torch.cuda.synchronize()
    for it, P in zip(items, P2):
        for t, x in zip(it, (P.U, P.sigma, P.V, P.a, P.b)):
            t.copy_(dev(x))
    b.launch(use_graph=True)
    assert b.status() == [lib.SVDU_OK] * len(items)
    for it, o in zip(items, b.outs):
        r = lib.rank1_update(*it)[:3]
        for x, y in zip(r, o):
            assert torch.equal(x, y)
    b.close()


def test_batched_per_problem_status(lib):
    """A bad problem reports its own error; the others are unaffected."""
    probs = _mixed_problems(seed0=80)[:6]
    items = _items(probs)
    a_bad = items[2][3].clone()
    a_bad[0] = float("nan")
    s_bad = items[4][1].clone()
    s_bad[0] = s_bad[1] * 0.5        # not descending
    items_b = list(items)
    items_b[2] = (items[2][0], items[2][1], items[2][2], a_bad, items[2][4])
    items_b[4] = (items[4][0], s_bad, items[4][2], items[4][3], items[4][4])
    b = lib.Batch(items_b)
    b.launch()
    st = b.status()
    assert st[2] == lib.SVDU_ENONFINITE
    assert st[4] == lib.SVDU_EBADSIGMA
    for i in (0, 1, 3, 5):
        assert st[i] == lib.SVDU_OK
        r = lib.rank1_update(*items[i])[:3]
        for x, y in zip(r, b.outs[i]):
            assert torch.equal(x, y)
    b.close()


@pytest.mark.parametrize("shape", [0, 1, 2, 3, 4, 5])
@pytest.mark.parametrize("m,n", [(300, 457), (301, 333), (20, 37)])
def test_tile_shapes_give_identical_results(lib, shape, m, n):
    """Every tile shape gives the same bits. 300 x 457: 16-byte rows of X and
    ragged last k steps (full vector steps, then element steps); 301 x 333: odd
    leading dimensions, so X is read element by element throughout; 20 x 37:
    fewer k steps than one LDS stage holds."""
    P = S.make_problem(m, n, "uniform", seed=7)
    args = (dev(P.U), dev(P.sigma), dev(P.V), dev(P.a), dev(P.b))
    old = lib.set_option(lib.SVDU_OPT_TILE_SHAPE, 0)
    try:
        ref = lib.rank1_update(*args)
        lib.set_option(lib.SVDU_OPT_TILE_SHAPE, shape)
        got = lib.rank1_update(*args)
        ref32 = None
        lib.set_option(lib.SVDU_OPT_TILE_SHAPE, 0)
        ref32 = lib.rank1_update(*args, precision=lib.SVDU_PREC_SPLIT32)
        lib.set_option(lib.SVDU_OPT_TILE_SHAPE, shape)
        got32 = lib.rank1_update(*args, precision=lib.SVDU_PREC_SPLIT32)
    finally:
        lib.set_option(lib.SVDU_OPT_TILE_SHAPE, old)
    for x, y in zip(ref, got):
        assert torch.equal(x, y)
    for x, y in zip(ref32, got32):
        assert torch.equal(x, y)
    r = O.svd_rank1_update(P.U, P.sigma, P.V, P.a, P.b)
    assert np.max(np.abs(host(got[1]) - r.sigma)) <= 1e-13 * r.sigma[0]


@pytest.mark.parametrize("shape", [-1, 4, 5])
def test_persistent_single_update(lib, shape):
    P = S.make_problem(513, 700, "uniform", seed=8)
    args = (dev(P.U), dev(P.sigma), dev(P.V), dev(P.a), dev(P.b))
    ref = lib.rank1_update(*args)
    old_s = lib.set_option(lib.SVDU_OPT_TILE_SHAPE, shape)
    old = lib.set_option(lib.SVDU_OPT_PERSISTENT, 1)
    try:
        got = lib.rank1_update(*args)
    finally:
        lib.set_option(lib.SVDU_OPT_PERSISTENT, old)
        lib.set_option(lib.SVDU_OPT_TILE_SHAPE, old_s)
    for x, y in zip(ref, got):
        assert torch.equal(x, y)


@functools.lru_cache(maxsize=1)
def _batched_workload(count, seed=4):
    """The batched workload: m log-uniform in [64, 1024], n = m + U{0..m},
    sigma uniform in [0.01, 10] descending, Haar factors, a, b ~ N(0, 1/n)."""
    ms, ns = S.batched_sizes(count, seed=seed)
    rng = np.random.default_rng(seed + 100)
    items = []
    for i, (m, n) in enumerate(zip(ms.tolist(), ns.tolist())):
        U = S.haar_torch(m, seed=10_000 + 2 * i, device="cuda")
        V = S.haar_torch(n, seed=10_001 + 2 * i, device="cuda")
        sig = S.sigma_uniform(m, 0.01, 10.0, rng)
        a = rng.standard_normal(m) / np.sqrt(n)
        b = rng.standard_normal(n) / np.sqrt(n)
        items.append((U, dev(sig), V, dev(a), dev(b)))
    return items


@pytest.mark.parametrize("precision", [0, 1])
def test_batched_workload_512(lib, precision):
    """The full batched workload (512 problems) in the configuration the
    benchmark times: one captured graph, every problem checked."""
    items = _batched_workload(512)
    b = lib.Batch(items, precision=precision)
    b.launch(use_graph=True)
    assert b.status() == [lib.SVDU_OK] * 512
    # every member: invariants
    tol_r, tol_o = (1e-12, 1e-12) if precision == 0 else (5e-6, 5e-6)
    worst = [0.0, 0.0, 0.0]
    for it, o in zip(items, b.outs):
        inv = _invariants(it, o)
        worst = [max(w, v) for w, v in zip(worst, inv)]
    assert worst[0] <= tol_r and worst[1] <= tol_o and worst[2] <= tol_o, worst
    # sampled members: bitwise equal to the single-problem path
    rng = np.random.default_rng(1)
    for i in rng.choice(512, size=24, replace=False).tolist():
        r = lib.rank1_update(*items[i], precision=precision)[:3]
        for x, y in zip(r, b.outs[i]):
            assert torch.equal(x, y), i
    # the smallest members against the oracle
    if precision == 0:
        order = np.argsort([it[2].shape[0] for it in items])[:3]
        for i in order.tolist():
            U, sg, V, a, bb = (host(t) for t in items[i])
            r = O.svd_rank1_update(U, sg, V, a, bb)
            assert np.max(np.abs(host(b.outs[i][1]) - r.sigma)) <= 1e-13 * r.sigma[0]
    b.close()


def test_autotune_table_and_results_unchanged(lib):
    P = S.make_problem(200, 333, "uniform", seed=3)
    args = (dev(P.U), dev(P.sigma), dev(P.V), dev(P.a), dev(P.b))
    before = lib.rank1_update(*args)
    saved = lib.tile_table(0)
    try:
        table, times = lib.autotune(0, max_n=512)
        assert len(table) == lib.SVDU_TILE_BUCKETS and all(0 <= s < lib.SVDU_TILE_SHAPES for s in table)
        for bk in range(4):   # buckets up to 512 were timed
            assert all(t > 0 for t in times[bk])
            assert times[bk][table[bk]] == min(times[bk])
        assert lib.tile_table(0) == table
        after = lib.rank1_update(*args)
    finally:
        lib.tile_table(0, saved)
    for x, y in zip(before, after):
        assert torch.equal(x, y)


# ---------------------------------------------------------------------------
# close-cluster refinement
# ---------------------------------------------------------------------------
def _planted_close_output(m, n, seed, gaps=(1e-9, 1e-11, 1e-13), triple=True):
    """Inputs whose updated matrix A^ has planted close singular values: A^ is
    built first (Haar factors, sigma^ with pairs at the given relative gaps),
    then A = A^ - a b^T is decomposed on the host (LAPACK, a library routine
    used only to make inputs)."""
    rng = np.random.default_rng(seed)
    Uh = S.haar(m, rng)
    Vh = S.haar(n, rng)
    sh = np.sort(rng.uniform(0.5, 10.0, m))[::-1].copy()
    pos = 1
    for g in gaps:
        sh[pos + 1] = sh[pos] * (1.0 - g)
        pos += 7
    if triple:
        sh[pos + 1] = sh[pos] * (1 - 3e-12)
        sh[pos + 2] = sh[pos] * (1 - 7e-12)
    sh = np.sort(sh)[::-1].copy()
    Ah = (Uh * sh[None, :]) @ Vh[:, :m].T
    a = rng.standard_normal(m) / np.sqrt(n)
    b = rng.standard_normal(n) / np.sqrt(n)
    A = Ah - np.outer(a, b)
    Ua, sa, Vta = np.linalg.svd(A, full_matrices=True)
    return Ua, sa, Vta.T.copy(), a, b, Ah


def _recon_np(Ah, U, s, V):
    m = U.shape[0]
    return np.linalg.norm((U * s[None, :]) @ V[:, :m].T - Ah) / np.linalg.norm(Ah)


@pytest.mark.parametrize("m,n,npairs", [(200, 200, 3), (150, 260, 3), (300, 333, 40), (450, 451, 60)])
def test_refinement_of_close_clusters(lib, m, n, npairs):
    """Planted close pairs (and one triple); 40 and 60 pairs gather 83 and 123
    columns, up to the 128 the refinement takes, with n not a multiple of 4."""
    gaps = tuple((1e-9, 1e-11, 1e-13)[i % 3] for i in range(npairs))
    U, s, V, a, b, Ah = _planted_close_output(m, n, seed=m + n, gaps=gaps)
    args = (dev(U), dev(s), dev(V), dev(a), dev(b))
    on = [host(t) for t in lib.rank1_update(*args)[:3]]
    old = lib.set_option(lib.SVDU_OPT_REFINE, 0)
    try:
        off = [host(t) for t in lib.rank1_update(*args)[:3]]
    finally:
        lib.set_option(lib.SVDU_OPT_REFINE, old)
    r_on, r_off = _recon_np(Ah, *on), _recon_np(Ah, *off)
    # rounding of the refined products grows with the order: 8 u sqrt(m n), well
    # inside the 1e-12 the update is held to (1.8e-13 at 200, 4e-13 at 450)
    assert r_on <= 8 * 2.0 ** -53 * np.sqrt(m * n), (r_on, r_off)
    assert r_on <= r_off * 1.01
    assert O.orth_error(on[0]) <= 1e-13 and O.orth_error(on[2]) <= 1e-13
    # singular values and the columns outside the close clusters are untouched
    sg = off[1]
    close = np.zeros(m, dtype=bool)
    d = (sg[:-1] - sg[1:]) <= 1e-6 * sg[:-1]
    close[:-1] |= d
    close[1:] |= d
    assert np.any(close)
    assert np.array_equal(on[0][:, ~close], off[0][:, ~close])
    assert np.array_equal(on[1], off[1])
    assert np.array_equal(on[2][:, np.r_[~close, np.ones(n - m, bool)]],
                          off[2][:, np.r_[~close, np.ones(n - m, bool)]])
    # singular values against the oracle
    r = O.svd_rank1_update(U, s, V, a, b)
    assert np.max(np.abs(on[1] - r.sigma)) <= 1e-13 * r.sigma[0]
