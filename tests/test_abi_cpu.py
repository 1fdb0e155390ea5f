"""Host-side checks of the C ABI: the library loads, exports every symbol that
include/svdu.h declares, sizes its workspace, and rejects bad arguments
before enqueuing anything (no GPU needed)."""
import ctypes
import os
import re

import pytest

import paper_1707_08369_amd as svdu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "svdu.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(svdu_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(svdu.LIB_PATH):
        pytest.skip("libsvdu.so not built")
    return svdu.load()


@pytest.fixture()
def ctx(lib):
    """A raw context handle (svdu_create makes no HIP call)."""
    h = ctypes.c_void_p()
    assert svdu.svdu_create(ctypes.byref(h), 0) == svdu.SVDU_OK and h.value
    yield h
    svdu.svdu_destroy(h)


def test_context_create_destroy(lib):
    h = ctypes.c_void_p(1234)
    assert svdu.svdu_create(ctypes.byref(h), -1) == svdu.SVDU_EINVAL
    assert h.value is None
    assert svdu.svdu_create(None, 0) == svdu.SVDU_EINVAL
    a, b = ctypes.c_void_p(), ctypes.c_void_p()
    assert svdu.svdu_create(ctypes.byref(a), 0) == svdu.SVDU_OK
    assert svdu.svdu_create(ctypes.byref(b), 0) == svdu.SVDU_OK
    assert a.value != b.value
    # options live in the context: b does not see a's change
    assert svdu.svdu_set_option(a, svdu.SVDU_OPT_SECULAR_MAXIT, 33) == 200
    assert svdu.svdu_set_option(b, svdu.SVDU_OPT_SECULAR_MAXIT, 200) == 200
    assert svdu.svdu_set_option(a, svdu.SVDU_OPT_SECULAR_MAXIT, 200) == 33
    assert svdu.svdu_set_option(None, svdu.SVDU_OPT_SECULAR_MAXIT, 5) == svdu.SVDU_EINVAL
    svdu.svdu_destroy(a)
    svdu.svdu_destroy(b)
    svdu.svdu_destroy(None)


def test_library_exports_every_declared_symbol(lib):
    syms = declared_symbols()
    assert len(syms) >= 9
    for name in syms:
        assert hasattr(lib, name), name
    assert set(svdu.EXPORTS) == set(syms)


def test_workspace_sizes(lib):
    assert svdu.svdu_workspace_bytes(0, 5) == 0
    assert svdu.svdu_workspace_bytes(6, 5) == 0
    small = svdu.svdu_workspace_bytes(256, 256)
    big = svdu.svdu_workspace_bytes(8192, 8192)
    # the intermediate bases U~ (m x m) and V~ (n x n) dominate; the FMM
    # path runs the two sides in turn through one of them
    assert big >= 2 * 8192 * 8192 * 8
    assert big < 2 * 8192 * 8192 * 8 * 1.1
    assert svdu.svdu_workspace_bytes(4096, 8192) < 8192 * 8192 * 8 * 1.35
    assert 0 < small < big
    assert svdu.svdu_eig_update_workspace_bytes(10, 7) > 0
    assert svdu.svdu_eig_update_workspace_bytes(10, 7, svdu.SVDU_PATH_FMM) > svdu.svdu_eig_update_workspace_bytes(10, 7)
    assert svdu.svdu_workspace_bytes(64, 64, svdu.SVDU_PATH_FMM) > svdu.svdu_workspace_bytes(64, 64)
    assert svdu.svdu_secular_workspace_bytes(7) > 0


def test_status_strings(lib):
    for code in (0, -1, -2, -3, -4, -5, -6, -7):
        assert svdu.svdu_status_string(code) != "unknown status"
    assert svdu.svdu_status_string(12345) == "unknown status"


def _p(v):
    return ctypes.c_void_p(v)


def test_host_argument_errors_return_before_enqueue(lib, ctx):
    fake = _p(0x10000)       # never dereferenced: every call below fails its host checks
    ws = _p(0x100000)
    args = dict(ctx=ctx, m=4, n=6, U=fake, ldu=4, sigma=fake, V=_p(0x20000), ldv=6, a=fake, b=fake, eps=1e-10, path=0,
                precision=0, U_out=_p(0x30000), ldu_out=4, sigma_out=fake, V_out=_p(0x40000), ldv_out=6, defl=None,
                workspace=ws, workspace_bytes=1 << 30, stream=None)

    def call(**kw):
        a = dict(args)
        a.update(kw)
        return svdu.svdu_rank1_update(*a.values())
    assert call(m=0) == svdu.SVDU_EINVAL
    assert call(m=7) == svdu.SVDU_EINVAL              # m > n
    assert call(ldu=3) == svdu.SVDU_EINVAL
    assert call(ldv_out=5) == svdu.SVDU_EINVAL
    assert call(U=None) == svdu.SVDU_EINVAL
    assert call(path=5) == svdu.SVDU_EINVAL
    assert call(U_out=fake, U=fake) == svdu.SVDU_EINVAL   # aliasing
    assert call(workspace=_p(0x100010)) == svdu.SVDU_EINVAL  # misaligned
    assert call(workspace_bytes=16) == svdu.SVDU_ENOMEM
    assert call(path=1, eps=0.0) == svdu.SVDU_EINVAL
    # p = ceil(log_5(1/eps)) above the largest order the kernels hold (16)
    assert call(path=1, eps=1e-13) == svdu.SVDU_ENOTSUP
    assert call(path=1, eps=5.0 ** -16 * 0.99) == svdu.SVDU_ENOTSUP
    assert call(path=1, eps=1e-13, workspace_bytes=16) == svdu.SVDU_ENOTSUP   # refused before sizing
    assert call(ctx=None) == svdu.SVDU_EINVAL
    assert call(precision=3) == svdu.SVDU_EINVAL
    assert call(precision=svdu.SVDU_PREC_SLICED_INT8, path=1) == svdu.SVDU_ENOTSUP   # INT8 form: direct path only
    # INT8 form: INT32 sums of S <= 8 slice products stay exact up to n = 32768
    assert call(precision=svdu.SVDU_PREC_SLICED_INT8, n=40000, ldv=40000, ldv_out=40000) == svdu.SVDU_ENOTSUP
    assert svdu.svdu_eig_update(ctx, 3, 0, fake, 1, fake, fake, 1.0, 0, 0.0, _p(0x50000), 1, fake, None, ws, 1 << 20,
                                None) == svdu.SVDU_EINVAL
    assert svdu.svdu_eig_update(ctx, 3, 4, fake, 4, fake, fake, 0.0, 0, 0.0, _p(0x50000), 4, fake, None, ws, 1 << 20,
                                None) == svdu.SVDU_EINVAL
    assert svdu.svdu_eig_update(ctx, 3, 4, fake, 4, fake, fake, 1.0, 1, 0.0, _p(0x50000), 4, fake, None, ws, 1 << 20,
                                None) == svdu.SVDU_EINVAL   # FMM needs 0 < eps < 1
    assert svdu.svdu_eig_update(ctx, 3, 4, fake, 4, fake, fake, 1.0, 1, 1e-13, _p(0x50000), 4, fake, None, ws, 1 << 20,
                                None) == svdu.SVDU_ENOTSUP  # order above 16
    assert svdu.svdu_secular(ctx, 0, fake, fake, 1.0, fake, fake, None, ws, 1 << 20, None) == svdu.SVDU_EINVAL
    assert svdu.svdu_secular(ctx, 4, fake, fake, 1.0, fake, fake, None, ws, 8, None) == svdu.SVDU_ENOMEM
    assert svdu.svdu_secular(None, 4, fake, fake, 1.0, fake, fake, None, ws, 1 << 20, None) == svdu.SVDU_EINVAL


def test_noalloc_host_checks(lib, ctx):
    """The update without a caller workspace refuses, on the host, sizes beyond
    its scratch array and bad arguments (nothing reaches the device)."""
    fake = _p(0x10000)
    args = [4, 6, fake, 4, fake, _p(0x20000), 6, fake, fake, 0, _p(0x30000), 4, fake, _p(0x40000), 6, None, None,
            None]
    assert svdu.svdu_rank1_update_noalloc(None, *args) == svdu.SVDU_EINVAL
    bad = list(args)
    bad[0] = 7                      # m > n
    assert svdu.svdu_rank1_update_noalloc(ctx, *bad) == svdu.SVDU_EINVAL
    bad = list(args)
    bad[9] = 9                      # precision
    assert svdu.svdu_rank1_update_noalloc(ctx, *bad) == svdu.SVDU_EINVAL
    big = 1400
    assert svdu.svdu_workspace_bytes(big, big) > svdu.SVDU_NOALLOC_SCRATCH_BYTES
    huge = [big, big, fake, big, fake, _p(0x20000), big, fake, fake, 0, _p(0x30000), big, fake, _p(0x40000), big,
            None, None, None]
    assert svdu.svdu_rank1_update_noalloc(ctx, *huge) == svdu.SVDU_ENOMEM
    assert svdu.svdu_workspace_bytes(1024, 1024) <= svdu.SVDU_NOALLOC_SCRATCH_BYTES
    assert svdu.svdu_workspace_bytes(1024, 1024, 0, 1) <= svdu.SVDU_NOALLOC_SCRATCH_BYTES


def test_options(lib, ctx):
    old = svdu.svdu_set_option(ctx, svdu.SVDU_OPT_SECULAR_MAXIT, 17)
    assert svdu.svdu_set_option(ctx, svdu.SVDU_OPT_SECULAR_MAXIT, old) == 17
    assert svdu.svdu_set_option(ctx, 999, 1) == svdu.SVDU_EINVAL
    old = svdu.svdu_set_option(ctx, svdu.SVDU_OPT_TILE_SHAPE, svdu.SVDU_TILE_64x64)
    assert old == -1
    assert svdu.svdu_set_option(ctx, svdu.SVDU_OPT_TILE_SHAPE, -1) == svdu.SVDU_TILE_64x64
    assert svdu.svdu_set_option(ctx, svdu.SVDU_OPT_TILE_SHAPE, svdu.SVDU_TILE_SHAPES) == svdu.SVDU_EINVAL
    assert svdu.svdu_set_option(ctx, svdu.SVDU_OPT_PERSISTENT, 1) == 0
    assert svdu.svdu_set_option(ctx, svdu.SVDU_OPT_PERSISTENT, 0) == 1
    assert svdu.svdu_set_option(ctx, svdu.SVDU_OPT_SLICES, 8) == 7
    assert svdu.svdu_set_option(ctx, svdu.SVDU_OPT_SLICES, 5) == svdu.SVDU_EINVAL
    assert svdu.svdu_set_option(ctx, svdu.SVDU_OPT_SLICES, 9) == svdu.SVDU_EINVAL
    assert svdu.svdu_set_option(ctx, svdu.SVDU_OPT_SLICES, 7) == 8
    assert svdu.svdu_set_option(ctx, svdu.SVDU_OPT_SECULAR_FMM, 0) == 1     # on above order 2048 by default
    assert svdu.svdu_set_option(ctx, svdu.SVDU_OPT_SECULAR_FMM, 2) == 0
    assert svdu.svdu_set_option(ctx, svdu.SVDU_OPT_SECULAR_FMM, 3) == svdu.SVDU_EINVAL
    assert svdu.svdu_set_option(ctx, svdu.SVDU_OPT_SECULAR_FMM, -1) == svdu.SVDU_EINVAL
    assert svdu.svdu_set_option(ctx, svdu.SVDU_OPT_SECULAR_FMM, 1) == 2


def _table(ctx, prec, new=None):
    buf = (ctypes.c_int * svdu.SVDU_TILE_BUCKETS)(*(new or [0] * svdu.SVDU_TILE_BUCKETS))
    rc = svdu.svdu_tile_table(ctx, prec, ctypes.cast(buf, ctypes.c_void_p), 1 if new is not None else 0)
    return rc, list(buf)


def test_tile_table_roundtrip(lib, ctx):
    rc, t = _table(ctx, svdu.SVDU_PREC_FP64)
    assert rc == svdu.SVDU_OK
    assert len(t) == svdu.SVDU_TILE_BUCKETS and all(0 <= x < svdu.SVDU_TILE_SHAPES for x in t)
    new = [(x + 1) % svdu.SVDU_TILE_SHAPES for x in t]
    assert _table(ctx, svdu.SVDU_PREC_FP64, new) == (svdu.SVDU_OK, new)
    assert _table(ctx, svdu.SVDU_PREC_FP64)[1] == new
    # another context keeps the built-in table
    other = ctypes.c_void_p()
    assert svdu.svdu_create(ctypes.byref(other), 0) == svdu.SVDU_OK
    assert _table(other, svdu.SVDU_PREC_FP64)[1] == t
    svdu.svdu_destroy(other)
    _table(ctx, svdu.SVDU_PREC_FP64, t)
    bad = (ctypes.c_int * svdu.SVDU_TILE_BUCKETS)(*([0] * 7 + [9]))
    assert svdu.svdu_tile_table(ctx, svdu.SVDU_PREC_FP64, ctypes.cast(bad, ctypes.c_void_p), 1) == svdu.SVDU_EINVAL
    assert svdu.svdu_tile_table(None, svdu.SVDU_PREC_FP64, ctypes.cast(bad, ctypes.c_void_p), 0) == svdu.SVDU_EINVAL
    assert _table(ctx, svdu.SVDU_PREC_FP64)[1] == t


def _prob(m, n, base, ld_extra=0, defl=False):
    """A problem whose buffers are fake, disjoint device addresses starting at base."""
    P = svdu.svdu_problem()
    P.m, P.n = m, n
    off = [base]

    def take(nbytes):
        p = off[0]
        off[0] += (nbytes + 255) // 256 * 256
        return p

    P.ldu, P.ldv, P.ldu_out, P.ldv_out = m + ld_extra, n + ld_extra, m, n
    P.U = take(8 * m * P.ldu)
    P.sigma = take(8 * m)
    P.V = take(8 * n * P.ldv)
    P.a = take(8 * m)
    P.b = take(8 * n)
    P.U_out = take(8 * m * m)
    P.sigma_out = take(8 * m)
    P.V_out = take(8 * n * n)
    P.defl = take(4 * n) if defl else None
    return P, off[0]


def test_batch_workspace_and_argument_errors(lib, ctx):
    """Host-side checks of the batched entry points (nothing reaches the device)."""
    arr = (svdu.svdu_problem * 3)()
    base = 0x10000000
    for i, (m, n) in enumerate([(64, 100), (17, 17), (300, 555)]):
        arr[i], base = _prob(m, n, base, defl=i == 1)
    wsb = svdu.svdu_batch_workspace_bytes(3, arr, svdu.SVDU_PREC_FP64)
    single = sum(svdu.svdu_workspace_bytes(arr[i].m, arr[i].n) for i in range(3))
    assert wsb > 0 and wsb >= single - 3 * 32768
    assert svdu.svdu_batch_workspace_bytes(3, arr, svdu.SVDU_PREC_SPLIT32) > 0
    assert svdu.svdu_batch_workspace_bytes(3, arr, svdu.SVDU_PREC_SLICED_INT8) > wsb
    assert svdu.svdu_batch_workspace_bytes(0, arr, 0) == 0
    ws = base + 0x100000
    h = ctypes.c_void_p()

    def create(a, count=3, prec=svdu.SVDU_PREC_FP64, flags=0, w=ws, wb=None):
        return svdu.svdu_batch_create(ctx, ctypes.byref(h), count, a, prec, flags, _p(w), wsb if wb is None else wb,
                                      None)

    assert create(arr, wb=wsb - 1) == svdu.SVDU_ENOMEM
    assert create(arr, w=ws + 8) == svdu.SVDU_EINVAL        # alignment
    assert create(arr, prec=7) == svdu.SVDU_EINVAL
    assert create(arr, flags=4) == svdu.SVDU_EINVAL
    assert create(arr, count=0) == svdu.SVDU_EINVAL
    assert h.value is None
    # an output overlapping another problem's input
    bad = (svdu.svdu_problem * 3)(*arr)
    bad[2].U_out = arr[0].V
    assert create(bad) == svdu.SVDU_EINVAL
    # two outputs overlapping
    bad = (svdu.svdu_problem * 3)(*arr)
    bad[1].sigma_out = arr[0].sigma_out
    assert create(bad) == svdu.SVDU_EINVAL
    # an input inside the workspace
    bad = (svdu.svdu_problem * 3)(*arr)
    bad[0].a = ws + 4096
    assert create(bad) == svdu.SVDU_EINVAL
    # m > n, small leading dimension
    bad = (svdu.svdu_problem * 3)(*arr)
    bad[1].m = 18
    assert create(bad) == svdu.SVDU_EINVAL
    bad = (svdu.svdu_problem * 3)(*arr)
    bad[2].ldv_out = 554
    assert create(bad) == svdu.SVDU_EINVAL
    assert svdu.svdu_batch_launch(None, 0, None) == svdu.SVDU_EINVAL
    assert svdu.svdu_batch_status(None, None, None) == svdu.SVDU_EINVAL
    svdu.svdu_batch_destroy(None)
    assert svdu.svdu_autotune_workspace_bytes(0) == 0
    assert svdu.svdu_autotune_workspace_bytes(256) > 8 * 256 * 256
    assert svdu.svdu_autotune(ctx, 5, 256, None, None, _p(ws), 1 << 30, None) == svdu.SVDU_EINVAL
    assert svdu.svdu_autotune(ctx, 0, 256, None, None, _p(ws), 16, None) == svdu.SVDU_ENOMEM
    assert svdu.svdu_autotune(None, 0, 256, None, None, _p(ws), 1 << 30, None) == svdu.SVDU_EINVAL
    assert svdu.svdu_batch_create(None, ctypes.byref(h), 3, arr, 0, 0, _p(ws), wsb, None) == svdu.SVDU_EINVAL


def test_server_argument_errors(lib, ctx):
    """Server configuration checks happen on the host before any device call."""
    h = ctypes.c_void_p()
    arena = _p(0x7000000000)

    def create(**kw):
        c = dict(workers=2, max_batch=8, precision=0, fmm_min_n=0, fmm_eps=1e-10, batch_cost_factor=2.0,
                 min_batch_cost=0.0, min_cost_ratio=0.25)
        c.update(kw)
        cfg = svdu.svdu_server_config(c["workers"], c["max_batch"], c["precision"], c["fmm_min_n"], c["fmm_eps"],
                                      c["batch_cost_factor"], c["min_batch_cost"], c["min_cost_ratio"])
        return svdu.svdu_server_create(kw.get("ctx", ctx), ctypes.byref(h), ctypes.byref(cfg), kw.get("arena", arena),
                                       kw.get("bytes", 1 << 30))

    assert create(workers=0) == svdu.SVDU_EINVAL
    assert create(workers=9) == svdu.SVDU_EINVAL
    assert create(max_batch=0) == svdu.SVDU_EINVAL
    assert create(precision=3) == svdu.SVDU_EINVAL
    assert create(fmm_min_n=100, fmm_eps=0.0) == svdu.SVDU_EINVAL
    assert create(batch_cost_factor=0.5) == svdu.SVDU_EINVAL
    assert create(min_batch_cost=-1.0) == svdu.SVDU_EINVAL
    assert create(min_cost_ratio=1.5) == svdu.SVDU_EINVAL
    assert create(arena=_p(0x7000000008)) == svdu.SVDU_EINVAL
    assert create(bytes=1000) == svdu.SVDU_EINVAL
    assert svdu.svdu_server_create(ctx, ctypes.byref(h), None, arena, 1 << 30) == svdu.SVDU_EINVAL
    assert create(ctx=None) == svdu.SVDU_EINVAL
    assert h.value is None
    assert svdu.svdu_server_start(None) == svdu.SVDU_EINVAL
    assert svdu.svdu_server_submit(None, 0, _p(8), _p(8), 0.0, None) == svdu.SVDU_EINVAL
    assert svdu.svdu_server_poll(None, None, 0) == svdu.SVDU_EINVAL
    assert svdu.svdu_server_drain(None, 1.0) == svdu.SVDU_EINVAL
    svdu.svdu_server_destroy(None)
