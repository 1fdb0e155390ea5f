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
    # the n x n intermediate basis dominates
    assert big >= 8192 * 8192 * 8
    assert big < 8192 * 8192 * 8 * 1.1
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


def test_host_argument_errors_return_before_enqueue(lib):
    fake = _p(0x10000)       # never dereferenced: every call below fails its host checks
    ws = _p(0x100000)
    args = dict(m=4, n=6, U=fake, ldu=4, sigma=fake, V=_p(0x20000), ldv=6, a=fake, b=fake, eps=1e-10, path=0,
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
    assert svdu.svdu_eig_update(3, 0, fake, 1, fake, fake, 1.0, 0, 0.0, _p(0x50000), 1, fake, None, ws, 1 << 20,
                                None) == svdu.SVDU_EINVAL
    assert svdu.svdu_eig_update(3, 4, fake, 4, fake, fake, 0.0, 0, 0.0, _p(0x50000), 4, fake, None, ws, 1 << 20,
                                None) == svdu.SVDU_EINVAL
    assert svdu.svdu_eig_update(3, 4, fake, 4, fake, fake, 1.0, 1, 0.0, _p(0x50000), 4, fake, None, ws, 1 << 20,
                                None) == svdu.SVDU_EINVAL   # FMM needs 0 < eps < 1
    assert svdu.svdu_secular(0, fake, fake, 1.0, fake, fake, None, ws, 1 << 20, None) == svdu.SVDU_EINVAL
    assert svdu.svdu_secular(4, fake, fake, 1.0, fake, fake, None, ws, 8, None) == svdu.SVDU_ENOMEM


def test_options(lib):
    old = svdu.svdu_set_option(svdu.SVDU_OPT_SECULAR_MAXIT, 17)
    assert svdu.svdu_set_option(svdu.SVDU_OPT_SECULAR_MAXIT, old) == 17
    assert svdu.svdu_set_option(999, 1) == svdu.SVDU_EINVAL
