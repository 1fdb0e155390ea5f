"""Python binding of libsvdu, the rank-1 SVD update library for MI355X (gfx950).

Argument marshalling only: every step of the update runs in the HIP kernels
of ``libsvdu.so``. Tensors are torch CUDA (HIP) float64 tensors, row-major with
unit column stride; torch provides device memory and the stream.

The functions named ``svdu_*`` mirror the C ABI in ``include/svdu.h`` one to
one. ``rank1_update``, ``eig_update`` and ``secular`` allocate outputs and a
workspace and raise on a non-zero status.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsvdu.so")

SVDU_OK = 0
SVDU_EINVAL = -1
SVDU_ENOMEM = -2
SVDU_EHIP = -3
SVDU_ENONFINITE = -4
SVDU_EBADSIGMA = -5
SVDU_ENOCONV = -6
SVDU_ENOTSUP = -7
SVDU_PATH_DIRECT = 0
SVDU_PATH_FMM = 1
SVDU_PREC_FP64 = 0
SVDU_PREC_SPLIT32 = 1
SVDU_PREC_SLICED_INT8 = 2
SVDU_OPT_SECULAR_MAXIT = 1
SVDU_OPT_TIMING = 2
SVDU_OPT_TILE_SHAPE = 3
SVDU_OPT_PERSISTENT = 4
SVDU_OPT_REFINE = 5
SVDU_OPT_SLICES = 6
SVDU_OPT_SECULAR_FMM = 7
SVDU_TILE_128x128 = 0
SVDU_TILE_64x128 = 1
SVDU_TILE_128x64 = 2
SVDU_TILE_64x64 = 3
SVDU_TILE_128x128_K32 = 4
SVDU_TILE_256x128_K64 = 5
SVDU_TILE_SHAPES = 6
SVDU_TILE_BUCKETS = 8
SVDU_BATCH_PERSISTENT = 1
TIMING_PHASES = 5

EXPORTS = ("svdu_create", "svdu_destroy", "svdu_workspace_bytes", "svdu_rank1_update", "svdu_get_status", "svdu_eig_update_workspace_bytes",
           "svdu_eig_update", "svdu_secular_workspace_bytes", "svdu_secular", "svdu_set_option",
           "svdu_status_string", "svdu_timing_read", "svdu_batch_workspace_bytes", "svdu_batch_create",
           "svdu_batch_launch", "svdu_batch_status", "svdu_batch_destroy", "svdu_rank1_update_batched",
           "svdu_autotune_workspace_bytes", "svdu_autotune", "svdu_tile_table", "svdu_server_create",
           "svdu_server_add_matrix", "svdu_server_start", "svdu_server_now", "svdu_server_submit",
           "svdu_server_poll", "svdu_server_stats", "svdu_server_drain", "svdu_server_current",
           "svdu_server_destroy", "svdu_rank1_update_noalloc", "svdu_rankk_workspace_bytes", "svdu_rankk_update")
SVDU_NOALLOC_SCRATCH_BYTES = 32 << 20


class svdu_problem(ctypes.Structure):
    """Mirror of the C struct svdu_problem (include/svdu.h)."""
    _fields_ = [("m", ctypes.c_int), ("n", ctypes.c_int),
                ("U", ctypes.c_void_p), ("ldu", ctypes.c_int),
                ("sigma", ctypes.c_void_p),
                ("V", ctypes.c_void_p), ("ldv", ctypes.c_int),
                ("a", ctypes.c_void_p), ("b", ctypes.c_void_p),
                ("U_out", ctypes.c_void_p), ("ldu_out", ctypes.c_int),
                ("sigma_out", ctypes.c_void_p),
                ("V_out", ctypes.c_void_p), ("ldv_out", ctypes.c_int),
                ("defl", ctypes.c_void_p)]



class svdu_server_config(ctypes.Structure):
    """Mirror of the C struct svdu_server_config (include/svdu.h)."""
    _fields_ = [("workers", ctypes.c_int), ("max_batch", ctypes.c_int), ("precision", ctypes.c_int),
                ("fmm_min_n", ctypes.c_int), ("fmm_eps", ctypes.c_double),
                ("batch_cost_factor", ctypes.c_double), ("min_batch_cost", ctypes.c_double),
                ("min_cost_ratio", ctypes.c_double)]


class svdu_completion(ctypes.Structure):
    """Mirror of the C struct svdu_completion (include/svdu.h)."""
    _fields_ = [("id", ctypes.c_longlong), ("matrix", ctypes.c_int), ("status", ctypes.c_int),
                ("batch", ctypes.c_int), ("t_release", ctypes.c_double), ("t_start", ctypes.c_double),
                ("t_done", ctypes.c_double)]


_lib = None


class SvduError(RuntimeError):
    def __init__(self, code: int, where: str):
        super().__init__(f"{where}: {svdu_status_string(code)} ({code})")
        self.code = code


def load():
    """Load libsvdu.so; raises if it has not been built (no fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
    lib = ctypes.CDLL(LIB_PATH)
    c_int, c_size, c_dbl, c_vp = ctypes.c_int, ctypes.c_size_t, ctypes.c_double, ctypes.c_void_p
    lib.svdu_create.argtypes = [ctypes.POINTER(c_vp), c_int]
    lib.svdu_create.restype = c_int
    lib.svdu_destroy.argtypes = [c_vp]
    lib.svdu_destroy.restype = None
    lib.svdu_workspace_bytes.argtypes = [c_int, c_int, c_int, c_int]
    lib.svdu_workspace_bytes.restype = c_size
    lib.svdu_rank1_update.argtypes = [c_vp, c_int, c_int, c_vp, c_int, c_vp, c_vp, c_int, c_vp, c_vp, c_dbl, c_int, c_int,
                                      c_vp, c_int, c_vp, c_vp, c_int, c_vp, c_vp, c_size, c_vp]
    lib.svdu_rank1_update.restype = c_int
    lib.svdu_rank1_update_noalloc.argtypes = [c_vp, c_int, c_int, c_vp, c_int, c_vp, c_vp, c_int, c_vp, c_vp, c_int,
                                              c_vp, c_int, c_vp, c_vp, c_int, c_vp, c_vp, c_vp]
    lib.svdu_rank1_update_noalloc.restype = c_int
    lib.svdu_rankk_workspace_bytes.argtypes = [c_int, c_int, c_int, c_int, c_int]
    lib.svdu_rankk_workspace_bytes.restype = c_size
    lib.svdu_rankk_update.argtypes = [c_vp, c_int, c_int, c_int, c_vp, c_int, c_vp, c_vp, c_int, c_vp, c_int, c_vp,
                                      c_int, c_dbl, c_int, c_int, c_vp, c_int, c_vp, c_vp, c_int, c_vp, c_size, c_vp]
    lib.svdu_rankk_update.restype = c_int
    lib.svdu_get_status.argtypes = [c_vp, c_vp]
    lib.svdu_get_status.restype = c_int
    lib.svdu_eig_update_workspace_bytes.argtypes = [c_int, c_int, c_int]
    lib.svdu_eig_update_workspace_bytes.restype = c_size
    lib.svdu_eig_update.argtypes = [c_vp, c_int, c_int, c_vp, c_int, c_vp, c_vp, c_dbl, c_int, c_dbl, c_vp, c_int, c_vp,
                                    c_vp, c_vp, c_size, c_vp]
    lib.svdu_eig_update.restype = c_int
    lib.svdu_secular_workspace_bytes.argtypes = [c_int]
    lib.svdu_secular_workspace_bytes.restype = c_size
    lib.svdu_secular.argtypes = [c_vp, c_int, c_vp, c_vp, c_dbl, c_vp, c_vp, c_vp, c_vp, c_size, c_vp]
    lib.svdu_secular.restype = c_int
    lib.svdu_set_option.argtypes = [c_vp, c_int, c_int]
    lib.svdu_set_option.restype = c_int
    lib.svdu_timing_read.argtypes = [c_vp, c_vp, c_int]
    lib.svdu_timing_read.restype = c_int
    lib.svdu_status_string.argtypes = [c_int]
    lib.svdu_status_string.restype = ctypes.c_char_p
    c_pp = ctypes.POINTER(svdu_problem)
    lib.svdu_batch_workspace_bytes.argtypes = [c_int, c_pp, c_int]
    lib.svdu_batch_workspace_bytes.restype = c_size
    lib.svdu_batch_create.argtypes = [c_vp, ctypes.POINTER(c_vp), c_int, c_pp, c_int, c_int, c_vp, c_size, c_vp]
    lib.svdu_batch_create.restype = c_int
    lib.svdu_batch_launch.argtypes = [c_vp, c_int, c_vp]
    lib.svdu_batch_launch.restype = c_int
    lib.svdu_batch_status.argtypes = [c_vp, c_vp, c_vp]
    lib.svdu_batch_status.restype = c_int
    lib.svdu_batch_destroy.argtypes = [c_vp]
    lib.svdu_batch_destroy.restype = None
    lib.svdu_rank1_update_batched.argtypes = [c_vp, c_int, c_pp, c_int, c_vp, c_size, c_vp]
    lib.svdu_rank1_update_batched.restype = c_int
    lib.svdu_autotune_workspace_bytes.argtypes = [c_int]
    lib.svdu_autotune_workspace_bytes.restype = c_size
    lib.svdu_autotune.argtypes = [c_vp, c_int, c_int, c_vp, c_vp, c_vp, c_size, c_vp]
    lib.svdu_autotune.restype = c_int
    lib.svdu_tile_table.argtypes = [c_vp, c_int, c_vp, c_int]
    lib.svdu_tile_table.restype = c_int
    lib.svdu_server_create.argtypes = [c_vp, ctypes.POINTER(c_vp), ctypes.POINTER(svdu_server_config), c_vp, c_size]
    lib.svdu_server_create.restype = c_int
    lib.svdu_server_add_matrix.argtypes = [c_vp, c_int, c_int, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp,
                                           ctypes.POINTER(c_int)]
    lib.svdu_server_add_matrix.restype = c_int
    lib.svdu_server_start.argtypes = [c_vp]
    lib.svdu_server_start.restype = c_int
    lib.svdu_server_now.argtypes = [c_vp]
    lib.svdu_server_now.restype = c_dbl
    lib.svdu_server_submit.argtypes = [c_vp, c_int, c_vp, c_vp, c_dbl, ctypes.POINTER(ctypes.c_longlong)]
    lib.svdu_server_submit.restype = c_int
    lib.svdu_server_poll.argtypes = [c_vp, ctypes.POINTER(svdu_completion), c_int]
    lib.svdu_server_poll.restype = c_int
    lib.svdu_server_stats.argtypes = [c_vp, ctypes.POINTER(ctypes.c_longlong)]
    lib.svdu_server_stats.restype = c_int
    lib.svdu_server_drain.argtypes = [c_vp, c_dbl]
    lib.svdu_server_drain.restype = c_int
    lib.svdu_server_current.argtypes = [c_vp, c_int, ctypes.POINTER(c_vp), ctypes.POINTER(c_vp),
                                        ctypes.POINTER(c_vp)]
    lib.svdu_server_current.restype = c_int
    lib.svdu_server_destroy.argtypes = [c_vp]
    lib.svdu_server_destroy.restype = None
    _lib = lib
    return lib


# ---------------------------------------------------------------------------
# one-to-one wrappers of the C ABI (raw pointers / ints)
# ---------------------------------------------------------------------------
def svdu_workspace_bytes(m, n, path=SVDU_PATH_DIRECT, precision=SVDU_PREC_FP64) -> int:
    return int(load().svdu_workspace_bytes(m, n, path, precision))


def svdu_create(ctx_out, device) -> int:
    return int(load().svdu_create(ctx_out, device))


def svdu_destroy(ctx) -> None:
    load().svdu_destroy(ctx)


def svdu_rank1_update(ctx, m, n, U, ldu, sigma, V, ldv, a, b, eps, path, precision, U_out, ldu_out, sigma_out,
                      V_out, ldv_out, defl, workspace, workspace_bytes, stream) -> int:
    return int(load().svdu_rank1_update(ctx, m, n, U, ldu, sigma, V, ldv, a, b, eps, path, precision, U_out, ldu_out,
                                        sigma_out, V_out, ldv_out, defl, workspace, workspace_bytes, stream))


def svdu_rank1_update_noalloc(ctx, m, n, U, ldu, sigma, V, ldv, a, b, precision, U_out, ldu_out, sigma_out,
                              V_out, ldv_out, defl, status, stream) -> int:
    return int(load().svdu_rank1_update_noalloc(ctx, m, n, U, ldu, sigma, V, ldv, a, b, precision, U_out, ldu_out,
                                                sigma_out, V_out, ldv_out, defl, status, stream))


def svdu_rankk_workspace_bytes(m, n, k, path=SVDU_PATH_DIRECT, precision=SVDU_PREC_FP64) -> int:
    return int(load().svdu_rankk_workspace_bytes(m, n, k, path, precision))


def svdu_rankk_update(ctx, m, n, k, U, ldu, sigma, V, ldv, A, lda, B, ldb, eps, path, precision, U_out, ldu_out,
                      sigma_out, V_out, ldv_out, workspace, workspace_bytes, stream) -> int:
    return int(load().svdu_rankk_update(ctx, m, n, k, U, ldu, sigma, V, ldv, A, lda, B, ldb, eps, path, precision,
                                        U_out, ldu_out, sigma_out, V_out, ldv_out, workspace, workspace_bytes,
                                        stream))


def svdu_get_status(workspace, stream) -> int:
    return int(load().svdu_get_status(workspace, stream))


def svdu_eig_update_workspace_bytes(R, N, path=SVDU_PATH_DIRECT) -> int:
    return int(load().svdu_eig_update_workspace_bytes(R, N, path))


def svdu_eig_update(ctx, R, N, X, ldx, lam, z, rho, path, eps, X_out, ldo, lam_out, defl, workspace,
                    workspace_bytes, stream) -> int:
    return int(load().svdu_eig_update(ctx, R, N, X, ldx, lam, z, rho, path, eps, X_out, ldo, lam_out, defl, workspace,
                                      workspace_bytes, stream))


def svdu_secular_workspace_bytes(K) -> int:
    return int(load().svdu_secular_workspace_bytes(K))


def svdu_secular(ctx, K, d, z, rho, org, tau, iters, workspace, workspace_bytes, stream) -> int:
    return int(load().svdu_secular(ctx, K, d, z, rho, org, tau, iters, workspace, workspace_bytes, stream))


def svdu_set_option(ctx, option, value) -> int:
    return int(load().svdu_set_option(ctx, option, value))


def svdu_timing_read(ctx, ms, max_calls) -> int:
    return int(load().svdu_timing_read(ctx, ms, max_calls))


class Context:
    """A libsvdu context (svdu_create / svdu_destroy): options, tile tables and
    the timing record of the calls made with it, bound to one device."""

    def __init__(self, device=None):
        torch = _torch()
        dev = torch.cuda.current_device() if device is None else int(device)
        h = ctypes.c_void_p()
        rc = svdu_create(ctypes.byref(h), dev)
        if rc != SVDU_OK:
            raise SvduError(rc, "svdu_create")
        self._h = h
        self.device = dev

    @property
    def handle(self):
        return self._h

    def set_option(self, option, value):
        """Sets an option; returns the previous value (or SVDU_EINVAL)."""
        return svdu_set_option(self._h, option, value)

    def close(self):
        if getattr(self, "_h", None):
            svdu_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_default_ctx = {}


def default_context(device=None):
    """The context the helpers below use when none is given (one per device)."""
    torch = _torch()
    dev = torch.cuda.current_device() if device is None else int(device)
    c = _default_ctx.get(dev)
    if c is None:
        c = _default_ctx[dev] = Context(dev)
    return c


def _ctx(ctx):
    return (ctx if ctx is not None else default_context()).handle


def set_option(option, value, ctx=None) -> int:
    """Sets an option of ``ctx`` (default: the default context); returns the previous value."""
    return svdu_set_option(_ctx(ctx), option, value)


def timing_read(max_calls=256, ctx=None):
    """Phase timings (ms) of the calls recorded since SVDU_OPT_TIMING was set: list of 5-tuples."""
    P = TIMING_PHASES
    buf = (ctypes.c_double * (P * max_calls))()
    n = svdu_timing_read(_ctx(ctx), ctypes.cast(buf, ctypes.c_void_p), max_calls)
    if n < 0:
        raise SvduError(n, "svdu_timing_read")
    return [tuple(buf[P * c + k] for k in range(P)) for c in range(n)]


def svdu_batch_workspace_bytes(count, probs, precision) -> int:
    return int(load().svdu_batch_workspace_bytes(count, probs, precision))


def svdu_batch_create(ctx, out, count, probs, precision, flags, workspace, workspace_bytes, stream) -> int:
    return int(load().svdu_batch_create(ctx, out, count, probs, precision, flags, workspace, workspace_bytes, stream))


def svdu_batch_launch(batch, use_graph, stream) -> int:
    return int(load().svdu_batch_launch(batch, use_graph, stream))


def svdu_batch_status(batch, status, stream) -> int:
    return int(load().svdu_batch_status(batch, status, stream))


def svdu_batch_destroy(batch) -> None:
    load().svdu_batch_destroy(batch)


def svdu_rank1_update_batched(ctx, count, probs, precision, workspace, workspace_bytes, stream) -> int:
    return int(load().svdu_rank1_update_batched(ctx, count, probs, precision, workspace, workspace_bytes, stream))


def svdu_autotune_workspace_bytes(max_n) -> int:
    return int(load().svdu_autotune_workspace_bytes(max_n))


def svdu_autotune(ctx, precision, max_n, times_ms, table, workspace, workspace_bytes, stream) -> int:
    return int(load().svdu_autotune(ctx, precision, max_n, times_ms, table, workspace, workspace_bytes, stream))


def svdu_tile_table(ctx, precision, table, set_) -> int:
    return int(load().svdu_tile_table(ctx, precision, table, set_))


def svdu_status_string(code) -> str:
    return load().svdu_status_string(code).decode()


# ---------------------------------------------------------------------------
# tensor-level helpers
# ---------------------------------------------------------------------------
def _torch():
    import torch
    return torch


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream_handle(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _check_mat(x, rows, cols, name):
    torch = _torch()
    if x.dtype != torch.float64 or not x.is_cuda or x.dim() != 2:
        raise ValueError(f"{name} must be a 2-D float64 device tensor")
    if x.shape[0] != rows or x.shape[1] != cols or (cols > 1 and x.stride(1) != 1):
        raise ValueError(f"{name} must be {rows} x {cols} with unit column stride")
    return max(x.stride(0), cols)


def _check_vec(x, n, name):
    torch = _torch()
    if x.dtype != torch.float64 or not x.is_cuda or x.dim() != 1 or x.shape[0] != n or x.stride(0) != 1:
        raise ValueError(f"{name} must be a contiguous float64 device vector of length {n}")


def new_workspace(nbytes, device):
    torch = _torch()
    return torch.empty(nbytes + 256, dtype=torch.uint8, device=device)


def _aligned(ws):
    p = ws.data_ptr()
    off = (-p) % 256
    return ctypes.c_void_p(p + off), ws.numel() - off


def rank1_update(U, sigma, V, a, b, eps=1e-10, path=SVDU_PATH_DIRECT, precision=SVDU_PREC_FP64, out=None,
                 workspace=None, want_defl=True, stream=None, check=True, ctx=None):
    """SVD of U diag(sigma) V^T + a b^T. Returns (U^, sigma^, V^, defl flags or None).

    ``out`` may pass preallocated (U_out, sigma_out, V_out); ``workspace`` a uint8
    device tensor of at least svdu_workspace_bytes(m, n) + 256 bytes.
    """
    torch = _torch()
    m, n = U.shape[0], V.shape[0]
    ldu = _check_mat(U, m, m, "U")
    ldv = _check_mat(V, n, n, "V")
    _check_vec(sigma, m, "sigma")
    _check_vec(a, m, "a")
    _check_vec(b, n, "b")
    dev = U.device
    if out is None:
        Uo = torch.empty((m, m), dtype=torch.float64, device=dev)
        so = torch.empty(m, dtype=torch.float64, device=dev)
        Vo = torch.empty((n, n), dtype=torch.float64, device=dev)
    else:
        Uo, so, Vo = out
    lduo = _check_mat(Uo, m, m, "U_out")
    ldvo = _check_mat(Vo, n, n, "V_out")
    _check_vec(so, m, "sigma_out")
    need = svdu_workspace_bytes(m, n, path, precision)
    if workspace is None:
        workspace = new_workspace(need, dev)
    wp, wb = _aligned(workspace)
    defl = torch.empty((4, n), dtype=torch.int8, device=dev) if want_defl else None
    sh = _stream_handle(stream)
    rc = svdu_rank1_update(_ctx(ctx), m, n, _ptr(U), ldu, _ptr(sigma), _ptr(V), ldv, _ptr(a), _ptr(b), float(eps), path,
                           precision, _ptr(Uo), lduo, _ptr(so), _ptr(Vo), ldvo, _ptr(defl), wp, wb, sh)
    if rc != SVDU_OK:
        raise SvduError(rc, "svdu_rank1_update")
    if check:
        rc = svdu_get_status(wp, sh)
        if rc != SVDU_OK:
            raise SvduError(rc, "svdu_rank1_update (device)")
    return Uo, so, Vo, defl


def rank1_update_noalloc(U, sigma, V, a, b, precision=SVDU_PREC_FP64, out=None, want_defl=True, stream=None,
                         check=True, ctx=None):
    """rank1_update on the direct path through svdu_rank1_update_noalloc (no
    workspace: the library's per-device scratch array). Returns (U^, sigma^,
    V^, defl flags or None)."""
    torch = _torch()
    m, n = U.shape[0], V.shape[0]
    ldu = _check_mat(U, m, m, "U")
    ldv = _check_mat(V, n, n, "V")
    _check_vec(sigma, m, "sigma")
    _check_vec(a, m, "a")
    _check_vec(b, n, "b")
    dev = U.device
    if out is None:
        Uo = torch.empty((m, m), dtype=torch.float64, device=dev)
        so = torch.empty(m, dtype=torch.float64, device=dev)
        Vo = torch.empty((n, n), dtype=torch.float64, device=dev)
    else:
        Uo, so, Vo = out
    lduo = _check_mat(Uo, m, m, "U_out")
    ldvo = _check_mat(Vo, n, n, "V_out")
    _check_vec(so, m, "sigma_out")
    defl = torch.empty((4, n), dtype=torch.int8, device=dev) if want_defl else None
    st = torch.full((1,), -99, dtype=torch.int32, device=dev) if check else None
    sh = _stream_handle(stream)
    rc = svdu_rank1_update_noalloc(_ctx(ctx), m, n, _ptr(U), ldu, _ptr(sigma), _ptr(V), ldv, _ptr(a), _ptr(b),
                                   precision, _ptr(Uo), lduo, _ptr(so), _ptr(Vo), ldvo, _ptr(defl), _ptr(st), sh)
    if rc != SVDU_OK:
        raise SvduError(rc, "svdu_rank1_update_noalloc")
    if check:
        (stream if stream is not None else torch.cuda.current_stream()).synchronize()
        code = int(st.item())
        if code != SVDU_OK:
            raise SvduError(code, "svdu_rank1_update_noalloc (device)")
    return Uo, so, Vo, defl


def rankk_update(U, sigma, V, A, B, eps=1e-10, path=SVDU_PATH_DIRECT, precision=SVDU_PREC_FP64, out=None,
                 stream=None, check=True, ctx=None):
    """SVD of U diag(sigma) V^T + A^T B for A (k x m) and B (k x n): row j of A
    and B is the pair (a_j, b_j). Returns (U^, sigma^, V^)."""
    torch = _torch()
    m, n = U.shape[0], V.shape[0]
    ldu = _check_mat(U, m, m, "U")
    ldv = _check_mat(V, n, n, "V")
    _check_vec(sigma, m, "sigma")
    k = A.shape[0]
    lda = _check_mat(A, k, m, "A")
    ldb = _check_mat(B, k, n, "B")
    dev = U.device
    if out is None:
        Uo = torch.empty((m, m), dtype=torch.float64, device=dev)
        so = torch.empty(m, dtype=torch.float64, device=dev)
        Vo = torch.empty((n, n), dtype=torch.float64, device=dev)
    else:
        Uo, so, Vo = out
    lduo = _check_mat(Uo, m, m, "U_out")
    ldvo = _check_mat(Vo, n, n, "V_out")
    _check_vec(so, m, "sigma_out")
    ws = new_workspace(svdu_rankk_workspace_bytes(m, n, k, path, precision), dev)
    wp, wb = _aligned(ws)
    sh = _stream_handle(stream)
    rc = svdu_rankk_update(_ctx(ctx), m, n, k, _ptr(U), ldu, _ptr(sigma), _ptr(V), ldv, _ptr(A), lda, _ptr(B), ldb,
                           float(eps), path, precision, _ptr(Uo), lduo, _ptr(so), _ptr(Vo), ldvo, wp, wb, sh)
    if rc != SVDU_OK:
        raise SvduError(rc, "svdu_rankk_update")
    if check:
        rc = svdu_get_status(wp, sh)
        if rc != SVDU_OK:
            raise SvduError(rc, "svdu_rankk_update (device)")
    return Uo, so, Vo


def eig_update(X, lam, z, rho, path=SVDU_PATH_DIRECT, eps=1e-10, stream=None, check=True, ctx=None):
    """One RankOneUpdate: returns (X C~, new eigenvalues ascending, flags)."""
    torch = _torch()
    R, N = X.shape
    ldx = _check_mat(X, R, N, "X")
    _check_vec(lam, N, "lam")
    _check_vec(z, N, "z")
    Xo = torch.empty((R, N), dtype=torch.float64, device=X.device)
    lo = torch.empty(N, dtype=torch.float64, device=X.device)
    fl = torch.empty(N, dtype=torch.int8, device=X.device)
    ws = new_workspace(svdu_eig_update_workspace_bytes(R, N, path), X.device)
    wp, wb = _aligned(ws)
    sh = _stream_handle(stream)
    rc = svdu_eig_update(_ctx(ctx), R, N, _ptr(X), ldx, _ptr(lam), _ptr(z), float(rho), path, float(eps), _ptr(Xo), max(N, 1),
                         _ptr(lo), _ptr(fl), wp, wb, sh)
    if rc != SVDU_OK:
        raise SvduError(rc, "svdu_eig_update")
    if check:
        rc = svdu_get_status(wp, sh)
        if rc != SVDU_OK:
            raise SvduError(rc, "svdu_eig_update (device)")
    return Xo, lo, fl


def secular(d, z, rho, stream=None, check=True, ctx=None):
    """Roots of 1 + rho sum z^2/(d - mu) for distinct ascending d: (org, tau, iters)."""
    torch = _torch()
    K = d.shape[0]
    _check_vec(d, K, "d")
    _check_vec(z, K, "z")
    org = torch.empty(K, dtype=torch.int32, device=d.device)
    tau = torch.empty(K, dtype=torch.float64, device=d.device)
    its = torch.empty(K, dtype=torch.int32, device=d.device)
    ws = new_workspace(svdu_secular_workspace_bytes(K), d.device)
    wp, wb = _aligned(ws)
    sh = _stream_handle(stream)
    rc = svdu_secular(_ctx(ctx), K, _ptr(d), _ptr(z), float(rho), _ptr(org), _ptr(tau), _ptr(its), wp, wb, sh)
    if rc != SVDU_OK:
        raise SvduError(rc, "svdu_secular")
    if check:
        rc = svdu_get_status(wp, sh)
        if rc != SVDU_OK:
            raise SvduError(rc, "svdu_secular (device)")
    return org, tau, its


# ---------------------------------------------------------------------------
# batched updates
# ---------------------------------------------------------------------------
class Batch:
    """A batch of independent rank-1 updates (svdu_batch_* in include/svdu.h).

    ``items`` is a list of (U, sigma, V, a, b) device tensors. Outputs are
    allocated unless ``outs`` gives (U_out, sigma_out, V_out) per item. The batch
    keeps references to every tensor it names, and its workspace.
    """

    def __init__(self, items, precision=SVDU_PREC_FP64, persistent=False, outs=None, want_defl=False,
                 stream=None, ctx=None):
        torch = _torch()
        self._lib = load()
        self._ctx_obj = ctx if ctx is not None else default_context()   # must outlive the batch
        self.precision = precision
        self.items = list(items)
        self.count = len(self.items)
        if self.count < 1:
            raise ValueError("empty batch")
        self.outs = []
        self.defl = []
        arr = (svdu_problem * self.count)()
        for i, (U, sigma, V, a, b) in enumerate(self.items):
            m, n = U.shape[0], V.shape[0]
            ldu = _check_mat(U, m, m, "U")
            ldv = _check_mat(V, n, n, "V")
            _check_vec(sigma, m, "sigma")
            _check_vec(a, m, "a")
            _check_vec(b, n, "b")
            if outs is None:
                Uo = torch.empty((m, m), dtype=torch.float64, device=U.device)
                so = torch.empty(m, dtype=torch.float64, device=U.device)
                Vo = torch.empty((n, n), dtype=torch.float64, device=U.device)
            else:
                Uo, so, Vo = outs[i]
            lduo = _check_mat(Uo, m, m, "U_out")
            ldvo = _check_mat(Vo, n, n, "V_out")
            _check_vec(so, m, "sigma_out")
            d = torch.empty((4, n), dtype=torch.int8, device=U.device) if want_defl else None
            self.outs.append((Uo, so, Vo))
            self.defl.append(d)
            arr[i] = svdu_problem(m, n, U.data_ptr(), ldu, sigma.data_ptr(), V.data_ptr(), ldv, a.data_ptr(),
                                  b.data_ptr(), Uo.data_ptr(), lduo, so.data_ptr(), Vo.data_ptr(), ldvo,
                                  None if d is None else d.data_ptr())
        self._arr = arr
        need = svdu_batch_workspace_bytes(self.count, arr, precision)
        if need == 0:
            raise ValueError("invalid batch")
        self.workspace = new_workspace(need, self.items[0][0].device)
        wp, wb = _aligned(self.workspace)
        h = ctypes.c_void_p()
        rc = svdu_batch_create(self._ctx_obj.handle, ctypes.byref(h), self.count, arr, precision,
                               SVDU_BATCH_PERSISTENT if persistent else 0, wp, wb, _stream_handle(stream))
        if rc != SVDU_OK:
            raise SvduError(rc, "svdu_batch_create")
        self._h = h

    def launch(self, use_graph=False, stream=None):
        rc = svdu_batch_launch(self._h, 1 if use_graph else 0, _stream_handle(stream))
        if rc != SVDU_OK:
            raise SvduError(rc, "svdu_batch_launch")

    def status(self, stream=None):
        """Per-problem device status codes (waits for the stream)."""
        st = (ctypes.c_int * self.count)()
        rc = svdu_batch_status(self._h, ctypes.cast(st, ctypes.c_void_p), _stream_handle(stream))
        if rc == SVDU_EHIP:
            raise SvduError(rc, "svdu_batch_status")
        return list(st)

    def close(self):
        if getattr(self, "_h", None):
            svdu_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def rank1_update_batched(items, precision=SVDU_PREC_FP64, use_graph=False, persistent=False, stream=None,
                         check=True, ctx=None):
    """Updates every (U, sigma, V, a, b) of ``items`` in one batch; returns [(U^, sigma^, V^), ...]."""
    b = Batch(items, precision=precision, persistent=persistent, stream=stream, ctx=ctx)
    b.launch(use_graph=use_graph, stream=stream)
    if check:
        st = b.status(stream)
        bad = [(i, c) for i, c in enumerate(st) if c != SVDU_OK]
        if bad:
            raise SvduError(bad[0][1], f"batched update, problem {bad[0][0]}")
    outs = b.outs
    b.close()
    return outs


def autotune(precision=SVDU_PREC_FP64, max_n=4096, stream=None, ctx=None):
    """Runs the tile-shape autotuner; returns (table, times_ms[bucket][shape])."""
    torch = _torch()
    need = svdu_autotune_workspace_bytes(max_n)
    ws = new_workspace(need, torch.device("cuda"))
    wp, wb = _aligned(ws)
    times = (ctypes.c_double * (SVDU_TILE_BUCKETS * SVDU_TILE_SHAPES))()
    table = (ctypes.c_int * SVDU_TILE_BUCKETS)()
    rc = svdu_autotune(_ctx(ctx), precision, max_n, ctypes.cast(times, ctypes.c_void_p), ctypes.cast(table, ctypes.c_void_p),
                       wp, wb, _stream_handle(stream))
    if rc != SVDU_OK:
        raise SvduError(rc, "svdu_autotune")
    return list(table), [[times[b * SVDU_TILE_SHAPES + s] for s in range(SVDU_TILE_SHAPES)]
                         for b in range(SVDU_TILE_BUCKETS)]


def tile_table(precision=SVDU_PREC_FP64, table=None, ctx=None):
    """Reads the tuning table of ``ctx``, or sets it when ``table`` is given."""
    buf = (ctypes.c_int * SVDU_TILE_BUCKETS)(*(table or [0] * SVDU_TILE_BUCKETS))
    rc = svdu_tile_table(_ctx(ctx), precision, ctypes.cast(buf, ctypes.c_void_p), 1 if table is not None else 0)
    if rc != SVDU_OK:
        raise SvduError(rc, "svdu_tile_table")
    return list(buf)


# ---------------------------------------------------------------------------
# serving runtime
# ---------------------------------------------------------------------------
def svdu_server_create(ctx, out, cfg, arena, arena_bytes) -> int:
    return int(load().svdu_server_create(ctx, out, cfg, arena, arena_bytes))


def svdu_server_add_matrix(server, m, n, U0, s0, V0, U1, s1, V1, id_out) -> int:
    return int(load().svdu_server_add_matrix(server, m, n, U0, s0, V0, U1, s1, V1, id_out))


def svdu_server_start(server) -> int:
    return int(load().svdu_server_start(server))


def svdu_server_now(server) -> float:
    return float(load().svdu_server_now(server))


def svdu_server_submit(server, matrix, a, b, t_release, req_id) -> int:
    return int(load().svdu_server_submit(server, matrix, a, b, t_release, req_id))


def svdu_server_poll(server, out, max_out) -> int:
    return int(load().svdu_server_poll(server, out, max_out))


def svdu_server_stats(server, stats) -> int:
    return int(load().svdu_server_stats(server, stats))


def svdu_server_drain(server, timeout_s) -> int:
    return int(load().svdu_server_drain(server, timeout_s))


def svdu_server_current(server, matrix, U, s, V) -> int:
    return int(load().svdu_server_current(server, matrix, U, s, V))


def svdu_server_destroy(server) -> None:
    load().svdu_server_destroy(server)


class Server:
    """Serving runtime (svdu_server_* in include/svdu.h).

    Matrices are registered with their current factors (the tensors become the
    first buffer set; a second set is allocated here). Request vectors are kept
    referenced until their completion has been polled.
    """

    def __init__(self, arena_bytes, workers=2, max_batch=64, precision=SVDU_PREC_FP64, fmm_min_n=0,
                 fmm_eps=1e-10, batch_cost_factor=2.0, min_batch_cost=4e9, min_cost_ratio=0.25, ctx=None):
        torch = _torch()
        self._arena = new_workspace(int(arena_bytes), torch.device("cuda"))
        ap, ab = _aligned(self._arena)
        cfg = svdu_server_config(workers, max_batch, precision, fmm_min_n, fmm_eps, batch_cost_factor,
                                 min_batch_cost, min_cost_ratio)
        h = ctypes.c_void_p()
        rc = svdu_server_create(_ctx(ctx), ctypes.byref(h), ctypes.byref(cfg), ap, ab)
        if rc != SVDU_OK:
            raise SvduError(rc, "svdu_server_create")
        self._h = h
        self._sets = []
        self._live = {}

    def add_matrix(self, U, sigma, V):
        torch = _torch()
        m, n = U.shape[0], V.shape[0]
        _check_mat(U, m, m, "U")
        _check_mat(V, n, n, "V")
        _check_vec(sigma, m, "sigma")
        if U.stride(0) != m or V.stride(0) != n:
            raise ValueError("resident factors must be contiguous")
        s1 = (torch.empty_like(U), torch.empty_like(sigma), torch.empty_like(V))
        mid = ctypes.c_int()
        rc = svdu_server_add_matrix(self._h, m, n, _ptr(U), _ptr(sigma), _ptr(V), _ptr(s1[0]), _ptr(s1[1]),
                                    _ptr(s1[2]), ctypes.byref(mid))
        if rc != SVDU_OK:
            raise SvduError(rc, "svdu_server_add_matrix")
        self._sets.append(((U, sigma, V), s1))
        return mid.value

    def start(self):
        rc = svdu_server_start(self._h)
        if rc != SVDU_OK:
            raise SvduError(rc, "svdu_server_start")

    def now(self):
        return svdu_server_now(self._h)

    def submit(self, matrix, a, b, t_release=0.0):
        rid = ctypes.c_longlong()
        rc = svdu_server_submit(self._h, matrix, _ptr(a), _ptr(b), float(t_release), ctypes.byref(rid))
        if rc != SVDU_OK:
            raise SvduError(rc, "svdu_server_submit")
        self._live[rid.value] = (a, b)
        return rid.value

    def poll(self, max_out=4096):
        buf = (svdu_completion * max_out)()
        n = svdu_server_poll(self._h, buf, max_out)
        out = []
        for i in range(n):
            c = buf[i]
            self._live.pop(c.id, None)
            out.append(dict(id=c.id, matrix=c.matrix, status=c.status, batch=c.batch, t_release=c.t_release,
                            t_start=c.t_start, t_done=c.t_done))
        return out

    def stats(self):
        st = (ctypes.c_longlong * 6)()
        svdu_server_stats(self._h, st)
        return dict(queued=st[0], running=st[1], batches=st[2], updates=st[3], largest_free=st[4],
                    error=st[5])

    def drain(self, timeout_s=600.0):
        return svdu_server_drain(self._h, float(timeout_s))

    def current(self, matrix):
        """The tensors that hold the matrix's factors now (matrix idle)."""
        U, s, V = ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_void_p()
        rc = svdu_server_current(self._h, matrix, ctypes.byref(U), ctypes.byref(s), ctypes.byref(V))
        if rc != SVDU_OK:
            raise SvduError(rc, "svdu_server_current")
        for st in self._sets[matrix]:
            if st[0].data_ptr() == U.value:
                return st
        raise RuntimeError("unknown buffer set")

    def close(self):
        if getattr(self, "_h", None):
            svdu_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
