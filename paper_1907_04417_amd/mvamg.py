"""Python binding of the C ABI in include/mvamg.h (ctypes, argument marshalling
only).  Every step of the solve runs in the HIP library ``libmvamg.so``; there
is no CPU fallback: if the library is missing or no GPU is present, the calls
raise.

Function names mirror the C entry points (``mvamg_`` prefix dropped).  Device
vectors are passed as torch CUDA tensors (float64, contiguous, on the handle's
device); their type, length and device are checked here before any call,
since the C ABI receives bare pointers.  Streams default to torch's current
stream.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmvamg.so")

OK, NOT_CONVERGED = 0, 1
ERR_ARG, ERR_FILE, ERR_NOT_SPD, ERR_NONFINITE, ERR_BREAKDOWN, ERR_HIP = -1, -2, -3, -4, -5, -6
SMOOTH_GS, SMOOTH_L1JACOBI = 0, 1
CYCLE_V, CYCLE_K = 0, 1

EXPORTED = ["mvamg_hier_read", "mvamg_hier_host_free", "mvamg_hier_host_info", "mvamg_arena_bytes",
            "mvamg_upload", "mvamg_free", "mvamg_batch_arena_bytes",
            "mvamg_levels", "mvamg_set_fine_values", "mvamg_spmv", "mvamg_cycle_apply", "mvamg_pcg_solve",
            "mvamg_adjoint_solve", "mvamg_grad_coeffs", "mvamg_profile", "mvamg_kernel_stats",
            "mvamg_last_error", "mvamg_spmv_block", "mvamg_cycle_apply_block", "mvamg_pcg_solve_block",
            "mvamg_batch_upload", "mvamg_batch_problems", "mvamg_batch_pcg_solve", "mvamg_autotune",
            "mvamg_tune_get", "mvamg_tune_set", "mvamg_signature", "mvamg_cycle_apply_noalloc",
            "mvamg_transfers", "mvamg_kcycle_apply", "mvamg_composite_work_bytes", "mvamg_composite_apply",
            "mvamg_composite_test", "mvamg_composite_pcg_solve", "mvamg_setup_bases", "mvamg_setup_pattern",
            "mvamg_setup_galerkin", "mvamg_setup_restrict", "mvamg_batch_small_path"]
# bytes of the static device array mvamg_cycle_apply_noalloc works in
NOALLOC_SCRATCH_BYTES = 32 << 20
BLOCK_MAX = 32
TUNE_GROUP_LANES, TUNE_BLOCK_COARSE, TUNE_BATCH_CHUNKS, TUNE_ALL = 1, 2, 4, 7

# kernel classes of mvamg_kernel_stats
KC_SMOOTH_FINE, KC_SMOOTH_COARSE, KC_SPMV, KC_RESIDUAL, KC_RESTRICT, KC_PROLONG, KC_COARSE = range(7)
KC_NAMES = ["smooth_fine", "smooth_coarse", "spmv", "residual", "restrict", "prolong", "coarse_solve"]


class MvamgError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"mvamg status {status}: {msg}")
        self.status = status


class SolveParams(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("smoother", ctypes.c_int), ("rtol", ctypes.c_double),
                ("maxit", ctypes.c_int), ("max_restarts", ctypes.c_int),
                ("history", ctypes.POINTER(ctypes.c_double)), ("cycle", ctypes.c_int)]


class Info(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("converged", ctypes.c_int), ("restarts", ctypes.c_int),
                ("rel_res", ctypes.c_double), ("rel_res_true", ctypes.c_double)]


_lib = None


def load(path: str = LIB_PATH):
    """Load libmvamg.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise RuntimeError(f"HIP library not built: {path} (run __graft_entry__.build())")
        L = ctypes.CDLL(path)
        vp, P = ctypes.c_void_p, ctypes.POINTER
        L.mvamg_hier_read.argtypes = [ctypes.c_char_p, P(vp)]
        L.mvamg_hier_host_free.argtypes = [vp]
        L.mvamg_hier_host_free.restype = None
        L.mvamg_hier_host_info.argtypes = [vp, P(ctypes.c_int), P(ctypes.c_int), P(ctypes.c_int64)]
        L.mvamg_arena_bytes.argtypes = [vp, ctypes.c_int, P(ctypes.c_size_t)]
        L.mvamg_upload.argtypes = [vp, vp, ctypes.c_size_t, vp, P(vp)]
        L.mvamg_batch_arena_bytes.argtypes = [P(vp), ctypes.c_int, ctypes.c_int, P(ctypes.c_size_t)]
        L.mvamg_free.argtypes = [vp]
        L.mvamg_free.restype = None
        L.mvamg_levels.argtypes = [vp, P(ctypes.c_int), P(ctypes.c_int), P(ctypes.c_int64), P(ctypes.c_int)]
        L.mvamg_set_fine_values.argtypes = [vp, vp, vp]
        L.mvamg_transfers.argtypes = [vp, P(ctypes.c_int), P(ctypes.c_int64)]
        L.mvamg_spmv.argtypes = [vp, vp, vp, vp]
        L.mvamg_cycle_apply.argtypes = [vp, vp, vp, ctypes.c_int, ctypes.c_int, vp]
        L.mvamg_cycle_apply_noalloc.argtypes = [vp, vp, vp, ctypes.c_int, ctypes.c_int, vp]
        L.mvamg_kcycle_apply.argtypes = [vp, vp, vp, ctypes.c_int, vp]
        L.mvamg_composite_work_bytes.argtypes = [ctypes.c_int, P(ctypes.c_size_t)]
        ci = ctypes.c_int
        L.mvamg_setup_bases.argtypes = [ci, ci, ci, ci, vp, vp, vp, ctypes.c_double, vp, vp, vp, vp, vp]
        IP = P(ctypes.c_int)
        L.mvamg_setup_pattern.argtypes = [ci, IP, IP, ci, IP, IP, IP, IP, IP, IP, IP, IP, IP, P(ctypes.c_int64)]
        L.mvamg_setup_galerkin.argtypes = [ci, ci, ci] + [vp] * 15 + [vp]
        L.mvamg_setup_restrict.argtypes = [ci, ci, vp, vp, vp, vp, vp, vp, vp]
        L.mvamg_composite_apply.argtypes = [P(vp), ctypes.c_int, ctypes.c_int, ctypes.c_int, vp, vp, vp,
                                            ctypes.c_size_t, vp]
        L.mvamg_composite_test.argtypes = [P(vp), ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, vp,
                                           P(ctypes.c_double), vp, ctypes.c_size_t, vp]
        L.mvamg_composite_pcg_solve.argtypes = [P(vp), ctypes.c_int, vp, vp, P(SolveParams), P(Info), vp,
                                                ctypes.c_size_t, vp]
        L.mvamg_pcg_solve.argtypes = [vp, vp, vp, vp, vp, vp, P(SolveParams), P(Info), vp]
        L.mvamg_adjoint_solve.argtypes = [vp, vp, vp, vp, vp, vp, P(SolveParams), P(Info), vp]
        L.mvamg_grad_coeffs.argtypes = [vp, vp, vp, vp, vp]
        L.mvamg_profile.argtypes = [vp, ctypes.c_int]
        L.mvamg_kernel_stats.argtypes = [vp, ctypes.c_int, P(ctypes.c_int64), P(ctypes.c_double),
                                         P(ctypes.c_double)]
        L.mvamg_last_error.restype = ctypes.c_char_p
        L.mvamg_spmv_block.argtypes = [vp, vp, vp, ctypes.c_int, vp]
        L.mvamg_cycle_apply_block.argtypes = [vp, vp, vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, vp]
        L.mvamg_pcg_solve_block.argtypes = [vp, vp, vp, ctypes.c_int, P(SolveParams), P(Info), vp]
        L.mvamg_batch_upload.argtypes = [P(vp), ctypes.c_int, ctypes.c_int, vp, ctypes.c_size_t, vp, P(vp)]
        L.mvamg_batch_small_path.argtypes = [vp, P(ctypes.c_int)]
        L.mvamg_batch_problems.argtypes = [vp, P(ctypes.c_int), P(ctypes.c_int)]
        L.mvamg_batch_pcg_solve.argtypes = [vp, vp, vp, P(SolveParams), P(Info), vp]
        L.mvamg_autotune.argtypes = [vp, ctypes.c_int, ctypes.c_char_p, ctypes.c_size_t, vp]
        L.mvamg_tune_get.argtypes = [vp, ctypes.c_char_p, ctypes.c_size_t]
        L.mvamg_tune_set.argtypes = [vp, ctypes.c_char_p]
        L.mvamg_signature.argtypes = [vp, ctypes.c_char_p, ctypes.c_size_t]
        for name in EXPORTED:
            if name not in ("mvamg_hier_host_free", "mvamg_free", "mvamg_last_error"):
                getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def last_error() -> str:
    return load().mvamg_last_error().decode()


def _check(st, allow=(OK,)):
    if st not in allow:
        raise MvamgError(st, last_error())
    return st


# Handles uploaded through this module: level-0 rows (all problems of a
# batch), stored level-0 entries, problem count and the device they live on.
# The C side cannot see the length or type of what a pointer points to, so
# every device vector is checked here against these before any call.
_HANDLES: dict = {}


def _register(h: int, arena, nrhs: int = 1) -> None:
    import torch
    lv = levels(h)
    k, off = batch_problems(h)
    if k > 0:  # a batch: the caller's vectors hold every problem, on either path
        lv = dict(n=[off[-1]] + lv["n"][1:], nnz=(lv["nnz"] or [0]))
    # the handle borrows the arena: the tensor is kept here until free(h)
    _HANDLES[h] = dict(n=lv["n"][0], nnz=lv["nnz"][0], nprob=k, device=torch.cuda.current_device(), arena=arena,
                      nrhs=nrhs)


def _hinfo(h: int) -> dict:
    try:
        return _HANDLES[h]
    except KeyError:
        raise ValueError("unknown or freed handle (upload it through this module)") from None


def _vec(h: int, t, numel: int, what: str, dtype: str = "float64") -> int:
    """Device address of t after checking that it is a contiguous torch tensor
    of `dtype` with `numel` elements on the handle's device."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{what}: expected a torch device tensor, got {type(t).__name__}")
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{what}: expected a contiguous device tensor")
    if t.dtype != getattr(torch, dtype):
        raise ValueError(f"{what}: expected {dtype}, got {t.dtype}")
    if t.numel() != numel:
        raise ValueError(f"{what}: expected {numel} elements, got {t.numel()}")
    dev = _hinfo(h)["device"]
    if t.device.index != dev:
        raise ValueError(f"{what}: tensor on cuda:{t.device.index}, handle on cuda:{dev}")
    return t.data_ptr()


def _history(history, rows: int, maxit: int):
    """Host history buffer: float64, C-contiguous, at least rows x (maxit + 1)."""
    if history is None:
        return None
    if not isinstance(history, np.ndarray) or history.dtype != np.float64 or not history.flags.c_contiguous:
        raise ValueError("history: expected a C-contiguous float64 numpy array")
    if history.size < rows * (maxit + 1):
        raise ValueError(f"history: needs {rows * (maxit + 1)} values, has {history.size}")
    if rows > 1 and (history.ndim != 2 or history.shape[1] != maxit + 1):
        raise ValueError(f"history: expected shape ({rows}, {maxit + 1})")
    return history.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _stream(stream) -> int | None:
    if stream is not None:
        return stream if isinstance(stream, int) else stream.cuda_stream
    import torch
    return torch.cuda.current_stream().cuda_stream


# ------------------------------------------------------------- raw entry points

def hier_read(path: str) -> int:
    h = ctypes.c_void_p()
    _check(load().mvamg_hier_read(path.encode(), ctypes.byref(h)))
    return h.value


def hier_host_free(hh: int) -> None:
    load().mvamg_hier_host_free(hh)


def hier_host_info(hh: int):
    nl, n, nnz = ctypes.c_int(), ctypes.c_int(), ctypes.c_int64()
    _check(load().mvamg_hier_host_info(hh, ctypes.byref(nl), ctypes.byref(n), ctypes.byref(nnz)))
    return nl.value, n.value, nnz.value


def arena_bytes(hh: int, nrhs: int = 1) -> int:
    """Device bytes mvamg_upload needs for a parsed hierarchy (nrhs > 1: with
    the work space of the block calls)."""
    b = ctypes.c_size_t()
    _check(load().mvamg_arena_bytes(hh, nrhs, ctypes.byref(b)))
    return b.value


def _arena(nbytes: int):
    import torch
    return torch.empty(max(nbytes, 1), dtype=torch.uint8, device="cuda")


def upload(hh: int, stream=None, nrhs: int = 1) -> int:
    """Uploads into a torch-owned arena sized by arena_bytes(hh, nrhs)."""
    arena = _arena(arena_bytes(hh, nrhs))
    h = ctypes.c_void_p()
    _check(load().mvamg_upload(hh, arena.data_ptr(), arena.numel(), _stream(stream), ctypes.byref(h)))
    _register(h.value, arena, nrhs)
    return h.value


def free(h: int) -> None:
    load().mvamg_free(h)  # waits for the device; the arena is then released with the entry
    _HANDLES.pop(h, None)


def levels(h: int):
    nl = ctypes.c_int()
    n = (ctypes.c_int * 32)()
    nnz = (ctypes.c_int64 * 32)()
    stg = (ctypes.c_int * 32)()
    _check(load().mvamg_levels(h, ctypes.byref(nl), n, nnz, stg))
    k = nl.value
    return dict(nlevels=k, n=list(n[:k]), nnz=list(nnz[:k]), stages=list(stg[:k]))


def transfers(h: int):
    """Aggregate counts and sum(n_a k_a) of the transfers P^l, l < nlevels - 1."""
    k = levels(h)["nlevels"] - 1
    na = (ctypes.c_int * 32)()
    nu = (ctypes.c_int64 * 32)()
    _check(load().mvamg_transfers(h, na, nu))
    return dict(nagg=list(na[:k]), nu=list(nu[:k]))


def set_fine_values(h: int, val, stream=None) -> None:
    _check(load().mvamg_set_fine_values(h, _vec(h, val, _hinfo(h)["nnz"], "val"), _stream(stream)))


def spmv(h: int, x, y, stream=None) -> None:
    n = _hinfo(h)["n"]
    _check(load().mvamg_spmv(h, _vec(h, x, n, "x"), _vec(h, y, n, "y"), _stream(stream)))


def cycle_apply(h: int, r, z, precision: int = 64, smoother: int = SMOOTH_GS, stream=None) -> None:
    n = _hinfo(h)["n"]
    _check(load().mvamg_cycle_apply(h, _vec(h, r, n, "r"), _vec(h, z, n, "z"), precision, smoother,
                                    _stream(stream)))


def cycle_apply_noalloc(h: int, r, z, precision: int = 64, smoother: int = SMOOTH_GS, stream=None) -> None:
    """z = B r as cycle_apply, with the cycle's work vectors in the library's
    static device array (no device allocation in the call)."""
    n = _hinfo(h)["n"]
    _check(load().mvamg_cycle_apply_noalloc(h, _vec(h, r, n, "r"), _vec(h, z, n, "z"), precision, smoother,
                                            _stream(stream)))


def kcycle_apply(h: int, r, z, smoother: int = SMOOTH_GS, stream=None) -> None:
    """z = K r, one K-cycle (binary64)."""
    n = _hinfo(h)["n"]
    _check(load().mvamg_kcycle_apply(h, _vec(h, r, n, "r"), _vec(h, z, n, "z"), smoother, _stream(stream)))


def _params(rtol, maxit, precision, smoother, max_restarts, history, rows=1, cycle=CYCLE_V):
    if not isinstance(maxit, int) or maxit < 0:
        raise ValueError("maxit must be a non-negative int")
    return SolveParams(precision, smoother, rtol, maxit, max_restarts, _history(history, rows, maxit), cycle)


def _matrix(h: int, A):
    """Device addresses of A = (rowptr, col, val) in the file's level-0 CSR
    form; any of them may be None (see mvamg_pcg_solve)."""
    if A is None:
        return None, None, None
    rowptr, col, val = A
    if (rowptr is None) != (col is None):
        raise ValueError("A: rowptr and col are passed together")
    hi = _hinfo(h)
    rp = None if rowptr is None else _vec(h, rowptr, hi["n"] + 1, "A.rowptr", "int32")
    ci = None if col is None else _vec(h, col, hi["nnz"], "A.col", "int32")
    v = None if val is None else _vec(h, val, hi["nnz"], "A.val")
    return rp, ci, v


def pcg_solve(h: int, b, x, rtol=1e-8, maxit=1000, precision=64, smoother=SMOOTH_GS, max_restarts=3,
              history: np.ndarray | None = None, stream=None, A=None, cycle=CYCLE_V) -> Info:
    """CG on A x = b.  A: (rowptr, col, val) device tensors of the finest
    matrix (same pattern as the hierarchy's, values may differ) or None for
    the values in use.  cycle: CYCLE_V or CYCLE_K (the preconditioner)."""
    info = Info()
    n = _hinfo(h)["n"]
    prm = _params(rtol, maxit, precision, smoother, max_restarts, history, cycle=cycle)
    rp, ci, v = _matrix(h, A)
    _check(load().mvamg_pcg_solve(h, rp, ci, v, _vec(h, b, n, "b"), _vec(h, x, n, "x"), ctypes.byref(prm),
                                  ctypes.byref(info), _stream(stream)), allow=(OK, NOT_CONVERGED))
    return info


def adjoint_solve(h: int, dLdx, lam, rtol=1e-8, maxit=1000, precision=64, smoother=SMOOTH_GS, max_restarts=3,
                  history: np.ndarray | None = None, stream=None, A=None, cycle=CYCLE_V) -> Info:
    info = Info()
    n = _hinfo(h)["n"]
    prm = _params(rtol, maxit, precision, smoother, max_restarts, history, cycle=cycle)
    rp, ci, v = _matrix(h, A)
    _check(load().mvamg_adjoint_solve(h, rp, ci, v, _vec(h, dLdx, n, "dLdx"), _vec(h, lam, n, "lambda"),
                                      ctypes.byref(prm), ctypes.byref(info), _stream(stream)),
           allow=(OK, NOT_CONVERGED))
    return info


def grad_coeffs(h: int, lam, x, dval, stream=None) -> None:
    hi = _hinfo(h)
    _check(load().mvamg_grad_coeffs(h, _vec(h, lam, hi["n"], "lambda"), _vec(h, x, hi["n"], "x"),
                                    _vec(h, dval, hi["nnz"], "dval"), _stream(stream)))


def _block_width(X) -> int:
    m = 1 if X.dim() == 1 else X.shape[1]
    if not 1 <= m <= BLOCK_MAX:
        raise ValueError(f"block width must be 1..{BLOCK_MAX}")
    return m


def _block(h: int, X, m: int, what: str) -> int:
    """An n x m row-major block (n x 1 may be a vector)."""
    if X.dim() not in (1, 2) or (X.dim() == 2 and X.shape[1] != m) or (X.dim() == 1 and m != 1):
        raise ValueError(f"{what}: expected shape (n, {m})")
    return _vec(h, X, _hinfo(h)["n"] * m, what)


def spmv_block(h: int, X, Y, stream=None) -> None:
    """Y = A X for an n x m row-major block (m <= 32)."""
    m = _block_width(X)
    _check(load().mvamg_spmv_block(h, _block(h, X, m, "X"), _block(h, Y, m, "Y"), m, _stream(stream)))


def cycle_apply_block(h: int, R, Z, precision: int = 64, smoother: int = SMOOTH_GS, stream=None) -> None:
    m = _block_width(R)
    _check(load().mvamg_cycle_apply_block(h, _block(h, R, m, "R"), _block(h, Z, m, "Z"), m, precision, smoother,
                                          _stream(stream)))


def pcg_solve_block(h: int, B, X, rtol=1e-8, maxit=1000, precision=64, smoother=SMOOTH_GS, max_restarts=3,
                    history: np.ndarray | None = None, stream=None) -> list:
    """CG on every column of the n x m block B (X: initial guesses, overwritten).
    history: m x (maxit + 1) array or None.  Returns one Info per column."""
    m = _block_width(B)
    infos = (Info * m)()
    prm = _params(rtol, maxit, precision, smoother, max_restarts, history, rows=m)
    _check(load().mvamg_pcg_solve_block(h, _block(h, B, m, "B"), _block(h, X, m, "X"), m, ctypes.byref(prm), infos,
                                        _stream(stream)), allow=(OK, NOT_CONVERGED))
    return list(infos)


def batch_upload(hhs, stream=None, mini_rows: int = 0) -> int:
    """Upload parsed hierarchies (mvamg_hier_read handles) as one batch, into
    a torch-owned arena; problems of at most mini_rows rows (and problems of
    an odd level count) take the one-launch small-problem path."""
    arr = (ctypes.c_void_p * len(hhs))(*hhs)
    nb = ctypes.c_size_t()
    _check(load().mvamg_batch_arena_bytes(arr, len(hhs), mini_rows, ctypes.byref(nb)))
    arena = _arena(nb.value)
    h = ctypes.c_void_p()
    _check(load().mvamg_batch_upload(arr, len(hhs), mini_rows, arena.data_ptr(), arena.numel(), _stream(stream),
                                     ctypes.byref(h)))
    _register(h.value, arena)
    return h.value


def batch_small_path(h: int) -> list:
    """Per problem: True if it is solved on the small-problem path."""
    k, _ = batch_problems(h)
    f = (ctypes.c_int * max(k, 1))()
    _check(load().mvamg_batch_small_path(h, f))
    return [bool(v) for v in f[:k]]


def batch_problems(h: int):
    """(problem count, row offsets) of a batch handle."""
    k = ctypes.c_int()
    _check(load().mvamg_batch_problems(h, ctypes.byref(k), None))
    off = (ctypes.c_int * (k.value + 1))()
    _check(load().mvamg_batch_problems(h, ctypes.byref(k), off))
    return k.value, list(off)


def batch_pcg_solve(h: int, b, x, rtol=1e-8, maxit=1000, precision=64, smoother=SMOOTH_GS, max_restarts=3,
                    history: np.ndarray | None = None, stream=None) -> list:
    """CG on every problem of a batch (b, x: the problems' vectors one after
    another).  history: nprob x (maxit + 1) array or None.  One Info per problem."""
    k, _ = batch_problems(h)
    n = _hinfo(h)["n"]
    infos = (Info * k)()
    prm = _params(rtol, maxit, precision, smoother, max_restarts, history, rows=max(k, 1))
    _check(load().mvamg_batch_pcg_solve(h, _vec(h, b, n, "b"), _vec(h, x, n, "x"), ctypes.byref(prm), infos,
                                        _stream(stream)), allow=(OK, NOT_CONVERGED))
    return list(infos)


def autotune(h: int, what: int = TUNE_ALL, stream=None) -> str:
    """Time the kernel variants on this hierarchy and keep the fastest; returns the report."""
    buf = ctypes.create_string_buffer(8192)
    _check(load().mvamg_autotune(h, what, buf, len(buf), _stream(stream)))
    return buf.value.decode()


def tune_get(h: int) -> str:
    buf = ctypes.create_string_buffer(1024)
    _check(load().mvamg_tune_get(h, buf, len(buf)))
    return buf.value.decode()


def tune_set(h: int, text: str) -> None:
    _check(load().mvamg_tune_set(h, text.encode()))


def signature(h: int) -> str:
    buf = ctypes.create_string_buffer(4096)
    _check(load().mvamg_signature(h, buf, len(buf)))
    return buf.value.decode()


def tuned(h: int, cache_path: str | None = None, what: int = TUNE_ALL, stream=None) -> str:
    """Apply cached tuning choices for this device and hierarchy signature, or
    autotune and add them to the cache (a JSON file, default
    $MVAMG_TUNE_CACHE or ~/.cache/mvamg_tune.json).  Returns the choices."""
    import json
    path = cache_path or os.environ.get("MVAMG_TUNE_CACHE",
                                        os.path.join(os.path.expanduser("~"), ".cache", "mvamg_tune.json"))
    # a handle without block work space skips the block-product choice
    key = f"{signature(h)}|what={what}" + ("|block" if _hinfo(h)["nrhs"] > 1 else "")
    cache = {}
    if os.path.exists(path):
        with open(path) as f:
            cache = json.load(f)
    if key in cache:
        tune_set(h, cache[key])
        return cache[key]
    autotune(h, what, stream)
    text = tune_get(h)
    cache[key] = text
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + f".{os.getpid()}.tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1)
    os.replace(tmp, path)
    return text


BOOK_COMPACT, BOOK_PLAIN = 1, 2


def profile(h: int, enable, booking: int = BOOK_COMPACT) -> None:
    """Turn per-launch kernel timing on or off (resets the totals).  booking:
    BOOK_COMPACT books the compact forms the kernels read, BOOK_PLAIN the
    plain model (12 bytes per stored binary64 entry)."""
    _check(load().mvamg_profile(h, booking if enable else 0))


def kernel_stats(h: int, kclass: int):
    """(launches, milliseconds, algorithmic bytes) of one kernel class."""
    n, ms, by = ctypes.c_int64(), ctypes.c_double(), ctypes.c_double()
    _check(load().mvamg_kernel_stats(h, kclass, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(by)))
    return n.value, ms.value, by.value


# ------------------------------------------------------------ convenience class

@dataclass
class SolveResult:
    iterations: int
    converged: bool
    rel_res: float
    rel_res_true: float
    restarts: int
    history: np.ndarray


class Solver:
    """A hierarchy file uploaded to the current GPU."""

    def __init__(self, path: str, stream=None, nrhs: int = 1):
        """nrhs > 1: the arena also holds the work space of block calls."""
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("mvamg needs a GPU (HIP device)")
        hh = hier_read(path)
        try:
            self.nlevels, self.n, self.nnz = hier_host_info(hh)
            self.h = upload(hh, stream, nrhs)
        finally:
            hier_host_free(hh)
        self.info = levels(self.h)

    def close(self):
        if getattr(self, "h", None):
            free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve(self, b, x=None, rtol=1e-8, maxit=1000, precision=64, smoother=SMOOTH_GS, max_restarts=3,
              stream=None, A=None, cycle=CYCLE_V):
        import torch
        if x is None:
            x = torch.zeros_like(b)
        hist = np.zeros(maxit + 1)
        inf = pcg_solve(self.h, b, x, rtol, maxit, precision, smoother, max_restarts, hist, stream, A, cycle)
        return x, SolveResult(inf.iterations, bool(inf.converged), inf.rel_res, inf.rel_res_true, inf.restarts,
                              hist[:inf.iterations + 1].copy())

    def cycle(self, r, precision=64, smoother=SMOOTH_GS, stream=None):
        import torch
        z = torch.empty_like(r)
        cycle_apply(self.h, r, z, precision, smoother, stream)
        return z

    def spmv(self, x, stream=None):
        import torch
        y = torch.empty_like(x)
        spmv(self.h, x, y, stream)
        return y


class Composite:
    """The bootstrap's composite AMG over Solvers of the stage hierarchies
    B_1..B_r (one fine matrix): the symmetrized multiplicative product, its
    testing phase and CG preconditioned by it.  r selects the first r
    hierarchies (default all)."""

    def __init__(self, solvers):
        import torch
        self.solvers = list(solvers)
        if not self.solvers:
            raise ValueError("no hierarchies")
        self.n = self.solvers[0].n
        for S in self.solvers:
            if S.n != self.n:
                raise ValueError("the hierarchies are not built on the same fine matrix")
        nb = ctypes.c_size_t()
        _check(load().mvamg_composite_work_bytes(self.n, ctypes.byref(nb)))
        self.work = torch.empty(nb.value, dtype=torch.uint8, device="cuda")

    def _hs(self, r):
        r = len(self.solvers) if r is None else r
        if not 1 <= r <= len(self.solvers):
            raise ValueError(f"r must be 1..{len(self.solvers)}")
        return (ctypes.c_void_p * r)(*[S.h for S in self.solvers[:r]]), r

    def apply(self, res, cycle=CYCLE_V, smoother=SMOOTH_GS, r=None, stream=None):
        import torch
        hs, r = self._hs(r)
        z = torch.empty_like(res)
        h0 = self.solvers[0].h
        _check(load().mvamg_composite_apply(hs, r, cycle, smoother, _vec(h0, res, self.n, "res"),
                                            _vec(h0, z, self.n, "z"), self.work.data_ptr(), self.work.numel(),
                                            _stream(stream)))
        return z

    def test(self, x, nu=15, cycle=CYCLE_V, smoother=SMOOTH_GS, r=None, stream=None) -> float:
        """Testing phase in place on x; returns the convergence estimate."""
        hs, r = self._hs(r)
        rho = ctypes.c_double()
        _check(load().mvamg_composite_test(hs, r, cycle, smoother, nu, _vec(self.solvers[0].h, x, self.n, "x"),
                                           ctypes.byref(rho), self.work.data_ptr(), self.work.numel(),
                                           _stream(stream)))
        return rho.value

    def solve(self, b, x=None, rtol=1e-8, maxit=1000, cycle=CYCLE_V, smoother=SMOOTH_GS, r=None, stream=None):
        import torch
        hs, r = self._hs(r)
        if x is None:
            x = torch.zeros_like(b)
        hist = np.zeros(maxit + 1)
        prm = _params(rtol, maxit, 64, smoother, 0, hist, cycle=cycle)
        info = Info()
        h0 = self.solvers[0].h
        _check(load().mvamg_composite_pcg_solve(hs, r, _vec(h0, b, self.n, "b"), _vec(h0, x, self.n, "x"),
                                                ctypes.byref(prm), ctypes.byref(info), self.work.data_ptr(),
                                                self.work.numel(), _stream(stream)), allow=(OK, NOT_CONVERGED))
        return x, SolveResult(info.iterations, bool(info.converged), info.rel_res, info.rel_res_true, 0,
                              hist[:info.iterations + 1].copy())


class BatchSolver:
    """Several hierarchy files uploaded as one batch (mini_rows: the size up to
    which problems take the one-launch small-problem path)."""

    def __init__(self, paths, stream=None, mini_rows: int = 0):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("mvamg needs a GPU (HIP device)")
        hhs = []
        try:
            for p in paths:
                hhs.append(hier_read(p))
            self.h = batch_upload(hhs, stream, mini_rows)
        finally:
            for hh in hhs:
                hier_host_free(hh)
        self.nprob, self.offsets = batch_problems(self.h)
        self.info = levels(self.h)

    def close(self):
        if getattr(self, "h", None):
            free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
