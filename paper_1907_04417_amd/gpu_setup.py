"""Numeric setup of one multiple-vector level on the GPU (Section 4), through
the C ABI: the per-aggregate local bases (eq. 4.3), the Galerkin coarse
matrix and the coarse smooth vectors.  Marshalling only: the arithmetic runs
in the library's kernels; the coarse pattern is integer bookkeeping that the
library does on the host.

    setup_level(rowptr, col, val, W, aptr, arows, tol=0.1)
        -> dict(k, U (list of n_a x k_a blocks), dropped, coff,
                rowptr_c, col_c, val_c, Wc)
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import mvamg


def _dev(torch, a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dtype)).cuda()


def _iptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def setup_level(rowptr, col, val, W, aptr, arows, tol: float = 0.1, stream=None):
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int32)
    col = np.ascontiguousarray(col, dtype=np.int32)
    aptr = np.ascontiguousarray(aptr, dtype=np.int32)
    arows = np.ascontiguousarray(arows, dtype=np.int32)
    W = np.ascontiguousarray(W, dtype=np.float64)
    n, m = W.shape
    nagg = aptr.shape[0] - 1
    # the kernels index with these arrays' contents, so they are checked here,
    # on the host, before anything reaches the device
    if rowptr.shape[0] != n + 1 or rowptr[0] != 0 or np.any(np.diff(rowptr) < 0):
        raise ValueError("rowptr must start at 0 and not decrease, with n + 1 entries")
    if col.shape[0] != rowptr[-1] or np.asarray(val).shape[0] != rowptr[-1]:
        raise ValueError("A's arrays do not match the level size")
    if col.size and (col.min() < 0 or col.max() >= n):
        raise ValueError("column index out of range")
    if aptr.shape[0] < 2 or aptr[0] != 0 or aptr[-1] != n or np.any(np.diff(aptr) < 1):
        raise ValueError("aggregates must be non-empty ranges that cover every row")
    if arows.shape[0] != n or (n and (arows.min() < 0 or arows.max() >= n)) or \
            np.any(np.bincount(arows, minlength=n) != 1):
        raise ValueError("aggregates must list every row once")
    import torch
    L = mvamg.load()
    st = mvamg._stream(stream)
    d_aptr, d_arows = _dev(torch, aptr, np.int32), _dev(torch, arows, np.int32)
    d_W = _dev(torch, W, np.float64)
    d_k = torch.zeros(nagg, dtype=torch.int32, device="cuda")
    d_U = torch.zeros(n * m, dtype=torch.float64, device="cuda")
    d_drop = torch.zeros(nagg, dtype=torch.float64, device="cuda")
    d_flag = torch.zeros(1, dtype=torch.int32, device="cuda")
    max_na = int(np.diff(aptr).max())
    mvamg._check(L.mvamg_setup_bases(n, m, nagg, max_na, d_aptr.data_ptr(), d_arows.data_ptr(), d_W.data_ptr(),
                                     tol, d_k.data_ptr(), d_U.data_ptr(), d_drop.data_ptr(), d_flag.data_ptr(), st))
    k = d_k.cpu().numpy().astype(np.int32)
    agg, loc = np.zeros(n, np.int32), np.zeros(n, np.int32)
    coff = np.zeros(nagg + 1, np.int32)
    nc_guess = int(k.sum())
    cagg = np.zeros(nc_guess, np.int32)
    nnz = ctypes.c_int64()
    args = [n, _iptr(rowptr), _iptr(col), nagg, _iptr(aptr), _iptr(arows), _iptr(k), _iptr(agg), _iptr(loc),
            _iptr(coff), _iptr(cagg)]
    mvamg._check(L.mvamg_setup_pattern(*args, None, None, ctypes.byref(nnz)))
    nc = int(coff[-1])
    crp = np.zeros(nc + 1, np.int32)
    ccol = np.zeros(nnz.value, np.int32)
    mvamg._check(L.mvamg_setup_pattern(*args, _iptr(crp), _iptr(ccol), ctypes.byref(nnz)))
    d_coff, d_agg, d_loc, d_cagg = (_dev(torch, a, np.int32) for a in (coff, agg, loc, cagg))
    d_rp, d_ci, d_val = _dev(torch, rowptr, np.int32), _dev(torch, col, np.int32), _dev(torch, val, np.float64)
    d_crp, d_ccol = _dev(torch, crp, np.int32), _dev(torch, ccol, np.int32)
    d_cval = torch.zeros(nnz.value, dtype=torch.float64, device="cuda")
    d_work = torch.zeros(max(nnz.value, 1), dtype=torch.float64, device="cuda")
    mvamg._check(L.mvamg_setup_galerkin(m, nagg, nc, d_aptr.data_ptr(), d_arows.data_ptr(), d_coff.data_ptr(),
                                        d_agg.data_ptr(), d_loc.data_ptr(), d_cagg.data_ptr(), d_rp.data_ptr(),
                                        d_ci.data_ptr(), d_val.data_ptr(), d_U.data_ptr(), d_crp.data_ptr(),
                                        d_ccol.data_ptr(), d_cval.data_ptr(), d_work.data_ptr(), d_flag.data_ptr(),
                                        st))
    d_Wc = torch.zeros(nc * m, dtype=torch.float64, device="cuda")
    mvamg._check(L.mvamg_setup_restrict(m, nagg, d_aptr.data_ptr(), d_arows.data_ptr(), d_coff.data_ptr(),
                                        d_U.data_ptr(), d_W.data_ptr(), d_Wc.data_ptr(), st))
    torch.cuda.synchronize()
    Upad = d_U.cpu().numpy().reshape(n, m)
    Us = [Upad[aptr[a]:aptr[a + 1], :k[a]].copy() for a in range(nagg)]
    return dict(k=k, U=Us, dropped=d_drop.cpu().numpy(), coff=coff, rowptr_c=crp, col_c=ccol,
                val_c=d_cval.cpu().numpy(), Wc=d_Wc.cpu().numpy().reshape(nc, m))
