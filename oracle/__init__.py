"""CPU oracle of the AMG-preconditioned CG solve phase.

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.  The arithmetic lives
in ``mvamg_oracle.c`` (plain single-threaded binary64 C, no FMA contraction);
this module reads the hierarchy file with its own parser (``hierfile``) and
marshals arrays.  It imports nothing from the GPU package.

Functions and the passages they follow:
  vcycle      one V-cycle z = B r (Section 5: forward/backward Gauss-Seidel,
              exact coarsest solve; block-diagonal P of Section 4)
  pcg         preconditioned CG with stopping rule ||r_k|| <= tol ||r_0|| (Section 5)
  pcg_mixed   binary32 cycle inside a binary64 flexible CG (extension)
  grad_coeffs dL/da_ij = -lambda_i x_j (extension)
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from .hierfile import Hierarchy, read_hierarchy

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "mvamg_oracle.c")
LIB = os.path.join(_HERE, "libmvamg_oracle.so")

GS_COLOUR, GS_LEX, L1_JACOBI = 0, 1, 2

_I = ctypes.POINTER(ctypes.c_int)
_D = ctypes.POINTER(ctypes.c_double)
_F = ctypes.POINTER(ctypes.c_float)


class _Level(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("rowptr", _I), ("col", _I), ("val", _D),
                ("order", _I),
                ("nagg", ctypes.c_int), ("aptr", _I), ("arows", _I), ("coff", _I),
                ("uoff", _I), ("U", _D)]


def build() -> str:
    """Compile the oracle (gcc -O2 -ffp-contract=off)."""
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-std=c99", "-Wall", "-fPIC", "-shared", SRC,
           "-o", LIB + ".tmp", "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        L = ctypes.CDLL(LIB)
        L.orc_create.argtypes = [ctypes.c_int, ctypes.POINTER(_Level), ctypes.c_int, _I]
        L.orc_create.restype = ctypes.c_void_p
        L.orc_destroy.argtypes = [ctypes.c_void_p]
        L.orc_vcycle.argtypes = [ctypes.c_void_p, _D, _D, _D]
        L.orc_vcycle32.argtypes = [ctypes.c_void_p, _F, _F, _F]
        L.orc_coarse_solve.argtypes = [ctypes.c_void_p, _D, _D]
        L.orc_smooth.argtypes = [ctypes.c_void_p, ctypes.c_int, _D, _D, ctypes.c_int]
        L.orc_smooth32.argtypes = [ctypes.c_void_p, ctypes.c_int, _F, _F, ctypes.c_int]
        L.orc_spmv.argtypes = [ctypes.c_int, _I, _I, _D, _D, _D]
        L.orc_pcg.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, _I, _I, _D, _D, _D,
                              ctypes.c_double, ctypes.c_int, _D, _I]
        L.orc_pcg.restype = ctypes.c_int
        L.orc_pcg_mixed.argtypes = [ctypes.c_void_p, ctypes.c_int, _I, _I, _D, _D, _D, ctypes.c_double,
                                    ctypes.c_int, ctypes.c_int, _D, _I, _D, _I]
        L.orc_pcg_mixed.restype = ctypes.c_int
        L.orc_grad_coeffs.argtypes = [ctypes.c_int, _I, _I, _D, _D, _D]
        L.orc_kcycle.argtypes = [ctypes.c_void_p, _D, _D, _D]
        L.orc_pcg_kcycle.argtypes = [ctypes.c_void_p, ctypes.c_int, _I, _I, _D, _D, _D, ctypes.c_double,
                                     ctypes.c_int, _D, _I]
        L.orc_pcg_kcycle.restype = ctypes.c_int
        VP = ctypes.POINTER(ctypes.c_void_p)
        L.orc_composite_apply.argtypes = [VP, ctypes.c_int, ctypes.c_int, ctypes.c_int, _I, _I, _D, _D, _D]
        L.orc_composite_test.argtypes = [VP, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, _I, _I, _D,
                                         _D, _D]
        L.orc_pcg_composite.argtypes = [VP, ctypes.c_int, ctypes.c_int, ctypes.c_int, _I, _I, _D, _D, _D,
                                        ctypes.c_double, ctypes.c_int, _D, _I]
        L.orc_pcg_composite.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a, t):
    return a.ctypes.data_as(t)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


class Oracle:
    """The oracle bound to one hierarchy (file path or parsed Hierarchy)."""

    def __init__(self, hier, smoother: int = GS_COLOUR):
        if isinstance(hier, str):
            hier = read_hierarchy(hier)
        self.h: Hierarchy = hier
        self._keep = []
        lv = (_Level * hier.nlevels)()
        for l, L in enumerate(hier.levels):
            rp, ci, v = _i32(L.rowptr), _i32(L.col), _f64(L.val)
            self._keep += [rp, ci, v]
            lv[l].n = L.n
            lv[l].rowptr, lv[l].col, lv[l].val = _p(rp, _I), _p(ci, _I), _p(v, _D)
            if l + 1 < hier.nlevels:
                od = _i32(L.order)
                if od.shape[0] != L.n or not np.array_equal(np.sort(od), np.arange(L.n)):
                    raise ValueError("smoother order is not a permutation of the rows")
                T = hier.transfers[l]
                arrs = [_i32(T.aptr), _i32(T.arows), _i32(T.coff), _i32(T.uoff), _f64(T.U)]
                self._keep += [od, *arrs]
                lv[l].order = _p(od, _I)
                lv[l].nagg = T.nagg
                lv[l].aptr, lv[l].arows, lv[l].coff, lv[l].uoff = (_p(a, _I) for a in arrs[:4])
                lv[l].U = _p(arrs[4], _D)
        self._lv = lv
        st = ctypes.c_int(0)
        self._h = _load().orc_create(hier.nlevels, lv, smoother, ctypes.byref(st))
        if st.value != 0:
            raise ValueError("coarsest matrix is not positive definite")
        L0 = hier.levels[0]
        self.n = L0.n
        self.rowptr, self.col, self.val = _i32(L0.rowptr), _i32(L0.col), _f64(L0.val)

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.orc_destroy(self._h)
            self._h = None

    def vcycle(self, r, val0=None) -> np.ndarray:
        r = _f64(r)
        z = np.zeros(self.n)
        v0 = None if val0 is None else _p(_f64(val0), _D)
        _load().orc_vcycle(self._h, v0, _p(r, _D), _p(z, _D))
        return z

    def kcycle(self, r, val0=None) -> np.ndarray:
        """z = K r: the K-cycle (two inner flexible-CG iterations on every
        level but the finest and the coarsest)."""
        r = _f64(r)
        z = np.zeros(self.n)
        v0 = None if val0 is None else _p(_f64(val0), _D)
        _load().orc_kcycle(self._h, v0, _p(r, _D), _p(z, _D))
        return z

    def pcg_kcycle(self, b, x0=None, tol=1e-8, maxit=1000, val=None):
        """Flexible CG preconditioned by the K-cycle: (x, hist, nit, status)."""
        b = _f64(b)
        x = np.zeros(self.n) if x0 is None else _f64(x0).copy()
        v = self.val if val is None else _f64(val)
        hist = np.zeros(maxit + 1)
        nit = ctypes.c_int(0)
        st = _load().orc_pcg_kcycle(self._h, self.n, _p(self.rowptr, _I), _p(self.col, _I), _p(v, _D), _p(b, _D),
                                    _p(x, _D), tol, maxit, _p(hist, _D), ctypes.byref(nit))
        return x, hist[:nit.value + 1].copy(), nit.value, st

    def vcycle32(self, r) -> np.ndarray:
        r = np.ascontiguousarray(r, dtype=np.float32)
        z = np.zeros(self.n, dtype=np.float32)
        _load().orc_vcycle32(self._h, None, _p(r, _F), _p(z, _F))
        return z

    def coarse_solve(self, r) -> np.ndarray:
        r = _f64(r)
        z = np.zeros(r.shape[0])
        _load().orc_coarse_solve(self._h, _p(r, _D), _p(z, _D))
        return z

    def smooth(self, level: int, r, x, forward: bool = True) -> np.ndarray:
        r = _f64(r)
        x = _f64(x).copy()
        _load().orc_smooth(self._h, level, _p(r, _D), _p(x, _D), 1 if forward else 0)
        return x

    def smooth32(self, level: int, r, x, forward: bool = True) -> np.ndarray:
        """One sweep in binary32 on the level's binary32 values."""
        r = np.ascontiguousarray(r, dtype=np.float32)
        x = np.ascontiguousarray(x, dtype=np.float32).copy()
        _load().orc_smooth32(self._h, level, _p(r, _F), _p(x, _F), 1 if forward else 0)
        return x

    def matrix_dense(self, level: int = 0) -> np.ndarray:
        L = self.h.levels[level]
        M = np.zeros((L.n, L.n))
        rows = np.repeat(np.arange(L.n), np.diff(L.rowptr))
        np.add.at(M, (rows, L.col), L.val)
        return M

    def pcg(self, b, x0=None, tol=1e-8, maxit=1000, val=None, precond=True):
        """Returns (x, hist, nit, status); val replaces level-0 values (same pattern)."""
        b = _f64(b)
        x = np.zeros(self.n) if x0 is None else _f64(x0).copy()
        v = self.val if val is None else _f64(val)
        hist = np.zeros(maxit + 1)
        nit = ctypes.c_int(0)
        st = _load().orc_pcg(self._h, 1 if precond else 0, self.n, _p(self.rowptr, _I), _p(self.col, _I),
                             _p(v, _D), _p(b, _D), _p(x, _D), tol, maxit, _p(hist, _D), ctypes.byref(nit))
        return x, hist[:nit.value + 1].copy(), nit.value, st

    def pcg_mixed(self, b, x0=None, tol=1e-8, maxit=1000, max_restarts=3, with_restarts=False):
        """Returns (x, hist, nit, status, true_rel), and the restart count as a
        sixth value when with_restarts is set."""
        b = _f64(b)
        x = np.zeros(self.n) if x0 is None else _f64(x0).copy()
        hist = np.zeros(maxit + 1)
        nit = ctypes.c_int(0)
        tr = ctypes.c_double(0.0)
        rs = ctypes.c_int(0)
        st = _load().orc_pcg_mixed(self._h, self.n, _p(self.rowptr, _I), _p(self.col, _I), _p(self.val, _D),
                                   _p(b, _D), _p(x, _D), tol, maxit, max_restarts, _p(hist, _D),
                                   ctypes.byref(nit), ctypes.byref(tr), ctypes.byref(rs))
        out = (x, hist[:nit.value + 1].copy(), nit.value, st, tr.value)
        return out + (rs.value,) if with_restarts else out


class Composite:
    """The composite AMG over bootstrap hierarchies B_1..B_r (Oracle objects
    of the same fine matrix): the symmetrized multiplicative product of
    Section 5 item (i), its testing phase and CG preconditioned by it.
    kcycle selects K-cycle components instead of V-cycles."""

    def __init__(self, oracles, kcycle: bool = False):
        self.os = list(oracles)
        self.r = len(self.os)
        self.k = 1 if kcycle else 0
        O0 = self.os[0]
        for O in self.os[1:]:
            if O.n != O0.n or not np.array_equal(O.val, O0.val) or not np.array_equal(O.col, O0.col):
                raise ValueError("the hierarchies are not built on the same fine matrix")
        self.n, self.rowptr, self.col, self.val = O0.n, O0.rowptr, O0.col, O0.val
        self._hs = (ctypes.c_void_p * self.r)(*[O._h for O in self.os])

    def apply(self, res) -> np.ndarray:
        res = _f64(res)
        z = np.zeros(self.n)
        _load().orc_composite_apply(self._hs, self.r, self.k, self.n, _p(self.rowptr, _I), _p(self.col, _I),
                                    _p(self.val, _D), _p(res, _D), _p(z, _D))
        return z

    def test(self, x0, nu: int = 15):
        """(x^nu / ||x^nu||_A, rho estimate) of the testing phase from x0."""
        x = _f64(x0).copy()
        rho = ctypes.c_double(0.0)
        _load().orc_composite_test(self._hs, self.r, self.k, nu, self.n, _p(self.rowptr, _I), _p(self.col, _I),
                                   _p(self.val, _D), _p(x, _D), ctypes.byref(rho))
        return x, rho.value

    def pcg(self, b, tol=1e-8, maxit=1000):
        """(x, hist, nit, status) of CG preconditioned by the composite."""
        b = _f64(b)
        x = np.zeros(self.n)
        hist = np.zeros(maxit + 1)
        nit = ctypes.c_int(0)
        st = _load().orc_pcg_composite(self._hs, self.r, self.k, self.n, _p(self.rowptr, _I), _p(self.col, _I),
                                       _p(self.val, _D), _p(b, _D), _p(x, _D), tol, maxit, _p(hist, _D),
                                       ctypes.byref(nit))
        return x, hist[:nit.value + 1].copy(), nit.value, st


def spmv(rowptr, col, val, x) -> np.ndarray:
    rp, ci, v, x = _i32(rowptr), _i32(col), _f64(val), _f64(x)
    y = np.zeros(rp.shape[0] - 1)
    _load().orc_spmv(rp.shape[0] - 1, _p(rp, _I), _p(ci, _I), _p(v, _D), _p(x, _D), _p(y, _D))
    return y


def grad_coeffs(rowptr, col, lam, x) -> np.ndarray:
    rp, ci, lam, x = _i32(rowptr), _i32(col), _f64(lam), _f64(x)
    d = np.zeros(ci.shape[0])
    _load().orc_grad_coeffs(rp.shape[0] - 1, _p(rp, _I), _p(ci, _I), _p(lam, _D), _p(x, _D), _p(d, _D))
    return d


__all__ = ["Oracle", "Composite", "read_hierarchy", "spmv", "grad_coeffs", "build", "GS_COLOUR", "GS_LEX", "L1_JACOBI"]
