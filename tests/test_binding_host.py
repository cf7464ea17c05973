"""Host checks of the Python binding's argument validation (no GPU).

The C ABI receives bare pointers and cannot see what they point to, so the
binding checks every device tensor's type, length and device, and every host
history buffer's size, before it calls the library.  These tests use a CPU
tensor subclass that reports itself as a device tensor, so the checks run
without a GPU; every case must raise before anything reaches the library.
"""
import numpy as np
import pytest
import torch

from paper_1907_04417_amd import mvamg


class _FakeDev(torch.Tensor):
    """CPU tensor that reports itself as living on cuda:<dev>."""
    dev = 0

    @property
    def is_cuda(self):
        return True

    @property
    def device(self):
        return torch.device("cuda", self.dev)


def _fake(n, dtype=torch.float64, dev=0):
    t = torch.zeros(n, dtype=dtype).as_subclass(_FakeDev)
    t.dev = dev
    return t


@pytest.fixture
def handle():
    h = 0x7fff0000
    mvamg._HANDLES[h] = dict(n=10, nnz=34, nprob=0, device=0, arena=None, nrhs=1)
    yield h
    mvamg._HANDLES.pop(h, None)


def test_vec_accepts_matching_tensor(handle):
    t = _fake(10)
    assert mvamg._vec(handle, t, 10, "x") == t.data_ptr()


@pytest.mark.parametrize("bad, msg", [
    (lambda: _fake(10, torch.float32), "expected float64"),
    (lambda: _fake(9), "expected 10 elements"),
    (lambda: _fake(11), "expected 10 elements"),
    (lambda: _fake(10, dev=1), "handle on cuda:0"),
    (lambda: torch.zeros(10, dtype=torch.float64), "contiguous device tensor"),
    (lambda: _fake(20)[::2], "contiguous device tensor"),
    (lambda: 12345, "torch device tensor"),
])
def test_bad_vectors_raise_before_the_call(handle, bad, msg):
    for call in (lambda t: mvamg.spmv(handle, t, _fake(10)),
                 lambda t: mvamg.spmv(handle, _fake(10), t),
                 lambda t: mvamg.cycle_apply(handle, t, _fake(10)),
                 lambda t: mvamg.pcg_solve(handle, t, _fake(10)),
                 lambda t: mvamg.adjoint_solve(handle, _fake(10), t),
                 lambda t: mvamg.grad_coeffs(handle, t, _fake(10), _fake(34))):
        with pytest.raises((ValueError, TypeError), match=msg):
            call(bad())


def test_coefficient_arrays_have_nnz_entries(handle):
    with pytest.raises(ValueError, match="expected 34 elements"):
        mvamg.grad_coeffs(handle, _fake(10), _fake(10), _fake(10))
    with pytest.raises(ValueError, match="expected 34 elements"):
        mvamg.set_fine_values(handle, _fake(33))


def test_block_shapes(handle):
    X = torch.zeros((10, 4), dtype=torch.float64).as_subclass(_FakeDev)
    with pytest.raises(ValueError, match=r"expected shape \(n, 4\)"):
        mvamg.spmv_block(handle, X, _fake(40))
    Y = torch.zeros((9, 4), dtype=torch.float64).as_subclass(_FakeDev)
    with pytest.raises(ValueError, match="expected 40 elements"):
        mvamg.spmv_block(handle, X, Y)
    with pytest.raises(ValueError, match="block width"):
        mvamg.spmv_block(handle, torch.zeros((10, 33), dtype=torch.float64).as_subclass(_FakeDev), X)


def test_history_buffers(handle):
    for bad in (np.zeros(100), np.zeros(101, dtype=np.float32), np.zeros((101, 2))[:, 0], [0.0] * 101):
        with pytest.raises(ValueError, match="history"):
            mvamg.pcg_solve(handle, _fake(10), _fake(10), maxit=100, history=bad)
    X = torch.zeros((10, 3), dtype=torch.float64).as_subclass(_FakeDev)
    with pytest.raises(ValueError, match="history"):
        mvamg.pcg_solve_block(handle, X, X.clone(), maxit=100, history=np.zeros((3, 100)))
    with pytest.raises(ValueError, match="maxit"):
        mvamg.pcg_solve(handle, _fake(10), _fake(10), maxit=-1)


def test_unknown_handle():
    with pytest.raises(ValueError, match="unknown or freed handle"):
        mvamg.spmv(0x1234, _fake(10), _fake(10))


def test_matrix_arrays_are_checked(handle):
    """A passed to a solve: rowptr int32 n+1, col int32 nnz, val float64 nnz,
    rowptr and col together."""
    ok = (_fake(11, torch.int32), _fake(34, torch.int32), _fake(34))
    cases = [
        ((_fake(10, torch.int32), ok[1], ok[2]), "expected 11 elements"),
        ((_fake(11, torch.int64), ok[1], ok[2]), "expected int32"),
        ((ok[0], _fake(33, torch.int32), ok[2]), "expected 34 elements"),
        ((ok[0], ok[1], _fake(34, torch.float32)), "expected float64"),
        ((ok[0], None, ok[2]), "passed together"),
    ]
    for A, msg in cases:
        with pytest.raises(ValueError, match=msg):
            mvamg.pcg_solve(handle, _fake(10), _fake(10), A=A)
        with pytest.raises(ValueError, match=msg):
            mvamg.adjoint_solve(handle, _fake(10), _fake(10), A=A)


def _level_args(n=6):
    """A valid 1-D Laplacian level of n rows with aggregates of two rows."""
    rowptr, col, val = [0], [], []
    for i in range(n):
        for j in (i - 1, i, i + 1):
            if 0 <= j < n:
                col.append(j)
                val.append(2.0 if i == j else -1.0)
        rowptr.append(len(col))
    W = np.ones((n, 1))
    aptr = np.arange(0, n + 1, 2)
    arows = np.arange(n)
    return [np.array(rowptr), np.array(col), np.array(val), W, aptr, arows]


@pytest.mark.parametrize("case", [
    "rowptr_len", "rowptr_start", "rowptr_decreasing", "col_len", "val_len",
    "col_negative", "col_high", "aptr_short", "aptr_empty_agg", "aptr_end",
    "arows_len", "arows_dup", "arows_high"])
def test_setup_level_rejects_bad_level(case):
    """Level set-up checks A and the aggregates before any device use."""
    from paper_1907_04417_amd import gpu_setup
    a = _level_args()
    rowptr, col, val, W, aptr, arows = a
    if case == "rowptr_len":
        a[0] = rowptr[:-1]
    elif case == "rowptr_start":
        a[0] = rowptr + 1
    elif case == "rowptr_decreasing":
        r = rowptr.copy(); r[2], r[3] = r[3], r[2]; a[0] = r
    elif case == "col_len":
        a[1] = col[:-1]
    elif case == "val_len":
        a[2] = val[:-1]
    elif case == "col_negative":
        c = col.copy(); c[0] = -1; a[1] = c
    elif case == "col_high":
        c = col.copy(); c[-1] = 6; a[1] = c
    elif case == "aptr_short":
        a[4] = np.array([0])
    elif case == "aptr_empty_agg":
        a[4] = np.array([0, 2, 2, 6])
    elif case == "aptr_end":
        a[4] = np.array([0, 2, 4, 5])
    elif case == "arows_len":
        a[5] = arows[:-1]
    elif case == "arows_dup":
        r = arows.copy(); r[1] = 0; a[5] = r
    elif case == "arows_high":
        r = arows.copy(); r[5] = 6; a[5] = r
    with pytest.raises(ValueError):
        gpu_setup.setup_level(*a, tol=0.1)
