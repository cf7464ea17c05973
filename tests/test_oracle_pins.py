"""Pins of the CPU oracle against closed forms, textbook special cases and
brute force on tiny inputs (no GPU).

Each test would fail on a plausible mistake in the oracle: a wrong sweep order
or sign in Gauss-Seidel, a transposed prolongator, a dropped coarse
correction, a wrong CG coefficient, or a wrong adjoint formula.
"""
import numpy as np
import pytest

import oracle
from oracle.hierfile import Hierarchy, Level, Transfer, read_hierarchy
from tests import dense_ref as dr


def _oracle_B(O):
    n = O.n
    return np.stack([O.vcycle(e) for e in np.eye(n)], axis=1)


@pytest.mark.parametrize("fx", ["tiny_hier", "small3d_hier"])
def test_gs_sweep_closed_form(fx, request):
    """One forward (backward) sweep equals x + M^{-1}(r - A x) (resp. M^{-T})
    with M = D + the part of A earlier in the colour order."""
    P, path, _ = request.getfixturevalue(fx)
    O = oracle.Oracle(path)
    H = O.h
    for l in range(H.nlevels - 1):
        L = H.levels[l]
        A = dr.dense(L.rowptr, L.col, L.val)
        M = dr.gs_splitting(A, L.order)
        rng = np.random.default_rng(l)
        r, x = rng.standard_normal(L.n), rng.standard_normal(L.n)
        xf = O.smooth(l, r, x, forward=True)
        xb = O.smooth(l, r, x, forward=False)
        np.testing.assert_allclose(xf, x + np.linalg.solve(M, r - A @ x), rtol=1e-11, atol=1e-11)
        np.testing.assert_allclose(xb, x + np.linalg.solve(M.T, r - A @ x), rtol=1e-11, atol=1e-11)


@pytest.mark.parametrize("fx", ["tiny_hier", "small3d_hier"])
def test_backward_sweep_ignores_last_stage_start(fx, request):
    """On a point level the backward sweep relaxes the last stage first, and a
    row's update reads only its neighbours, never its own old value: the
    sweep's result is bitwise independent of the last stage's starting values
    (so the prolongation before it may leave those rows out), while any row
    of an earlier stage does change it."""
    P, path, _ = request.getfixturevalue(fx)
    H = read_hierarchy(path)
    L0 = H.levels[0]
    assert len(L0.gptr) - 1 == L0.n  # point level
    O = oracle.Oracle(path)
    rng = np.random.default_rng(31)
    r = rng.standard_normal(L0.n)
    x1 = rng.standard_normal(L0.n)
    last = L0.order[L0.gptr[L0.sptr[-2]]:]
    x2 = x1.copy()
    x2[last] = rng.standard_normal(len(last))
    y1 = O.smooth(0, r, x1, forward=False)
    assert np.array_equal(O.smooth(0, r, x2, forward=False), y1)
    x3 = x1.copy()
    x3[L0.order[0]] += 1.0
    assert not np.array_equal(O.smooth(0, r, x3, forward=False), y1)


def test_lexicographic_gs_closed_form(tiny_hier):
    """The paper's sequential GS (natural order) is the same closed form with O = 0..n-1."""
    _, path, _ = tiny_hier
    O = oracle.Oracle(path, smoother=oracle.GS_LEX)
    L = O.h.levels[0]
    A = dr.dense(L.rowptr, L.col, L.val)
    M = np.tril(A)
    rng = np.random.default_rng(7)
    r, x = rng.standard_normal(L.n), rng.standard_normal(L.n)
    np.testing.assert_allclose(O.smooth(0, r, x, True), x + np.linalg.solve(M, r - A @ x), rtol=1e-11)
    np.testing.assert_allclose(O.smooth(0, r, x, False), x + np.linalg.solve(np.triu(A), r - A @ x),
                               rtol=1e-11)


@pytest.mark.parametrize("fx", ["tiny_hier", "small3d_hier"])
def test_vcycle_equals_closed_form(fx, request):
    """B from the oracle's cycle equals the recursive error-propagator form."""
    P, path, st = request.getfixturevalue(fx)
    O = oracle.Oracle(path)
    assert O.h.nlevels >= 3, st
    B = _oracle_B(O)
    Bc = dr.vcycle_matrix(O.h)
    assert np.abs(B - Bc).max() <= 1e-10 * np.abs(Bc).max()


@pytest.mark.parametrize("fx", ["tiny_hier", "small3d_hier"])
def test_vcycle_spd_and_contractive(fx, request):
    """The symmetric V-cycle is s.p.d. and E = I - BA has spectrum in [0, 1)."""
    P, path, _ = request.getfixturevalue(fx)
    O = oracle.Oracle(path)
    B = _oracle_B(O)
    A = O.matrix_dense(0)
    assert np.abs(B - B.T).max() <= 1e-12 * np.abs(B).max()
    np.linalg.cholesky(0.5 * (B + B.T))
    Lc = np.linalg.cholesky(A)
    # E is similar to I - L^T B L (symmetric), so its eigenvalues are real
    S = np.eye(A.shape[0]) - Lc.T @ B @ Lc
    ev = np.linalg.eigvalsh(0.5 * (S + S.T))
    assert ev.min() >= -1e-10 and ev.max() < 1.0


def test_nearby_matrix_keeps_spd(tiny_hier):
    """Level-0 values replaced by a near-by s.p.d. matrix (same pattern): the
    cycle stays symmetric positive definite and PCG converges to its solution."""
    P, path, _ = tiny_hier
    O = oracle.Oracle(path)
    rng = np.random.default_rng(11)
    A = O.matrix_dense(0)
    # scale rows and columns by a positive diagonal: D A D keeps pattern and s.p.d.
    d = np.exp(0.2 * rng.standard_normal(O.n))
    rows = np.repeat(np.arange(O.n), np.diff(O.rowptr))
    val2 = O.val * d[rows] * d[O.col]
    A2 = np.diag(d) @ A @ np.diag(d)
    B = np.stack([O.vcycle(e, val0=val2) for e in np.eye(O.n)], axis=1)
    assert np.abs(B - B.T).max() <= 1e-12 * np.abs(B).max()
    np.linalg.cholesky(0.5 * (B + B.T))
    b = rng.standard_normal(O.n)
    x, hist, nit, st = O.pcg(b, val=val2, tol=1e-12)
    assert st == 0
    np.testing.assert_allclose(x, np.linalg.solve(A2, b), rtol=1e-9, atol=1e-9)


def _singleton_hierarchy(P):
    n = P.n
    lv0 = Level(n, P.rowptr, P.col, P.val)
    # greedy colouring by brute force for the fine level
    A = dr.dense(P.rowptr, P.col, P.val)
    colour = -np.ones(n, dtype=int)
    for i in range(n):
        used = {colour[j] for j in np.nonzero(A[i])[0] if j != i and colour[j] >= 0}
        c = 0
        while c in used:
            c += 1
        colour[i] = c
    order = np.argsort(colour, kind="stable").astype(np.int32)
    lv0.sptr = np.concatenate([[0], np.cumsum(np.bincount(colour))]).astype(np.int32)
    lv0.gptr = np.arange(n + 1, dtype=np.int32)
    lv0.order = order
    lv1 = Level(n, P.rowptr, P.col, P.val)
    ar = np.arange(n + 1, dtype=np.int32)
    T = Transfer(ar, np.arange(n, dtype=np.int32), ar, ar, np.ones(n), np.zeros(n))
    return Hierarchy([lv0, lv1], [T], 1, np.zeros(0), np.zeros(7, dtype=np.int64))


def test_all_singleton_prolongator_is_exact():
    """P = I makes the coarse correction exact, so B = A^{-1} and PCG
    converges in one iteration to the dense solution."""
    from paper_1907_04417_amd import problems
    P = problems.aniso9(7, seed=1)
    O = oracle.Oracle(_singleton_hierarchy(P))
    A = O.matrix_dense(0)
    B = _oracle_B(O)
    np.testing.assert_allclose(B @ A, np.eye(P.n), atol=1e-10)
    x, hist, nit, st = O.pcg(P.b, tol=1e-10)
    assert nit == 1 and st == 0
    np.testing.assert_allclose(x, np.linalg.solve(A, P.b), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("fx", ["tiny_hier", "small3d_hier"])
def test_pcg_equals_dense_pcg(fx, request):
    """Oracle PCG matches the textbook PCG with the explicit matrix B, step by
    step, and the A-norm of the error never increases."""
    P, path, _ = request.getfixturevalue(fx)
    O = oracle.Oracle(path)
    A = O.matrix_dense(0)
    B = dr.vcycle_matrix(O.h)
    x, hist, nit, st = O.pcg(P.b, tol=1e-10)
    xd, hd = dr.pcg_dense(A, B, P.b, 1e-10, 1000)
    assert st == 0 and nit == len(hd) - 1
    np.testing.assert_allclose(hist, hd, rtol=1e-7)
    xs = np.linalg.solve(A, P.b)
    np.testing.assert_allclose(x, xs, rtol=1e-8, atol=1e-8 * np.abs(xs).max())
    # A-norm error monotone along the iteration (rerun with maxit = k)
    errs = []
    for k in range(1, nit + 1):
        xk, _, _, _ = O.pcg(P.b, tol=0.0, maxit=k)
        e = xk - xs
        errs.append(np.sqrt(e @ A @ e))
    assert all(errs[i + 1] <= errs[i] * (1 + 1e-9) for i in range(len(errs) - 1))


def test_plain_cg_is_textbook():
    """precond=False reduces to plain CG (B = I)."""
    from paper_1907_04417_amd import problems
    P = problems.aniso9(7, seed=2)
    O = oracle.Oracle(_singleton_hierarchy(P))
    A = O.matrix_dense(0)
    x, hist, nit, st = O.pcg(P.b, tol=1e-10, precond=False)
    xd, hd = dr.pcg_dense(A, np.eye(P.n), P.b, 1e-10, 1000)
    assert nit == len(hd) - 1
    np.testing.assert_allclose(hist, hd, rtol=1e-8)


def test_convergence_factor_estimate(tiny_hier):
    """The ratio estimate ||E x||_A / ||x||_A after nu applications of
    E = I - BA to a random vector never exceeds rho(E) and approaches it."""
    P, path, _ = tiny_hier
    O = oracle.Oracle(path)
    A = O.matrix_dense(0)
    B = _oracle_B(O)
    Lc = np.linalg.cholesky(A)
    S = np.eye(O.n) - Lc.T @ B @ Lc
    rho = np.abs(np.linalg.eigvalsh(0.5 * (S + S.T))).max()
    x = np.random.default_rng(0).standard_normal(O.n)
    anorm = lambda v: np.sqrt(v @ A @ v)
    for _ in range(50):
        xp = x
        x = x - O.vcycle(A @ x)
    est = anorm(x) / anorm(xp)
    assert est <= rho * (1 + 1e-10)
    assert est >= 0.9 * rho


def test_mixed_precision_cycle_and_pcg(small3d_hier):
    P, path, _ = small3d_hier
    O = oracle.Oracle(path)
    r = np.random.default_rng(4).standard_normal(O.n)
    z64 = O.vcycle(r)
    z32 = O.vcycle32(r.astype(np.float32)).astype(np.float64)
    assert np.linalg.norm(z32 - z64) <= 1e-5 * np.linalg.norm(z64)
    x, hist, nit, st, tr = O.pcg_mixed(P.b, tol=1e-10)
    assert st == 0 and tr <= 1e-10
    A = O.matrix_dense(0)
    np.testing.assert_allclose(x, np.linalg.solve(A, P.b), rtol=1e-7, atol=1e-8)


def test_gradient_formula_matches_finite_differences():
    """dL/da_ij = -lambda_i x_j, lambda = A^{-T} dL/dx: checked against central
    differences of L(x(A)) computed with dense solves, entry by entry."""
    from paper_1907_04417_amd import problems
    P = problems.aniso9(5, seed=4)
    A = dr.dense(P.rowptr, P.col, P.val)
    rng = np.random.default_rng(3)
    xobs = rng.standard_normal(P.n)
    loss = lambda M: np.sum((np.linalg.solve(M, P.b) - xobs) ** 2)
    x = np.linalg.solve(A, P.b)
    lam = np.linalg.solve(A.T, 2 * (x - xobs))
    g = oracle.grad_coeffs(P.rowptr, P.col, lam, x)
    rows = np.repeat(np.arange(P.n), np.diff(P.rowptr))
    h = 1e-6
    for k in range(0, P.nnz, 7):
        Ap, Am = A.copy(), A.copy()
        Ap[rows[k], P.col[k]] += h
        Am[rows[k], P.col[k]] -= h
        fd = (loss(Ap) - loss(Am)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(g[k]))


def test_oracle_spmv_matches_dense():
    from paper_1907_04417_amd import problems
    P = problems.jump7(5, cube=1, seed=1)
    A = dr.dense(P.rowptr, P.col, P.val)
    x = np.random.default_rng(1).standard_normal(P.n)
    np.testing.assert_allclose(oracle.spmv(P.rowptr, P.col, P.val, x), A @ x, rtol=1e-13)


def test_zero_rhs_returns_zero(tiny_hier):
    P, path, _ = tiny_hier
    O = oracle.Oracle(path)
    x, hist, nit, st = O.pcg(np.zeros(P.n))
    assert nit == 0 and st == 0 and not x.any()


def test_maxit_reports_not_converged(tiny_hier):
    P, path, _ = tiny_hier
    O = oracle.Oracle(path)
    x, hist, nit, st = O.pcg(P.b, tol=1e-14, maxit=2)
    assert st == 1 and nit == 2 and len(hist) == 3


def test_hierarchy_file_rejects_corruption(tiny_hier, tmp_path):
    _, path, _ = tiny_hier
    buf = open(path, "rb").read()
    bad = tmp_path / "bad.bin"
    bad.write_bytes(b"XXXXXXXX" + buf[8:])
    with pytest.raises(ValueError):
        read_hierarchy(str(bad))
    bad.write_bytes(buf[: len(buf) // 2])
    with pytest.raises(ValueError):
        read_hierarchy(str(bad))


# ------------------------------------------------------------ l1-Jacobi

@pytest.mark.parametrize("fx", ["tiny_hier", "small3d_hier"])
def test_l1_sweep_closed_form(fx, request):
    """One l1-Jacobi sweep equals x + D_l1^{-1}(r - A x) with
    D_l1 = diag(sum_j |a_ij|), the full l1 row norm, built densely; in
    binary64, and in binary32 to the binary32 rounding of the same map."""
    P, path, _ = request.getfixturevalue(fx)
    O = oracle.Oracle(path, smoother=oracle.L1_JACOBI)
    H = O.h
    for l in range(H.nlevels - 1):
        L = H.levels[l]
        A = dr.dense(L.rowptr, L.col, L.val)
        M = dr.l1_splitting(A)
        rng = np.random.default_rng(40 + l)
        r, x = rng.standard_normal(L.n), rng.standard_normal(L.n)
        want = x + np.linalg.solve(M, r - A @ x)
        for fwd in (True, False):  # l1-Jacobi has no direction
            np.testing.assert_allclose(O.smooth(l, r, x, forward=fwd), want, rtol=1e-12, atol=1e-12)
        r32, x32 = r.astype(np.float32), x.astype(np.float32)
        A32 = dr.dense(L.rowptr, L.col, L.val.astype(np.float32).astype(np.float64))
        want32 = x32 + np.linalg.solve(dr.l1_splitting(A32), r32 - A32 @ x32)
        got32 = O.smooth32(l, r32, x32).astype(np.float64)
        assert np.abs(got32 - want32).max() <= 1e-5 * np.abs(want32).max()


@pytest.mark.parametrize("fx", ["tiny_hier", "small3d_hier"])
def test_l1_vcycle_equals_closed_form(fx, request):
    """The l1-Jacobi V-cycle equals the recursive error-propagator form with
    M_l = D_l1 on every level (pre and post alike, so B is symmetric); it is
    s.p.d. with the spectrum of E = I - BA in [0, 1), and the binary32 cycle
    stays within binary32 rounding of it."""
    P, path, _ = request.getfixturevalue(fx)
    O = oracle.Oracle(path, smoother=oracle.L1_JACOBI)
    B = _oracle_B(O)
    Bc = dr.vcycle_matrix(O.h, smoother="l1")
    assert np.abs(B - Bc).max() <= 1e-10 * np.abs(Bc).max()
    assert np.abs(B - B.T).max() <= 1e-12 * np.abs(B).max()
    A = O.matrix_dense(0)
    Lc = np.linalg.cholesky(A)
    S = np.eye(O.n) - Lc.T @ B @ Lc
    ev = np.linalg.eigvalsh(0.5 * (S + S.T))
    assert ev.min() >= -1e-10 and ev.max() < 1.0
    r = np.random.default_rng(41).standard_normal(O.n)
    z32 = O.vcycle32(r.astype(np.float32)).astype(np.float64)
    zc = Bc @ r.astype(np.float32).astype(np.float64)
    assert np.abs(z32 - zc).max() <= 1e-5 * np.abs(zc).max()


# --------------------------------------------- binary32 cycle under CG

def _directions_conjugacy(A, xs):
    """|d_{k+1}^T A d_k| / (||d_{k+1}||_A ||d_k||_A) for d_k = x_{k+1} - x_k."""
    d = [xs[k + 1] - xs[k] for k in range(len(xs) - 1)]
    an = lambda v: np.sqrt(v @ A @ v)
    return np.array([abs(d[k + 1] @ A @ d[k]) / (an(d[k + 1]) * an(d[k])) for k in range(len(d) - 1)])


def test_mixed_pcg_is_flexible_cg(small3d_hier):
    """The binary64 CG around the binary32 cycle is flexible CG (Notay 2000).

    1. Step by step against a NumPy flexible CG written from Notay's
       definition, beta = z_{k+1}^T (r_{k+1} - r_k) / rho_k, calling the same
       binary32 cycle: the first four residuals agree to 1e-12.  (After that a
       one-unit difference in r flips the binary32 rounding of some entries at
       the cycle's entry and the two runs separate by ~10x per iteration; the
       Fletcher-Reeves rule already differs by ~1e-9 at the second step.)
    2. A property that holds for the flexible rule only: consecutive search
       directions, recovered from the iterates as x_{k+1} - x_k, are
       A-conjugate (Notay's beta makes p_{k+1}^T A p_k = 0 whatever the cycle
       returns); with the standard rule the binary32 cycle's asymmetry leaves
       ~1e-8.  Checked on the first pairs, before the differences of iterates
       lose digits to cancellation."""
    P, path, _ = small3d_hier
    O = oracle.Oracle(path)
    A = O.matrix_dense(0)
    mv = lambda x: dr.seq_csr_mv(O.rowptr, O.col, O.val, x)
    prec = lambda r: O.vcycle32(r.astype(np.float32)).astype(np.float64)
    xo, ho, nito, sto, tro = O.pcg_mixed(P.b, tol=1e-10, maxit=100)
    xn, hn, nitn, stn, trn, rsn, _ = dr.flexible_pcg(mv, prec, P.b, 1e-10, 100, 3)
    assert sto == stn == 0 and abs(nito - nitn) <= 1
    np.testing.assert_allclose(ho[:5], hn[:5], rtol=1e-12)
    _, hf, *_ = dr.flexible_pcg(mv, prec, P.b, 1e-10, 4, 0, beta_rule="fletcher_reeves")
    assert (np.abs(hf[:5] - hn[:5]) / hn[:5]).max() > 1e-9  # the pin tells the rules apart
    xs = [np.zeros(O.n)] + [O.pcg_mixed(P.b, tol=0.0, maxit=k, max_restarts=0)[0] for k in range(1, 6)]
    assert _directions_conjugacy(A, xs)[:3].max() <= 1e-12
    xf = [np.zeros(O.n)] + [dr.flexible_pcg(mv, prec, P.b, 0.0, k, 0, "fletcher_reeves")[0] for k in range(1, 6)]
    assert _directions_conjugacy(A, xf)[:3].max() > 1e-10
    np.testing.assert_allclose(xo, np.linalg.solve(A, P.b), rtol=1e-8, atol=1e-9)


def test_mixed_pcg_restarts(small3d_hier):
    """True-residual restarts.  With tol = 1e-17, below what binary64 can
    reach on the true residual (~1e-16 here), the recursive residual still
    meets tol; the recomputed b - A x then misses it, so every allowed restart
    is taken and the call ends not converged, with x at the binary64 floor.
    The restart count, the status and the history before the first restart
    match the NumPy flexible CG; max_restarts bounds the
    count.  (Where a segment ends is decided by residuals within rounding of
    tol, so the restart points themselves may differ by an iteration.)"""
    P, path, _ = small3d_hier
    O = oracle.Oracle(path)
    A = O.matrix_dense(0)
    mv = lambda x: dr.seq_csr_mv(O.rowptr, O.col, O.val, x)
    prec = lambda r: O.vcycle32(r.astype(np.float32)).astype(np.float64)
    xs = np.linalg.solve(A, P.b)
    for mr in (3, 1):
        xo, ho, nito, sto, tro, rso = O.pcg_mixed(P.b, tol=1e-17, maxit=200, max_restarts=mr, with_restarts=True)
        xn, hn, nitn, stn, trn, rsn, rits = dr.flexible_pcg(mv, prec, P.b, 1e-17, 200, mr)
        assert rso == rsn == mr and sto == stn == 1
        assert abs(nito - nitn) <= 1 + mr
        # a segment stops at the first recursive residual that meets tol, so
        # the history holds exactly one such value per segment, the last last
        assert np.sum(ho <= 1e-17) == mr + 1 and ho[-1] <= 1e-17 and len(rits) == mr
        np.testing.assert_allclose(ho[:5], hn[:5], rtol=1e-12)
        assert 0.0 < tro <= 1e-14
        np.testing.assert_allclose(xo, xs, rtol=0, atol=1e-12 * np.abs(xs).max())
