"""Input generators (no GPU): the finite-volume map g -> A(g) used by the
differentiable solve, the Gaussian random field, and the linear-element
anisotropic problems of the paper's Section 5.1."""
import math

import numpy as np
import pytest
import scipy.sparse as sp
import torch

from paper_1907_04417_amd import problems


def test_fv5_matrix_is_spd_and_matches_definition():
    m = 6
    rng = np.random.default_rng(0)
    g = rng.standard_normal((m, m))
    fv = problems.FV5(m)
    v = fv.values(np.exp(g))
    A = np.zeros((m * m, m * m))
    rows = np.repeat(np.arange(m * m), np.diff(fv.rowptr))
    A[rows, fv.col] = v
    k = np.exp(g)
    # definition, cell by cell: harmonic-mean transmissibilities, 2 k_c on the boundary
    for j in range(m):
        for i in range(m):
            c = j * m + i
            d = 0.0
            for (jj, ii) in ((j, i - 1), (j, i + 1), (j - 1, i), (j + 1, i)):
                if 0 <= jj < m and 0 <= ii < m:
                    t = 2 * k[j, i] * k[jj, ii] / (k[j, i] + k[jj, ii])
                    assert A[c, jj * m + ii] == -t
                    d += t
                else:
                    d += 2 * k[j, i]
            assert np.isclose(A[c, c], d, rtol=1e-14)
    assert np.array_equal(A, A.T)
    np.linalg.cholesky(A)


def test_fv5_torch_values_and_derivative():
    m = 5
    fv = problems.FV5(m)
    g = torch.tensor(np.random.default_rng(1).standard_normal(m * m), dtype=torch.float64, requires_grad=True)
    v = fv.values_torch(g)
    assert np.array_equal(v.detach().numpy(), fv.values(np.exp(g.detach().numpy())))
    w = torch.tensor(np.random.default_rng(2).standard_normal(v.shape[0]), dtype=torch.float64)
    (v * w).sum().backward()
    h = 1e-6
    for i in range(0, m * m, 3):
        gp = g.detach().numpy().copy()
        gm = gp.copy()
        gp[i] += h
        gm[i] -= h
        fd = (fv.values(np.exp(gp)) - fv.values(np.exp(gm))) @ w.numpy() / (2 * h)
        assert abs(fd - g.grad[i].item()) <= 1e-6 * max(1.0, abs(fd))


def test_grf_moments_and_correlation_length():
    g = problems.grf(128, length=0.05, seed=4)
    assert abs(g.mean()) < 1e-12 and abs(g.std() - 1.0) < 1e-12
    # neighbouring cells (h = 1/128 << 0.05) are strongly correlated, far ones are not
    c1 = np.corrcoef(g[:, :-1].ravel(), g[:, 1:].ravel())[0, 1]
    c40 = np.corrcoef(g[:, :-40].ravel(), g[:, 40:].ravel())[0, 1]
    assert c1 > 0.9 and abs(c40) < 0.2


def test_q1_stiffness_kernel_is_the_rigid_body_modes():
    """The trilinear element matrix is symmetric positive semidefinite and its
    null space is exactly the 6 rigid-body modes (3 translations, 3 rotations)."""
    from paper_1907_04417_amd import problems
    h = 0.25
    K = problems.q1_hex_stiffness(1.0, 0.3, h)
    assert np.abs(K - K.T).max() <= 1e-14 * np.abs(K).max()
    ev = np.linalg.eigvalsh(K)
    assert np.sum(np.abs(ev) <= 1e-12 * ev.max()) == 6 and ev.min() > -1e-12 * ev.max()
    corners = np.array([[(a >> 0) & 1, (a >> 1) & 1, (a >> 2) & 1] for a in range(8)], dtype=float) * h
    modes = []
    for d in range(3):
        t = np.zeros((8, 3))
        t[:, d] = 1.0
        modes.append(t.ravel())
    for (i, j) in ((0, 1), (1, 2), (0, 2)):
        r = np.zeros((8, 3))
        r[:, i], r[:, j] = -corners[:, j], corners[:, i]
        modes.append(r.ravel())
    for v in modes:
        assert np.abs(K @ v).max() <= 1e-12 * np.abs(K).max() * np.abs(v).max()


def test_elast_q1_assembly():
    """Clamped assembly is symmetric positive definite with node-based
    ordering; away from the clamp a translation is in the kernel of the rows
    whose element patch is complete (interior nodes)."""
    from paper_1907_04417_amd import problems
    P = problems.elast_q1(5, seed=1)
    A = P.scipy().toarray()
    assert P.n == 3 * 5 ** 3 and np.array_equal(A, A.T)
    assert np.linalg.eigvalsh(A).min() > 0.0
    # rows of an interior node (ix = 2, iy = 2, iz = 2 of the free grid) annihilate translations
    node = (2 * 5 + 2) * 5 + 2
    for d in range(3):
        t = np.zeros(P.n)
        t[d::3] = 1.0
        assert np.abs((A @ t)[3 * node:3 * node + 3]).max() <= 1e-12 * np.abs(A).max()
    # load on the face x = 1 only, downward
    assert np.all(P.b[0::3] == 0.0) and np.all(P.b[1::3] == 0.0) and P.b.sum() < 0.0
    assert 0.1 <= P.meta["frac"]


def test_block_rhs_and_batch_draws():
    from paper_1907_04417_amd import problems
    P = problems.aniso9(8, seed=0)
    B, X = problems.block_rhs(P, 3, seed=2)
    assert B.shape == (P.n, 3) and B.flags.c_contiguous
    assert np.allclose(B, P.scipy() @ X, rtol=0, atol=1e-14)
    Ps = problems.aniso_batch(5, 10, 20, seed=3)
    sides = [p.meta["m"] for p in Ps]
    assert all(10 <= s <= 20 for s in sides)
    assert all(1e-4 <= p.meta["eps"] <= 1.0 and 0.0 <= p.meta["theta"] < np.pi for p in Ps)
    assert [p.meta["seed"] for p in Ps] == [3001 + p for p in range(5)]


def test_ani_p1_reduces_to_five_point_at_theta_zero():
    """Linear elements on right triangles couple no nodes across the
    diagonals when K is diagonal: at theta = 0 the matrix is the 5-point
    difference stencil (times h^2)."""
    rp, ci, v = problems.ani_p1_matrix(9, 1e-3, 0.0)
    r2, c2, v2 = problems.aniso9_matrix(9, 1e-3, 0.0)
    A = sp.csr_matrix((v, ci, rp), shape=(81, 81)).toarray()
    B = sp.csr_matrix((v2, c2, r2), shape=(81, 81)).toarray()
    assert np.abs(A - B).max() <= 1e-14


@pytest.mark.parametrize("theta", [0.0, math.pi / 8, 1.0])
def test_ani_p1_consistent_on_quadratics(theta):
    """At nodes whose neighbours are all interior, the element stencil applied
    to u = x^2, x y, y^2 gives h^2 (-div K grad u) = -2 h^2 a, -2 h^2 c,
    -2 h^2 b exactly (up to rounding); the matrix is symmetric and s.p.d."""
    m, eps = 12, 1e-3
    h = 1.0 / (m + 1)
    a = eps + math.cos(theta) ** 2
    b = eps + math.sin(theta) ** 2
    c = math.cos(theta) * math.sin(theta)
    P = problems.ani_p1(m, eps, theta)
    A = P.scipy()
    assert abs(A - A.T).max() == 0.0
    assert np.linalg.eigvalsh(A.toarray()).min() > 0
    ix, iy = np.arange(m * m) % m, np.arange(m * m) // m
    x, y = (ix + 1) * h, (iy + 1) * h
    inner = (ix > 0) & (ix < m - 1) & (iy > 0) & (iy < m - 1)
    for u, want in ((x * x, -2 * a), (x * y, -2 * c), (y * y, -2 * b)):
        got = (A @ u)[inner] / h ** 2
        assert np.abs(got - want).max() <= 1e-9
    assert np.array_equal(P.b, np.ones(m * m))
