"""Input generators (no GPU): the finite-volume map g -> A(g) used by the
differentiable solve, and the Gaussian random field."""
import numpy as np
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
