"""Pins of the setup oracle (oracle/setup_ref.py): the per-aggregate bases of
eq. 4.3, the Galerkin product and the restricted smooth vectors.

* Identities of the SVD: U^T U = I, ||(I - U U^T) W_a||_F^2 equals the sum of
  the squared dropped singular values, a rank-deficient block keeps only its
  rank, a one-row aggregate gives U = [1].
* The dense products P^T A P and P^T W.
* The host setup (a separate C++ implementation: one-sided Jacobi SVD,
  its own Galerkin loop) wrote the same bases, coarse matrices and coarse
  smooth vectors into the hierarchy files.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import setup_ref
from oracle.hierfile import read_hierarchy


def test_basis_identities():
    rng = np.random.default_rng(0)
    for na, m in ((40, 4), (7, 6), (3, 5), (64, 10)):
        Wa = rng.standard_normal((na, m)) * np.array([1.0, 1e-1, 1e-3, 1e-5, 1e-7, 1e-9, 1, 1, 1, 1][:m])
        U, k, dropped = setup_ref.aggregate_basis(Wa, 1e-4)
        s = np.linalg.svd(Wa, compute_uv=False)
        assert k == max(1, min(np.count_nonzero(s > 1e-4), na, m))
        assert np.abs(U.T @ U - np.eye(k)).max() <= 1e-14
        res = Wa - U @ (U.T @ Wa)
        assert abs(np.sum(res ** 2) - dropped) <= 1e-12 * max(np.sum(Wa ** 2), 1e-300)
        for l in range(k):
            i = np.argmax(np.abs(U[:, l]))
            assert U[i, l] > 0


def test_basis_special_cases():
    rng = np.random.default_rng(1)
    a = rng.standard_normal(20)
    Wa = np.stack([a, 2 * a, rng.standard_normal(20)], axis=1)  # rank 2
    U, k, dropped = setup_ref.aggregate_basis(Wa, 1e-10)
    assert k == 2 and dropped <= 1e-26 * np.sum(Wa ** 2)
    U, k, dropped = setup_ref.aggregate_basis(np.array([[-3.0, 1.0, 2.0]]), 0.1)
    assert k == 1 and U.shape == (1, 1) and U[0, 0] == 1.0
    assert abs(dropped) <= 1e-28


def test_dense_products():
    rng = np.random.default_rng(2)
    n = 30
    M = rng.standard_normal((n, n))
    A = sp.csr_matrix(M @ M.T + n * np.eye(n))
    aptr = np.array([0, 7, 15, 22, 30])
    arows = rng.permutation(n)
    W = rng.standard_normal((n, 3))
    Us, ks, _ = setup_ref.level_bases(W, aptr, arows, 1e-3)
    P = setup_ref.prolongator(n, aptr, arows, Us)
    Pd = np.zeros((n, int(ks.sum())))
    c = 0
    for a in range(4):
        Pd[arows[aptr[a]:aptr[a + 1]], c:c + ks[a]] = Us[a]
        c += ks[a]
    assert np.abs(P.toarray() - Pd).max() == 0.0
    assert np.abs(Pd.T @ Pd - np.eye(c)).max() <= 1e-14
    Ac = setup_ref.galerkin(A, P).toarray()
    assert np.abs(Ac - Pd.T @ A.toarray() @ Pd).max() <= 1e-12 * np.abs(Ac).max()
    assert np.array_equal(Ac, Ac.T)
    assert np.abs(setup_ref.restrict_vectors(P, W) - Pd.T @ W).max() <= 1e-13


@pytest.mark.parametrize("fx", ["tiny_hier", "small3d_hier"])
def test_host_setup_agrees(fx, request):
    P, path, st = request.getfixturevalue(fx)
    H = read_hierarchy(path)
    for l, T in enumerate(H.transfers):
        lev, nxt = H.levels[l], H.levels[l + 1]
        assert lev.W is not None and nxt.W is not None
        # params[0] is TOL of the truncation (Section 5: 0.1)
        Us, ks, drops = setup_ref.level_bases(lev.W, T.aptr, T.arows, float(H.params[0]))
        assert np.array_equal(ks, np.diff(T.coff)), l
        for a in range(T.nagg):
            Uf = T.U[T.uoff[a]:T.uoff[a + 1]].reshape(-1, ks[a])
            assert np.abs(Uf - Us[a]).max() <= 1e-10, (l, a)
        assert np.allclose(drops, T.drop2, rtol=1e-8, atol=1e-14 * max(np.abs(lev.W).max(), 1.0) ** 2)
        A = sp.csr_matrix((lev.val, lev.col, lev.rowptr), shape=(lev.n, lev.n))
        Pm = setup_ref.prolongator(lev.n, T.aptr, T.arows, Us)
        Ac = setup_ref.galerkin(A, Pm)
        Af = sp.csr_matrix((nxt.val, nxt.col, nxt.rowptr), shape=(nxt.n, nxt.n))
        assert np.abs((Ac - Af).toarray()).max() <= 1e-10 * np.abs(Af.data).max()
        Wc = setup_ref.restrict_vectors(Pm, lev.W)
        assert np.abs(Wc - nxt.W).max() <= 1e-10 * np.abs(nxt.W).max()
