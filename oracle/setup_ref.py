"""Oracle of the numeric setup of one multiple-vector level (Section 4).

TEST INFRASTRUCTURE ONLY: plain, slow NumPy/SciPy restatements of what the
GPU setup kernels compute, used by the test suite.  Nothing in the product
path imports this module, and it shares no code with the library.

    aggregate_basis  eq. 4.3: the SVD of the n_a x m block of the smooth
                     vectors on one aggregate, truncated at TOL_a
    level_bases      every aggregate of a level, TOL_a = TOL * n_a / n_l
    prolongator      P = blockdiag(U_a) as a sparse matrix
    galerkin         A_c = P^T A P, made exactly symmetric
    restrict_vectors W_c = P^T W (the smooth vectors on the coarse level,
                     Section 4.1)
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def aggregate_basis(Wa: np.ndarray, tol_a: float):
    """Local basis of the smooth vectors on one aggregate (eq. 4.3): the left
    singular vectors of Wa (n_a x m) whose singular values exceed tol_a, at
    least one and at most min(n_a, m); each column's sign is fixed so that
    its entry of largest magnitude (the lowest row on ties) is positive.
    Returns (U, k, dropped), dropped the sum of the squared singular values
    not kept."""
    U, s, _ = np.linalg.svd(Wa, full_matrices=False)
    k = int(np.count_nonzero(s > tol_a))
    k = max(1, min(k, Wa.shape[0], Wa.shape[1]))
    U = U[:, :k].copy()
    for l in range(k):
        i = int(np.argmax(np.abs(U[:, l])))
        if U[i, l] < 0.0:
            U[:, l] = -U[:, l]
    return U, k, float(np.sum(s[k:] ** 2))


def level_bases(W: np.ndarray, aptr, arows, tol: float):
    """Every aggregate's basis with TOL_a = tol * n_a / n (n the level's size):
    (list of U_a, k array, dropped array)."""
    n = W.shape[0]
    Us, ks, drops = [], [], []
    for a in range(len(aptr) - 1):
        rows = np.asarray(arows[aptr[a]:aptr[a + 1]])
        U, k, d = aggregate_basis(W[rows], tol * len(rows) / n)
        Us.append(U)
        ks.append(k)
        drops.append(d)
    return Us, np.array(ks), np.array(drops)


def prolongator(n: int, aptr, arows, Us) -> sp.csr_matrix:
    """P with P[arows of a, coff_a .. coff_a + k_a) = U_a, coff the running
    sum of the k_a."""
    R, C, V = [], [], []
    c0 = 0
    for a in range(len(aptr) - 1):
        rows = np.asarray(arows[aptr[a]:aptr[a + 1]])
        U = Us[a]
        k = U.shape[1]
        R.append(np.repeat(rows, k))
        C.append(np.tile(np.arange(c0, c0 + k), len(rows)))
        V.append(U.ravel())
        c0 += k
    return sp.csr_matrix((np.concatenate(V), (np.concatenate(R), np.concatenate(C))), shape=(n, c0))


def galerkin(A: sp.csr_matrix, P: sp.csr_matrix) -> sp.csr_matrix:
    """A_c = P^T A P, with (A_c + A_c^T) / 2 so that it is exactly symmetric."""
    Ac = (P.T @ A @ P).tocsr()
    Ac = ((Ac + Ac.T) * 0.5).tocsr()
    Ac.sort_indices()
    return Ac


def restrict_vectors(P: sp.csr_matrix, W: np.ndarray) -> np.ndarray:
    """W_c = P^T W."""
    return np.asarray(P.T @ W)
