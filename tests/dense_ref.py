"""Dense NumPy restatements used to pin the oracle on tiny inputs.

These build the textbook closed forms of the operators (Gauss-Seidel
splitting matrices, block-diagonal prolongators, the V-cycle error
propagator) directly from the definitions, independent of the oracle's loops.
"""
import numpy as np


def dense(rowptr, col, val, n=None):
    n = len(rowptr) - 1 if n is None else n
    M = np.zeros((n, n))
    rows = np.repeat(np.arange(len(rowptr) - 1), np.diff(rowptr))
    np.add.at(M, (rows, np.asarray(col)), np.asarray(val))
    return M


def prolongator(T, nf, nc):
    """P = blockdiag(U_a) placed on the aggregates' rows and coarse columns."""
    P = np.zeros((nf, nc))
    for a in range(T.nagg):
        rows = T.arows[T.aptr[a]:T.aptr[a + 1]]
        k = T.coff[a + 1] - T.coff[a]
        U = T.U[T.uoff[a]:T.uoff[a + 1]].reshape(len(rows), k)
        P[rows, T.coff[a]:T.coff[a] + k] = U
    return P


def gs_splitting(A, order):
    """M = D + (part of A strictly earlier in the ordering): a forward
    Gauss-Seidel sweep in `order` maps x to x + M^{-1}(r - A x)."""
    n = A.shape[0]
    pos = np.empty(n, dtype=int)
    pos[np.asarray(order)] = np.arange(n)
    earlier = pos[None, :] < pos[:, None]
    return np.where(earlier | np.eye(n, dtype=bool), A, 0.0)


def vcycle_matrix(H):
    """B_0 of the symmetric V-cycle from the recursion
    E_l = (I - M_l^{-T} A_l)(I - P_l B_{l+1} P_l^T A_l)(I - M_l^{-1} A_l),
    B_l = (I - E_l) A_l^{-1}, B_L = A_L^{-1}."""
    L = H.nlevels - 1
    As = [dense(l.rowptr, l.col, l.val) for l in H.levels]
    B = np.linalg.inv(As[L])
    for l in range(L - 1, -1, -1):
        A = As[l]
        n = A.shape[0]
        M = gs_splitting(A, H.levels[l].order)
        P = prolongator(H.transfers[l], n, As[l + 1].shape[0])
        I = np.eye(n)
        E = (I - np.linalg.solve(M.T, A)) @ (I - P @ B @ P.T @ A) @ (I - np.linalg.solve(M, A))
        B = (I - E) @ np.linalg.inv(A)
    return B


def pcg_dense(A, B, b, tol, maxit):
    """Textbook preconditioned CG with an explicit preconditioner matrix B."""
    x = np.zeros_like(b)
    r = b.copy()
    r0 = np.linalg.norm(r)
    hist = [1.0]
    z = B @ r
    p = z.copy()
    rho = r @ z
    for _ in range(maxit):
        q = A @ p
        alpha = rho / (p @ q)
        x = x + alpha * p
        r = r - alpha * q
        hist.append(np.linalg.norm(r) / r0)
        if hist[-1] <= tol:
            break
        z = B @ r
        rho_new = r @ z
        p = z + (rho_new / rho) * p
        rho = rho_new
    return x, np.array(hist)
