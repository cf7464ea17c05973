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


def l1_splitting(A):
    """M = diag(sum_j |a_ij|): an l1-Jacobi sweep maps x to x + M^{-1}(r - A x)
    (Baker, Falgout, Kolev and Yang, "Multigrid smoothers for ultraparallel
    computing", 2011)."""
    return np.diag(np.abs(A).sum(axis=1))


def vcycle_matrix(H, smoother="gs"):
    """B_0 of the symmetric V-cycle from the recursion
    E_l = (I - M_l^{-T} A_l)(I - P_l B_{l+1} P_l^T A_l)(I - M_l^{-1} A_l),
    B_l = (I - E_l) A_l^{-1}, B_L = A_L^{-1}; M_l is the Gauss-Seidel
    splitting in the level's order ("gs") or the l1 diagonal ("l1")."""
    L = H.nlevels - 1
    As = [dense(l.rowptr, l.col, l.val) for l in H.levels]
    B = np.linalg.inv(As[L])
    for l in range(L - 1, -1, -1):
        A = As[l]
        n = A.shape[0]
        M = gs_splitting(A, H.levels[l].order) if smoother == "gs" else l1_splitting(A)
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


def seq_dot(a, b):
    """Inner product summed left to right in binary64 (the order of a plain loop)."""
    s = 0.0
    for u, v in zip(a.tolist(), b.tolist()):
        s += u * v
    return s


def seq_csr_mv(rowptr, col, val, x):
    """y = A x with every row summed left to right over its stored entries."""
    y = np.zeros(len(rowptr) - 1)
    xl = x.tolist()
    for i in range(len(rowptr) - 1):
        s = 0.0
        for k in range(rowptr[i], rowptr[i + 1]):
            s += val[k] * xl[col[k]]
        y[i] = s
    return y


def flexible_pcg(mv, prec, b, tol, maxit, max_restarts, beta_rule="notay"):
    """Flexible preconditioned CG (Notay, "Flexible conjugate gradients",
    SIAM J. Sci. Comput. 22, 2000) with the truncation to one previous
    direction: beta_k = z_{k+1}^T (r_{k+1} - r_k) / (z_k^T r_k), which keeps
    p_{k+1} A-orthogonal to p_k when the preconditioner varies.  beta_rule
    "fletcher_reeves" uses z_{k+1}^T r_{k+1} / (z_k^T r_k) instead (the
    standard CG rule, for showing that the two are told apart).

    Stops when ||r_k|| <= tol ||r_0|| on the recursive residual; then the true
    residual b - A x is recomputed and, if it misses tol, the iteration starts
    again from x (r = b - A x, p = z), at most max_restarts times.  Returns
    (x, hist, nit, status, true_rel, restarts, restart_its): status 0
    converged, 1 not; restart_its lists the iteration count at each restart."""
    n = b.shape[0]
    x = np.zeros(n)
    r = b - mv(x)
    r0 = np.sqrt(seq_dot(r, r))
    hist = [1.0]
    it, restarts, restart_its, true_rel, status = 0, 0, [], 0.0, 1
    if r0 == 0.0:
        return x, np.array(hist), 0, 0, 0.0, 0, []
    for restart in range(max_restarts + 1):
        if it >= maxit:
            break
        if restart > 0:
            restarts = restart
            restart_its.append(it)
            r = b - mv(x)
        z = prec(r)
        p = z.copy()
        rho = seq_dot(r, z)
        met = False
        while it < maxit:
            q = mv(p)
            alpha = rho / seq_dot(p, q)
            x = x + alpha * p
            r_old = r
            r = r - alpha * q
            it += 1
            hist.append(np.sqrt(seq_dot(r, r)) / r0)
            if hist[-1] <= tol:
                met = True
                break
            z = prec(r)
            rho_new = seq_dot(r, z)
            if beta_rule == "notay":
                beta = seq_dot(z, r - r_old) / rho
            else:
                beta = rho_new / rho
            rho = rho_new
            p = z + beta * p
        res = b - mv(x)
        true_rel = np.sqrt(seq_dot(res, res)) / r0
        if met and true_rel <= tol:
            status = 0
            break
    return x, np.array(hist), it, status, true_rel, restarts, restart_its


def kcycle_dense(H, r, smoother="gs", level=0):
    """K-cycle of the hierarchy H applied to r, from its definition with dense
    matrices: the V-cycle's smoothing and transfers, and on a coarse level that
    is not the coarsest, the A-orthogonal projection of A_c^{-1} r_c on the
    span of c1 = K r_c and c2 = K (r_c - alpha1 A_c c1), alpha1 = c1^T r_c /
    c1^T A_c c1 (what two steps of flexible CG produce: Notay and
    Vassilevski, "Recursive Krylov-based multigrid cycles", 2008).  The
    projection is taken by solving the 2 x 2 Galerkin system, not by the CG
    recurrences."""
    L = H.nlevels - 1
    lv = H.levels[level]
    A = dense(lv.rowptr, lv.col, lv.val)
    if level == L:
        return np.linalg.solve(A, r)
    M = gs_splitting(A, lv.order) if smoother == "gs" else l1_splitting(A)
    nc = H.levels[level + 1].n
    P = prolongator(H.transfers[level], A.shape[0], nc)
    x = np.linalg.solve(M, r)
    rc = P.T @ (r - A @ x)
    if level + 1 == L:
        xc = np.linalg.solve(dense(H.levels[L].rowptr, H.levels[L].col, H.levels[L].val), rc)
    else:
        Ac = dense(H.levels[level + 1].rowptr, H.levels[level + 1].col, H.levels[level + 1].val)
        c1 = kcycle_dense(H, rc, smoother, level + 1)
        alpha1 = (c1 @ rc) / (c1 @ Ac @ c1)
        c2 = kcycle_dense(H, rc - alpha1 * (Ac @ c1), smoother, level + 1)
        V = np.stack([c1, c2], axis=1)
        xc = V @ np.linalg.solve(V.T @ Ac @ V, V.T @ rc)
    x = x + P @ xc
    x = x + np.linalg.solve(M.T, r - A @ x)
    return x
