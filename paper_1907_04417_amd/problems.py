"""Seeded synthetic PDE matrices and right-hand sides.

This module only assembles test problems (sparse s.p.d. matrices in CSR form,
exact solutions and right-hand sides).  It contains none of the AMG method's
arithmetic, so both the HIP solve path and the CPU oracle may take their inputs
from it.  Every random draw comes from ``numpy.random.default_rng(seed)``
(PCG64), in the order documented in each function.

Problem families (stand-ins for the paper's test matrices, Section 5):

* ``aniso9``   -- rotated anisotropic diffusion -div(K grad u) on the unit
  square with the coefficient matrix K of Section 5.1 (a = eps + cos^2 theta,
  b = eps + sin^2 theta, c = cos theta sin theta), 9-point finite differences.
* ``jump7``    -- 3-D diffusion with piecewise-constant jumping coefficient,
  7-point finite differences, harmonic-mean face coefficients.
* ``elast_q1`` -- 3-D linear elasticity (Lame equations of Section 5.2) with
  trilinear hexahedral elements and node-based ordering of the three
  displacement components per node.
* ``grf_fv5``  -- cell-centred 5-point finite volumes with conductivity exp(g),
  g a Gaussian random field.
* ``block_rhs``   -- many right-hand sides B = A X* for one matrix.
* ``aniso_batch`` -- many independent ``aniso9`` problems of uneven size,
  anisotropy and angle.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp


@dataclass
class Problem:
    """A sparse s.p.d. system A x = b in CSR form (int32 indices, float64 values)."""

    name: str
    rowptr: np.ndarray
    col: np.ndarray
    val: np.ndarray
    b: np.ndarray
    x_star: np.ndarray | None = None
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.rowptr.shape[0] - 1)

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def scipy(self) -> sp.csr_matrix:
        return sp.csr_matrix((self.val, self.col, self.rowptr), shape=(self.n, self.n))


def _to_csr(rows, cols, vals, n) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    A = sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()
    A.sum_duplicates()
    A.sort_indices()
    A.eliminate_zeros()
    return (A.indptr.astype(np.int32), A.indices.astype(np.int32),
            A.data.astype(np.float64))


def _symmetrize_exact(rowptr, col, val):
    """Make the stored values bitwise symmetric: v_ij = v_ji = (v_ij + v_ji)/2."""
    n = rowptr.shape[0] - 1
    A = sp.csr_matrix((val, col, rowptr), shape=(n, n))
    S = ((A + A.T) * 0.5).tocsr()
    S.sort_indices()
    return S.indptr.astype(np.int32), S.indices.astype(np.int32), S.data.astype(np.float64)


def aniso9_matrix(m: int, eps: float, theta: float):
    """9-point FD matrix (times h^2) of -div(K grad u) on an m x m interior grid.

    K = [[a, c], [c, b]] with a = eps + cos^2(theta), b = eps + sin^2(theta),
    c = cos(theta) sin(theta) (Section 5.1).  The mixed derivative uses the
    central cross difference, so the stencil is
        centre 2(a+b); east/west -a; north/south -b; NE/SW -c/2; NW/SE +c/2.
    It is s.p.d. for every eps > 0 since ab - c^2 = eps(1 + eps) > 0.
    Nodes are numbered x-fastest: k = iy*m + ix.  Homogeneous Dirichlet.
    """
    a = eps + math.cos(theta) ** 2
    b = eps + math.sin(theta) ** 2
    c = math.cos(theta) * math.sin(theta)
    iy, ix = np.meshgrid(np.arange(m), np.arange(m), indexing="ij")
    ix = ix.ravel()
    iy = iy.ravel()
    k = iy * m + ix
    stencil = [(0, 0, 2.0 * (a + b)), (1, 0, -a), (-1, 0, -a), (0, 1, -b), (0, -1, -b),
               (1, 1, -0.5 * c), (-1, -1, -0.5 * c), (-1, 1, 0.5 * c), (1, -1, 0.5 * c)]
    R, C, V = [], [], []
    for dx, dy, w in stencil:
        if w == 0.0:
            continue
        jx = ix + dx
        jy = iy + dy
        ok = (jx >= 0) & (jx < m) & (jy >= 0) & (jy < m)
        R.append(k[ok])
        C.append((jy * m + jx)[ok])
        V.append(np.full(int(ok.sum()), w))
    return _to_csr(np.concatenate(R), np.concatenate(C), np.concatenate(V), m * m)


def aniso9(m: int = 64, eps: float = 1e-2, theta: float = math.pi / 4, seed: int = 0) -> Problem:
    """Rotated anisotropic diffusion; b = A x*, x* ~ U[-1, 1] (one draw of n uniforms)."""
    rp, ci, v = aniso9_matrix(m, eps, theta)
    n = m * m
    rng = np.random.default_rng(seed)
    xs = rng.uniform(-1.0, 1.0, n)
    A = sp.csr_matrix((v, ci, rp), shape=(n, n))
    return Problem(f"aniso9_m{m}", rp, ci, v, A @ xs, xs,
                   dict(m=m, eps=eps, theta=theta, seed=seed))


def ani_p1_matrix(m: int, eps: float, theta: float):
    """Linear finite elements for -div(K grad u) (K of Section 5.1) on the unit
    square with homogeneous Dirichlet boundary: a structured triangulation of
    (m + 1)^2 squares, each cut by its south-west to north-east diagonal, and
    the m^2 interior nodes as unknowns (numbered x-fastest).  The element
    matrix of a triangle T is |T| G^T K G, G the gradients of its barycentric
    functions; the sum over elements is exact (no quadrature error)."""
    a = eps + math.cos(theta) ** 2
    b = eps + math.sin(theta) ** 2
    c = math.cos(theta) * math.sin(theta)
    K = np.array([[a, c], [c, b]])
    N = m + 2  # grid points per side, boundary included
    h = 1.0 / (m + 1)
    gy, gx = np.meshgrid(np.arange(N - 1), np.arange(N - 1), indexing="ij")
    gx, gy = gx.ravel(), gy.ravel()
    node = lambda x, y: y * N + x  # noqa: E731
    # the two triangles of every square, vertices counter-clockwise
    tris = np.concatenate([
        np.stack([node(gx, gy), node(gx + 1, gy), node(gx + 1, gy + 1)], axis=1),
        np.stack([node(gx, gy), node(gx + 1, gy + 1), node(gx, gy + 1)], axis=1)])
    xy = np.stack([(np.arange(N * N) % N) * h, (np.arange(N * N) // N) * h], axis=1)
    p = xy[tris]                      # (ntri, 3, 2)
    e1, e2 = p[:, 1] - p[:, 0], p[:, 2] - p[:, 0]
    det = e1[:, 0] * e2[:, 1] - e1[:, 1] * e2[:, 0]
    area = 0.5 * det
    # gradients of the barycentric functions: rows of inv([e1 e2])^T, lambda_0 = 1 - l1 - l2
    g1 = np.stack([e2[:, 1], -e2[:, 0]], axis=1) / det[:, None]
    g2 = np.stack([-e1[:, 1], e1[:, 0]], axis=1) / det[:, None]
    G = np.stack([-(g1 + g2), g1, g2], axis=1)  # (ntri, 3, 2)
    Ke = area[:, None, None] * np.einsum("tik,kl,tjl->tij", G, K, G)
    rows = np.repeat(tris, 3, axis=1).ravel()
    cols = np.tile(tris, (1, 3)).ravel()
    Aall = sp.coo_matrix((Ke.ravel(), (rows, cols)), shape=(N * N, N * N)).tocsr()
    inner = ((xy[:, 0] > 0.5 * h) & (xy[:, 0] < 1 - 0.5 * h) & (xy[:, 1] > 0.5 * h) & (xy[:, 1] < 1 - 0.5 * h))
    idx = np.flatnonzero(inner)
    A = Aall[idx][:, idx].tocsr()
    A.eliminate_zeros()
    A.sort_indices()
    rp, ci, v = A.indptr.astype(np.int32), A.indices.astype(np.int32), A.data.astype(np.float64)
    return _symmetrize_exact(rp, ci, v)


def ani_p1(m: int, eps: float = 1e-3, theta: float = 0.0) -> Problem:
    """The paper's ANI test problems (Section 5.1: eps = 1e-3, theta = 0 for
    ANI1, pi/8 for ANI2) with linear elements on a structured triangulation of
    m^2 interior nodes, and the unit vector as right-hand side, as in the
    paper's runs (no random draw)."""
    rp, ci, v = ani_p1_matrix(m, eps, theta)
    n = m * m
    return Problem(f"ani_p1_m{m}", rp, ci, v, np.ones(n), None, dict(m=m, eps=eps, theta=theta))


def block_rhs(P: Problem, k: int, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """k right-hand sides B = A X* for one matrix, X* ~ U[-1, 1] drawn as one
    (n, k) array (row-major: row i holds the k values of unknown i).
    Returns (B, X*), both n x k C-contiguous."""
    rng = np.random.default_rng(seed)
    X = rng.uniform(-1.0, 1.0, size=(P.n, k))
    B = np.ascontiguousarray(P.scipy() @ X)
    return B, X


def aniso_batch(nprob: int = 64, smin: int = 32, smax: int = 512, seed: int = 0) -> list[Problem]:
    """Independent rotated anisotropic problems of uneven size.

    Draws from default_rng(seed), in this order: nprob grid sides uniform on
    the integers smin..smax, nprob values log10(eps) uniform on [-4, 0], nprob
    angles theta uniform on [0, pi).  Problem p is then aniso9(side_p, eps_p,
    theta_p, seed = 1000 * seed + 1 + p) (its own x*)."""
    rng = np.random.default_rng(seed)
    sides = rng.integers(smin, smax + 1, size=nprob)
    leps = rng.uniform(-4.0, 0.0, size=nprob)
    theta = rng.uniform(0.0, math.pi, size=nprob)
    return [aniso9(int(sides[p]), float(10.0 ** leps[p]), float(theta[p]), seed=1000 * seed + 1 + p)
            for p in range(nprob)]


def jump7_coefficient(m: int, cube: int, p: float, rng) -> np.ndarray:
    """Nodal coefficient kappa on an m^3 grid (x fastest).

    The grid is cut into (m/cube)^3 cubes.  Each cube is selected with
    probability p (first draw: one uniform per cube); a selected cube gets
    1e3 or 1e-3 with equal probability (second draw: one uniform per cube);
    all other cubes get 1.
    """
    nc = m // cube
    sel = rng.uniform(size=(nc, nc, nc)) < p
    hi = rng.uniform(size=(nc, nc, nc)) < 0.5
    kc = np.where(sel, np.where(hi, 1e3, 1e-3), 1.0)
    kc = np.repeat(np.repeat(np.repeat(kc, cube, 0), cube, 1), cube, 2)
    return kc  # indexed [z, y, x]


def jump7_matrix(kappa: np.ndarray):
    """7-point FD diffusion matrix from nodal kappa[z, y, x] (x fastest numbering).

    Face coefficient = harmonic mean of the two nodes' kappa; a Dirichlet
    boundary face takes the node's own kappa; diagonal = sum of the six face
    coefficients.
    """
    mz, my, mx = kappa.shape
    n = mx * my * mz
    idx = np.arange(n).reshape(mz, my, mx)
    diag = np.zeros((mz, my, mx))
    R, C, V = [], [], []
    for axis in range(3):
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[axis] = slice(0, -1)
        hi[axis] = slice(1, None)
        k1 = kappa[tuple(lo)]
        k2 = kappa[tuple(hi)]
        f = 2.0 * k1 * k2 / (k1 + k2)
        i1 = idx[tuple(lo)].ravel()
        i2 = idx[tuple(hi)].ravel()
        R += [i1, i2]
        C += [i2, i1]
        V += [-f.ravel(), -f.ravel()]
        diag[tuple(lo)] += f
        diag[tuple(hi)] += f
        # boundary faces (Dirichlet ghost) on both ends of this axis
        first = [slice(None)] * 3
        last = [slice(None)] * 3
        first[axis] = slice(0, 1)
        last[axis] = slice(-1, None)
        diag[tuple(first)] += kappa[tuple(first)]
        diag[tuple(last)] += kappa[tuple(last)]
    R.append(idx.ravel())
    C.append(idx.ravel())
    V.append(diag.ravel())
    return _to_csr(np.concatenate(R), np.concatenate(C), np.concatenate(V), n)


def jump7(m: int = 128, cube: int = 8, p: float = 0.5, seed: int = 0) -> Problem:
    """3-D jump-coefficient diffusion.  Draw order: cube selection, cube
    high/low, then x* ~ U[-1, 1]; b = A x*."""
    rng = np.random.default_rng(seed)
    kap = jump7_coefficient(m, cube, p, rng)
    rp, ci, v = jump7_matrix(kap)
    n = m ** 3
    xs = rng.uniform(-1.0, 1.0, n)
    A = sp.csr_matrix((v, ci, rp), shape=(n, n))
    return Problem(f"jump7_m{m}", rp, ci, v, A @ xs, xs, dict(m=m, cube=cube, p=p, seed=seed))


def laplace7(m: int) -> Problem:
    """Constant-coefficient 7-point Laplacian on m^3 (b = A 1)."""
    rp, ci, v = jump7_matrix(np.ones((m, m, m)))
    n = m ** 3
    A = sp.csr_matrix((v, ci, rp), shape=(n, n))
    xs = np.ones(n)
    return Problem(f"laplace7_m{m}", rp, ci, v, A @ xs, xs, dict(m=m))


def q1_hex_stiffness(E: float, nu: float, h: float) -> np.ndarray:
    """24 x 24 stiffness matrix of a trilinear hexahedron (cube of side h) for
    isotropic linear elasticity (Lame equations, Section 5.2) with Young's
    modulus E and Poisson ratio nu: K = sum over the 2 x 2 x 2 Gauss points of
    B^T D B |J| w.  Local nodes in the order (x, y, z) in {0,1}^3, x fastest;
    dofs node-major (3 per node)."""
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    D = np.zeros((6, 6))
    D[:3, :3] = lam
    D[np.arange(3), np.arange(3)] += 2.0 * mu
    D[3:, 3:] = np.eye(3) * mu
    corners = np.array([[(a >> 0) & 1, (a >> 1) & 1, (a >> 2) & 1] for a in range(8)], dtype=float)
    g = 0.5 / math.sqrt(3.0)
    K = np.zeros((24, 24))
    for gp in np.array(np.meshgrid([0.5 - g, 0.5 + g], [0.5 - g, 0.5 + g], [0.5 - g, 0.5 + g], indexing="ij")).reshape(3, -1).T:
        # derivatives of the shape functions prod_d (c_d xi_d + (1 - c_d)(1 - xi_d)) on the unit cube
        dN = np.zeros((8, 3))
        for a, c in enumerate(corners):
            f = [c[d] * gp[d] + (1 - c[d]) * (1 - gp[d]) for d in range(3)]
            df = [2 * c[d] - 1 for d in range(3)]
            dN[a] = [df[0] * f[1] * f[2], f[0] * df[1] * f[2], f[0] * f[1] * df[2]]
        dN /= h
        B = np.zeros((6, 24))
        for a in range(8):
            bx, by, bz = dN[a]
            B[0, 3 * a], B[1, 3 * a + 1], B[2, 3 * a + 2] = bx, by, bz
            B[3, 3 * a], B[3, 3 * a + 1] = by, bx
            B[4, 3 * a + 1], B[4, 3 * a + 2] = bz, by
            B[5, 3 * a], B[5, 3 * a + 2] = bz, bx
        K += B.T @ D @ B * (h ** 3) / 8.0
    return K


def elast_q1(m: int = 48, radius: float = 3.0, frac: float = 0.1, seed: int = 0) -> Problem:
    """3-D linear elasticity (Section 5.2), trilinear hexahedra, node-based
    ordering (the three displacement components of a node are consecutive).

    Grid: m x m x m free nodes (x fastest) plus one clamped node layer at
    x = 0, i.e. m elements along x and m - 1 along y and z, spacing h = 1/m.
    Material: E = 1, nu = 0.3, with spherical inclusions of nu = 0.49 (radius
    `radius` cells): sphere centres are drawn uniformly in the box (three
    uniforms each, x then y then z) until the elements whose centre lies in a
    sphere make up at least `frac` of all elements.  Load: the face x = 1 is
    pushed downward (a force -h^2 in z on each of its nodes).  n = 3 m^3."""
    h = 1.0 / m
    nex, ney, nez = m, m - 1, m - 1
    rng = np.random.default_rng(seed)
    ex, ey, ez = np.meshgrid(np.arange(nex), np.arange(ney), np.arange(nez), indexing="ij")
    ex, ey, ez = ex.ravel(), ey.ravel(), ez.ravel()
    cx, cy, cz = (ex + 0.5) * h, (ey + 0.5) * h, (ez + 0.5) * h
    incl = np.zeros(ex.shape[0], dtype=bool)
    r2 = (radius * h) ** 2
    while incl.mean() < frac:
        c = rng.uniform(0.0, 1.0, size=3) * np.array([1.0, (m - 1) * h, (m - 1) * h])
        incl |= (cx - c[0]) ** 2 + (cy - c[1]) ** 2 + (cz - c[2]) ** 2 <= r2
    Ks = [q1_hex_stiffness(1.0, 0.3, h), q1_hex_stiffness(1.0, 0.49, h)]
    # global node of local corner (a, b, c) of element (ex, ey, ez): layer ex + a in x (0 = clamped)
    rows, cols, vals = [], [], []
    for mat in (0, 1):
        sel = incl if mat == 1 else ~incl
        exs, eys, ezs = ex[sel], ey[sel], ez[sel]
        dofs = np.empty((exs.shape[0], 24), dtype=np.int64)
        free = np.empty((exs.shape[0], 24), dtype=bool)
        for a in range(8):
            ix, iy, iz = exs + (a & 1), eys + ((a >> 1) & 1), ezs + ((a >> 2) & 1)
            node = (iz * m + iy) * m + (ix - 1)
            for d in range(3):
                dofs[:, 3 * a + d] = 3 * node + d
                free[:, 3 * a + d] = ix >= 1
        K = Ks[mat]
        ok = free[:, :, None] & free[:, None, :]
        R = np.broadcast_to(dofs[:, :, None], ok.shape)[ok]
        C = np.broadcast_to(dofs[:, None, :], ok.shape)[ok]
        V = np.broadcast_to(K[None, :, :], ok.shape)[ok]
        rows.append(R)
        cols.append(C)
        vals.append(V)
    n = 3 * m ** 3
    rp, ci, v = _to_csr(np.concatenate(rows), np.concatenate(cols), np.concatenate(vals), n)
    rp, ci, v = _symmetrize_exact(rp, ci, v)
    b = np.zeros(n)
    face = np.arange(m * m) * m + (m - 1)  # nodes with ix = m (x = 1): last free layer
    b[3 * face + 2] = -h * h
    return Problem(f"elast_q1_m{m}", rp, ci, v, b, None,
                   dict(m=m, radius=radius, frac=float(incl.mean()), seed=seed))


def random_vectors(n: int, k: int, seed: int) -> np.ndarray:
    """k independent U[-1, 1] vectors of length n, column-major (k, n) array.

    These are the random initial iterates of the bootstrap's testing phase
    (Algorithm 1); they are drawn here so that every consumer sees the same
    numbers."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, size=(k, n))


# ----------------------------------------------------------------------------
# Cell-centred finite volumes with conductivity exp(g), g a Gaussian random field

def grf(m: int, length: float = 0.05, sigma: float = 1.0, seed: int = 0) -> np.ndarray:
    """Gaussian random field on an m x m cell grid of the unit square with
    squared-exponential covariance sigma^2 exp(-r^2 / (2 length^2)).

    Sampled by spectral filtering of white noise (one standard-normal draw per
    node of a 2m x 2m periodic grid, row-major) with the square root of the
    covariance's spectral density exp(-2 pi^2 length^2 |k|^2), cropped to
    m x m and rescaled to zero mean and unit pointwise variance times sigma."""
    rng = np.random.default_rng(seed)
    M = 2 * m
    h = 1.0 / m
    noise = rng.standard_normal((M, M))
    k = np.fft.fftfreq(M, d=h)
    k2 = k[:, None] ** 2 + k[None, :] ** 2
    filt = np.exp(-np.pi ** 2 * length ** 2 * k2)  # sqrt of exp(-2 pi^2 l^2 |k|^2)
    f = np.real(np.fft.ifft2(np.fft.fft2(noise) * filt))[:m, :m]
    f = (f - f.mean()) / f.std()
    return sigma * f


class FV5:
    """Pattern of the 5-point cell-centred finite-volume matrix on m x m cells
    (x fastest) and the map from conductivities to its CSR values.

    Face transmissibility between cells a and b: 2 k_a k_b / (k_a + k_b);
    Dirichlet boundary face of cell c: 2 k_c; A_cc = sum of the cell's face
    transmissibilities, A_ab = -T_ab.  Right-hand side h^2 * 1."""

    def __init__(self, m: int):
        self.m = m
        n = m * m
        self.n = n
        idx = np.arange(n).reshape(m, m)
        fa = np.concatenate([idx[:, :-1].ravel(), idx[:-1, :].ravel()])
        fb = np.concatenate([idx[:, 1:].ravel(), idx[1:, :].ravel()])
        self.fa, self.fb = fa, fb
        # boundary faces: one per cell side on the domain boundary
        bc = np.concatenate([idx[:, 0], idx[:, -1], idx[0, :], idx[-1, :]])
        self.bc = bc
        rows = np.concatenate([np.arange(n), fa, fb])
        cols = np.concatenate([np.arange(n), fb, fa])
        A = sp.coo_matrix((np.arange(rows.shape[0], dtype=np.float64) + 1, (rows, cols)), shape=(n, n)).tocsr()
        A.sort_indices()
        self.rowptr = A.indptr.astype(np.int32)
        self.col = A.indices.astype(np.int32)
        order = (A.data - 1).astype(np.int64)  # position k of the CSR array came from triple order[k]
        inv = np.empty_like(order)
        inv[order] = np.arange(order.shape[0])
        self.pos_diag = inv[:n]
        nf = fa.shape[0]
        self.pos_ab = inv[n:n + nf]
        self.pos_ba = inv[n + nf:]
        self.b = np.full(n, 1.0 / (m * m))

    def values(self, kappa: np.ndarray) -> np.ndarray:
        k = kappa.ravel()
        T = 2.0 * k[self.fa] * k[self.fb] / (k[self.fa] + k[self.fb])
        v = np.zeros(self.col.shape[0])
        d = np.zeros(self.n)
        np.add.at(d, self.fa, T)
        np.add.at(d, self.fb, T)
        np.add.at(d, self.bc, 2.0 * k[self.bc])
        v[self.pos_diag] = d
        v[self.pos_ab] = -T
        v[self.pos_ba] = -T
        return v

    def values_torch(self, g):
        """CSR values as a differentiable function of g (torch), kappa = exp(g)."""
        import torch
        k = torch.exp(g.reshape(-1))
        dev = k.device
        fa = torch.as_tensor(self.fa, device=dev)
        fb = torch.as_tensor(self.fb, device=dev)
        bc = torch.as_tensor(self.bc, device=dev)
        T = 2.0 * k[fa] * k[fb] / (k[fa] + k[fb])
        d = torch.zeros(self.n, dtype=k.dtype, device=dev)
        d = d.index_add(0, fa, T).index_add(0, fb, T).index_add(0, bc, 2.0 * k[bc])
        v = torch.zeros(self.col.shape[0], dtype=k.dtype, device=dev)
        v = v.index_copy(0, torch.as_tensor(self.pos_diag, device=dev), d)
        v = v.index_copy(0, torch.as_tensor(self.pos_ab, device=dev), -T)
        v = v.index_copy(0, torch.as_tensor(self.pos_ba, device=dev), -T)
        return v


def grf_fv5(m: int = 1024, seed: int = 0) -> Problem:
    """The differentiable-solve workload: kappa = exp(g), g a GRF (seed), the
    5-point FV matrix and b = h^2 * 1."""
    g = grf(m, seed=seed)
    fv = FV5(m)
    v = fv.values(np.exp(g))
    return Problem(f"grf_fv5_m{m}", fv.rowptr, fv.col, v, fv.b.copy(), None, dict(m=m, seed=seed, g=g, fv=fv))
