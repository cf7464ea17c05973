"""Numeric level setup on the GPU (Section 4: local bases of eq. 4.3, the
Galerkin product, the coarse smooth vectors) through the C ABI, against the
setup oracle on the inputs stored in the hierarchy files (every level's
matrix, smooth vectors and aggregates):

* the widths k_a exactly (the truncation decision, both sides in binary64);
* U_a element by element to 1e-10 (both sides fix the sign, unit columns);
* the dropped sum of squares to 1e-8 relative (plus 1e-14 of the largest);
* A_c = P^T A P against the oracle's product with the same bases, exactly
  symmetric, every entry within 2 N u of the sum of the absolute values of
  its terms, (|P|^T |A| |P|)_IJ: both sides add the same N terms (N at most
  n_a times the longest row) in different orders, each with a rounding error
  of at most N u relative to that sum (u = 1.2e-16, a little above 2^-53 for
  the FMA the GPU may use);
* W_c = P^T W the same way with (|P|^T |W|) and N = n_a;
and the host setup's own coarse matrices (built on bases up to 2e-11 away)
to 1e-7 of the same sums plus 1e-14 of the largest entry."""
import sys

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import setup_ref
from oracle.hierfile import read_hierarchy
from paper_1907_04417_amd import gpu_setup, workloads

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _check_level(H, l, tol):
    lev, nxt, T = H.levels[l], H.levels[l + 1], H.transfers[l]
    out = gpu_setup.setup_level(lev.rowptr, lev.col, lev.val, lev.W, T.aptr, T.arows, tol)
    # the bases against the oracle's SVD
    Us, ks, drops = setup_ref.level_bases(lev.W, T.aptr, T.arows, tol)
    assert np.array_equal(out["k"], ks)
    du = max(np.abs(out["U"][a] - Us[a]).max() for a in range(T.nagg))
    assert du <= 1e-10, du
    scale = max(float(np.max(np.sum(lev.W ** 2, axis=0))), 1e-300)
    assert np.all(np.abs(out["dropped"] - drops) <= 1e-8 * np.abs(drops) + 1e-14 * scale)
    # the products against the oracle's with the same (GPU) bases: rounding only
    A = sp.csr_matrix((lev.val, lev.col, lev.rowptr), shape=(lev.n, lev.n))
    P = setup_ref.prolongator(lev.n, T.aptr, T.arows, out["U"])
    Aco = setup_ref.galerkin(A, P)
    nc = int(out["coff"][-1])
    Acg = sp.csr_matrix((out["val_c"], out["col_c"], out["rowptr_c"]), shape=(nc, nc))
    assert (Acg - Acg.T).count_nonzero() == 0  # exactly symmetric (sparse: no dense copies)
    u = 1.2e-16
    N = int(np.diff(T.aptr).max()) * int(np.diff(lev.rowptr).max())
    absP = abs(P)
    bound = (absP.T @ abs(A) @ absP).tocsr()
    excess = (abs(Acg - Aco) - bound * (2 * N * u)).tocsr()
    assert excess.nnz == 0 or excess.data.max() <= 0.0, excess.data.max()
    Wco = setup_ref.restrict_vectors(P, lev.W)
    wb = (absP.T @ np.abs(lev.W)) * (2 * int(np.diff(T.aptr).max()) * u)
    assert np.all(np.abs(out["Wc"] - Wco) <= wb)
    # the host setup's coarse matrix (its own bases, up to 2e-11 away from the
    # oracle's on these inputs): agreement to 1e-7 of the same sums, plus 1e-14
    # of the largest entry for entries whose sums nearly vanish
    Af = sp.csr_matrix((nxt.val, nxt.col, nxt.rowptr), shape=(nxt.n, nxt.n))
    excess = (abs(Acg - Af) - bound * 1e-7).tocsr()
    assert excess.nnz == 0 or excess.data.max() <= 1e-14 * np.abs(Af.data).max()
    dA = abs(Acg - Aco).max() / np.abs(Aco.data).max()
    return T.nagg, nc, du, dA


@pytest.mark.parametrize("name", ["jump16", "aniso64", "elast12", "jump32", "aniso520"])
def test_level_setup_parity(name, torch_gpu):
    P, path, st = workloads.load(name)
    H = read_hierarchy(path)
    for l in range(len(H.transfers)):
        nagg, nc, du, da = _check_level(H, l, float(H.params[0]))
        _say(f"[gpu setup] {name} level {l}: {nagg} aggregates -> {nc} coarse dofs, |dU| {du:.1e}, |dA|/max {da:.1e}")


@pytest.mark.slow
def test_level_setup_full_size_jump128(torch_gpu):
    P, path, st = workloads.load("jump128")
    H = read_hierarchy(path)
    for l in range(len(H.transfers)):
        nagg, nc, du, da = _check_level(H, l, float(H.params[0]))
        _say(f"[gpu setup] jump128 level {l}: {nagg} aggregates -> {nc} coarse dofs, |dU| {du:.1e}, |dA|/max {da:.1e}")
