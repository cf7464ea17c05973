"""Pins of the oracle's K-cycle (nonlinear AMLI cycle, Section 5: two inner
flexible-CG iterations per level but the coarsest) and of CG preconditioned
by it, on tiny hierarchies of three and four levels.

* Against the cycle's definition in dense NumPy (tests.dense_ref.kcycle_dense),
  where the inner correction is the A-orthogonal projection on the two
  preconditioned directions, solved as a 2 x 2 Galerkin system.
* On a two-level hierarchy there is no inner level: K = V, bit for bit.
* K is homogeneous (K(2r) = 2 K(r) exactly) but not additive.
* The CG with K as preconditioner equals a NumPy flexible CG (Notay's beta)
  with the dense K, step by step.
"""
import numpy as np
import pytest

import oracle
from paper_1907_04417_amd import problems
from tests.conftest import make_hierarchy
from tests.dense_ref import dense, flexible_pcg, kcycle_dense


@pytest.fixture(scope="module")
def hier4(setup_lib, tmp_path_factory):
    """14 x 14 rotated anisotropic problem, four levels (inner FCG on levels 1
    and 2, the second nested in the first)."""
    P = problems.aniso9(14, seed=9)
    path, st = make_hierarchy(tmp_path_factory.mktemp("k4"), P, 3, boot_coarse_min=2, coarse_cap=6, compose=1)
    assert st["nlevels"] >= 4, st["n"]
    return P, path, st


@pytest.fixture(scope="module")
def hier2(setup_lib, tmp_path_factory):
    P = problems.aniso9(10, seed=4)
    path, st = make_hierarchy(tmp_path_factory.mktemp("k2"), P, 2, boot_coarse_min=4, coarse_cap=60, compose=1)
    assert st["nlevels"] == 2, st["n"]
    return P, path, st


@pytest.mark.parametrize("fx", ["tiny_hier", "small3d_hier", "hier4"])
@pytest.mark.parametrize("smoother", ["gs", "l1"])
def test_kcycle_equals_definition(fx, smoother, request):
    P, path, st = request.getfixturevalue(fx)
    assert st["nlevels"] >= 3
    O = oracle.Oracle(path, smoother=oracle.GS_COLOUR if smoother == "gs" else oracle.L1_JACOBI)
    rng = np.random.default_rng(7)
    for _ in range(3):
        r = rng.standard_normal(P.n)
        z = O.kcycle(r)
        zd = kcycle_dense(O.h, r, smoother)
        assert np.abs(z - zd).max() <= 1e-10 * np.abs(zd).max()
    # not the V-cycle: the inner iterations change the result
    assert np.abs(O.kcycle(r) - O.vcycle(r)).max() > 1e-6 * np.abs(zd).max()


def test_two_levels_kcycle_is_vcycle(hier2):
    P, path, st = hier2
    O = oracle.Oracle(path)
    r = np.random.default_rng(3).standard_normal(P.n)
    assert np.array_equal(O.kcycle(r), O.vcycle(r))


def test_kcycle_homogeneous_not_additive(hier4):
    P, path, st = hier4
    O = oracle.Oracle(path)
    rng = np.random.default_rng(5)
    r1, r2 = rng.standard_normal(P.n), rng.standard_normal(P.n)
    k1, k2 = O.kcycle(r1), O.kcycle(r2)
    assert np.array_equal(O.kcycle(2.0 * r1), 2.0 * k1)
    k12 = O.kcycle(r1 + r2)
    assert np.abs(k12 - (k1 + k2)).max() > 1e-6 * np.abs(k12).max()


@pytest.mark.parametrize("fx", ["small3d_hier", "hier4"])
def test_kcycle_pcg_is_flexible_cg(fx, request):
    P, path, st = request.getfixturevalue(fx)
    O = oracle.Oracle(path)
    A = O.matrix_dense(0)
    b = P.b
    x, hist, nit, status = O.pcg_kcycle(b, tol=1e-10, maxit=200)
    xd, hd, nitd, std, tr, _, _ = flexible_pcg(lambda v: A @ v, lambda v: kcycle_dense(O.h, v), b, 1e-10, 200, 0)
    assert status == 0 and std == 0 and nit == nitd
    # histories agree to rounding (relative to each entry, down to the 1e-10 tolerance)
    assert np.all(np.abs(hist - hd) <= 1e-8 * hd)
    assert np.abs(x - np.linalg.solve(A, b)).max() <= 1e-8 * np.abs(x).max()
    # no slower than the V-cycle preconditioner on the same system
    _, _, nit_v, _ = O.pcg(b, tol=1e-10, maxit=200)
    assert nit <= nit_v
