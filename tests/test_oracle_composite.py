"""Pins of the oracle's composite AMG (the paper's original bootstrap AMG:
eq. 1.1, Algorithm 1, Section 5 item (i)) on the bootstrap hierarchies the
host setup writes for a tiny problem.

* The composite preconditioner equals (I - E) A^{-1} with
  E = F_1 .. F_r F_r .. F_1, F_k = I - B_k A, B_k the dense V-cycle matrix of
  hierarchy k from its recursion (tests.dense_ref.vcycle_matrix); with K-cycle
  components, the same product of the dense K-cycle definitions.
* The testing phase equals nu applications of the dense E and the A-norm
  ratio of the last two iterates.
* The setup's own estimate and smooth vector (computed by the host setup's
  separate C++ cycle) are reproduced from the same random start.
* CG preconditioned by the composite equals a NumPy flexible CG with the
  dense composite.
"""
import numpy as np
import pytest

import oracle
from oracle.hierfile import read_hierarchy
from paper_1907_04417_amd import problems
from paper_1907_04417_amd.setup import SetupParams, build_hierarchy
from tests.dense_ref import dense, flexible_pcg, kcycle_dense, vcycle_matrix

NVEC = 4


@pytest.fixture(scope="module")
def boot(setup_lib, tmp_path_factory):
    """16 x 16 rotated anisotropic problem, 3 bootstrap stages (B_1..B_3)."""
    d = tmp_path_factory.mktemp("boot")
    P = problems.aniso9(16, 1e-2, np.pi / 4, seed=6)
    x0 = problems.random_vectors(P.n, NVEC - 1, 1000)
    st = build_hierarchy(P.rowptr, P.col, P.val, str(d / "main.bin"), x0,
                         SetupParams(nvec_max=NVEC, boot_coarse_min=6, rho_des=0.0),
                         boot_prefix=str(d / "boot"))
    paths = [str(d / f"boot_b{r}.bin") for r in range(1, len(st["rho"]) + 1)]
    assert len(paths) == NVEC - 1
    return P, x0, st, str(d / "main.bin"), paths


def _E(P, Bs):
    A = dense(P.rowptr, P.col, P.val)
    I = np.eye(P.n)
    E = I
    for k in list(range(len(Bs))) + list(reversed(range(len(Bs)))):
        E = (I - Bs[k] @ A) @ E
    return A, E


def test_bootstrap_files_are_hierarchies(boot):
    P, x0, st, main, paths = boot
    for p in paths:
        H = read_hierarchy(p)
        assert H.levels[0].n == P.n and np.array_equal(H.levels[0].val, P.val)
        for l, T in enumerate(H.transfers):
            assert np.array_equal(np.diff(T.coff), np.ones(T.nagg, dtype=np.int64))  # one column each
            for a in range(T.nagg):
                u = T.U[T.uoff[a]:T.uoff[a + 1]]
                assert abs(u @ u - 1.0) <= 1e-14


@pytest.mark.parametrize("r", [1, 2, 3])
def test_composite_equals_closed_form(boot, r):
    P, x0, st, main, paths = boot
    Os = [oracle.Oracle(p) for p in paths[:r]]
    C = oracle.Composite(Os)
    Bs = [vcycle_matrix(O.h) for O in Os]
    A, E = _E(P, Bs)
    Bc = (np.eye(P.n) - E) @ np.linalg.inv(A)
    rng = np.random.default_rng(2)
    for _ in range(2):
        v = rng.standard_normal(P.n)
        z = C.apply(v)
        zd = Bc @ v
        assert np.abs(z - zd).max() <= 1e-10 * np.abs(zd).max()
    if r == 1:
        # one hierarchy: (I - B A)^2 gives 2 B - B A B
        assert np.allclose(Bc, 2 * Bs[0] - Bs[0] @ A @ Bs[0], rtol=0, atol=1e-10 * np.abs(Bc).max())


def test_composite_with_kcycles(boot):
    P, x0, st, main, paths = boot
    Os = [oracle.Oracle(p) for p in paths]
    C = oracle.Composite(Os, kcycle=True)
    A = dense(P.rowptr, P.col, P.val)
    v = np.random.default_rng(4).standard_normal(P.n)
    z = np.zeros(P.n)
    for k in [0, 1, 2, 2, 1, 0]:
        z = z + kcycle_dense(Os[k].h, v - A @ z)
    got = C.apply(v)
    assert np.abs(got - z).max() <= 1e-10 * np.abs(z).max()
    assert np.abs(got - oracle.Composite(Os).apply(v)).max() > 1e-8 * np.abs(z).max()


def test_testing_phase_equals_power_iteration(boot):
    P, x0, st, main, paths = boot
    Os = [oracle.Oracle(p) for p in paths[:2]]
    A, E = _E(P, [vcycle_matrix(O.h) for O in Os])
    x = x0[1].copy()
    prev = None
    for _ in range(15):
        prev = x
        x = E @ x
    an, ap = np.sqrt(x @ A @ x), np.sqrt(prev @ A @ prev)
    w, rho = oracle.Composite(Os).test(x0[1], nu=15)
    assert abs(rho - an / ap) <= 1e-10 * rho
    assert np.abs(w - x / an).max() <= 1e-9 * np.abs(x / an).max()


def test_testing_phase_reproduces_the_setup(boot):
    """Stage r of the setup tested the composite of B_1..B_r from the r-th
    random start and kept x^nu / ||x^nu||_A as w_r: the oracle, from the same
    start, gets the setup's estimate and vector."""
    P, x0, st, main, paths = boot
    W0 = read_hierarchy(main).levels[0].W  # n x nvec, column r is w_r
    for r in range(1, len(paths) + 1):
        C = oracle.Composite([oracle.Oracle(p) for p in paths[:r]])
        w, rho = C.test(x0[r - 1], nu=15)
        assert abs(rho - st["rho"][r - 1]) <= 1e-9 * rho, (r, rho, st["rho"][r - 1])
        assert np.abs(w - W0[:, r]).max() <= 1e-8 * np.abs(W0[:, r]).max(), r


@pytest.mark.parametrize("kcyc", [False, True])
def test_composite_pcg_is_flexible_cg(boot, kcyc):
    P, x0, st, main, paths = boot
    Os = [oracle.Oracle(p) for p in paths]
    C = oracle.Composite(Os, kcycle=kcyc)
    A = dense(P.rowptr, P.col, P.val)
    x, hist, nit, status = C.pcg(P.b, tol=1e-10, maxit=100)
    xd, hd, nitd, std, _, _, _ = flexible_pcg(lambda v: A @ v, C.apply, P.b, 1e-10, 100, 0)
    assert status == 0 and std == 0 and nit == nitd
    assert np.all(np.abs(hist - hd) <= 1e-8 * hd)
    assert np.abs(x - np.linalg.solve(A, P.b)).max() <= 1e-8 * np.abs(x).max()


def test_testing_phase_with_kcycles_reproduces_the_setup(setup_lib, tmp_path):
    """With boot_kcycle the setup tests its composite with K-cycle components
    (two inner flexible-CG iterations per level, as Section 5 describes for the
    original bootstrap); the oracle's composite of the same stage files with
    K-cycle components, from the same random starts, gets the setup's
    estimates and smooth vectors.  The 24 x 24 problem gives stage
    hierarchies of four levels, so the inner iterations run on two levels."""
    P = problems.aniso9(24, 1e-2, np.pi / 4, seed=6)
    x0 = problems.random_vectors(P.n, NVEC - 1, 1000)
    st = build_hierarchy(P.rowptr, P.col, P.val, str(tmp_path / "main.bin"), x0,
                         SetupParams(nvec_max=NVEC, boot_coarse_min=6, rho_des=0.0, boot_kcycle=1),
                         boot_prefix=str(tmp_path / "boot"))
    paths = [str(tmp_path / f"boot_b{r}.bin") for r in range(1, len(st["rho"]) + 1)]
    assert len(paths) == NVEC - 1
    assert min(len(read_hierarchy(p).levels) for p in paths) >= 4
    W0 = read_hierarchy(str(tmp_path / "main.bin")).levels[0].W
    for r in range(1, len(paths) + 1):
        C = oracle.Composite([oracle.Oracle(p) for p in paths[:r]], kcycle=True)
        w, rho = C.test(x0[r - 1], nu=15)
        assert abs(rho - st["rho"][r - 1]) <= 1e-9 * rho, (r, rho, st["rho"][r - 1])
        assert np.abs(w - W0[:, r]).max() <= 1e-8 * np.abs(W0[:, r]).max(), r
    # and the V-cycle testing phase gives other estimates on the same problem
    C = oracle.Composite([oracle.Oracle(paths[0])], kcycle=False)
    assert abs(C.test(x0[0], nu=15)[1] - st["rho"][0]) > 1e-6 * st["rho"][0]
