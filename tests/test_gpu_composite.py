"""The bootstrap's composite AMG on the GPU (eq. 1.1, Algorithm 1, Section 5
item (i): the symmetrized multiplicative product of the stage hierarchies
B_1..B_r) against the oracle's composite on the same hierarchy files: one
application 1e-11 relative, the testing phase's estimate 1e-10 and smooth
vector 1e-9, CG history 1e-10 with the same iteration count and solution
1e-9; with V-cycle and K-cycle components.  The GPU testing phase also
reproduces the host setup's own estimate and smooth vector from the same
random start."""
import sys

import numpy as np
import pytest

import oracle
from oracle.hierfile import read_hierarchy
from paper_1907_04417_amd import mvamg, problems, workloads

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


@pytest.fixture(scope="module")
def boot(torch_gpu):
    P, main, st, paths, x0 = workloads.load_bootstrap("ani2_160")
    _say(f"[composite] ani2_160: {len(paths)} bootstrap hierarchies, rho {st['rho']}")
    Ss = [mvamg.Solver(p) for p in paths]
    Os = [oracle.Oracle(p) for p in paths]
    yield P, main, st, paths, x0, Ss, Os
    for S in Ss:
        S.close()


def _t(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _relinf(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.mark.parametrize("cycle", [mvamg.CYCLE_V, mvamg.CYCLE_K])
def test_composite_apply_parity(boot, torch_gpu, cycle):
    torch = torch_gpu
    P, main, st, paths, x0, Ss, Os = boot
    C = mvamg.Composite(Ss)
    r = np.random.default_rng(9).standard_normal(P.n)
    for k in (1, len(Ss)):
        _say(f"[composite apply] r={k} cycle={cycle}")
        z = C.apply(_t(torch, r), cycle=cycle, r=k).cpu().numpy()
        zo = oracle.Composite(Os[:k], kcycle=cycle == mvamg.CYCLE_K).apply(r)
        assert _relinf(z, zo) <= 1e-11


def test_testing_phase_parity(boot, torch_gpu):
    torch = torch_gpu
    P, main, st, paths, x0, Ss, Os = boot
    C = mvamg.Composite(Ss)
    W0 = read_hierarchy(main).levels[0].W
    for r in range(1, len(Ss) + 1):
        x = _t(torch, x0[r - 1])
        rho = C.test(x, nu=15, r=r)
        w, rho_o = oracle.Composite(Os[:r]).test(x0[r - 1], nu=15)
        _say(f"[composite test] r={r}: rho gpu {rho:.12f} oracle {rho_o:.12f} setup {st['rho'][r - 1]:.12f}")
        xg = x.cpu().numpy()
        assert abs(rho - rho_o) <= 1e-10 * rho_o and _relinf(xg, w) <= 1e-9
        assert abs(rho - st["rho"][r - 1]) <= 1e-9 * rho and _relinf(xg, W0[:, r]) <= 1e-8


@pytest.mark.parametrize("cycle", [mvamg.CYCLE_V, mvamg.CYCLE_K])
def test_composite_pcg_parity(boot, torch_gpu, cycle):
    torch = torch_gpu
    P, main, st, paths, x0, Ss, Os = boot
    C = mvamg.Composite(Ss)
    x, res = C.solve(_t(torch, P.b), rtol=1e-6, cycle=cycle)
    xo, ho, nito, sto = oracle.Composite(Os, kcycle=cycle == mvamg.CYCLE_K).pcg(P.b, tol=1e-6)
    _say(f"[composite pcg] cycle={cycle}: gpu it {res.iterations}, oracle it {nito}")
    assert sto == 0 and res.converged and res.iterations == nito
    assert np.all(np.abs(res.history - ho) <= 1e-10 * ho)
    assert _relinf(x.cpu().numpy(), xo) <= 1e-9


def test_composite_rejects_other_matrices(boot, torch_gpu):
    torch = torch_gpu
    P, main, st, paths, x0, Ss, Os = boot
    Q, qpath, qst = workloads.load("ani1_160")
    S2 = mvamg.Solver(qpath)
    try:
        with pytest.raises(mvamg.MvamgError) as ei:
            mvamg.Composite([Ss[0], S2]).apply(_t(torch, P.b))
        assert ei.value.status == mvamg.ERR_ARG and "same fine matrix" in str(ei.value)
    finally:
        S2.close()
