"""GPU K-cycle (two inner flexible-CG iterations on every level but the
finest and the coarsest, Section 5) through the C ABI against the oracle's
K-cycle on the same hierarchy files.

Tolerances as for the V-cycle: one cycle 1e-11 relative (the inner
coefficients are ratios of inner products summed in another order), the CG
history 1e-10 relative and the solution 1e-9 relative with the same
iteration count.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_1907_04417_amd import mvamg, problems, workloads
from tests.conftest import make_hierarchy

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
def kcases(torch_gpu, setup_lib, tmp_path_factory):
    out = {}
    for name in ["jump16", "jump32", "elast12", "aniso520"]:
        P, path, st = workloads.load(name)
        out[name] = (P, path, st)
    # five levels: inner iterations on levels 1, 2 and 3, each nested in the one above
    P = problems.aniso9(96, 1e-2, np.pi / 4, seed=2)
    path, st = make_hierarchy(tmp_path_factory.mktemp("k5"), P, 3, boot_coarse_min=8, coarse_cap=300, compose=1)
    assert st["nlevels"] >= 5
    out["aniso96_deep"] = (P, path, st)
    for name, (P, path, st) in out.items():
        _say(f"[kcycle case] {name}: levels {st['n']}")
    return out


def _t(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _relinf(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.mark.parametrize("name", ["jump16", "jump32", "elast12", "aniso520", "aniso96_deep"])
@pytest.mark.parametrize("smoother", [mvamg.SMOOTH_GS, mvamg.SMOOTH_L1JACOBI])
def test_kcycle_parity(name, smoother, kcases, torch_gpu):
    torch = torch_gpu
    P, path, st = kcases[name]
    S = mvamg.Solver(path)
    O = oracle.Oracle(path, smoother=oracle.GS_COLOUR if smoother == mvamg.SMOOTH_GS else oracle.L1_JACOBI)
    try:
        rng = np.random.default_rng(21)
        for rep in range(2):
            r = rng.standard_normal(P.n)
            z = torch.empty(P.n, dtype=torch.float64, device="cuda")
            _say(f"[kcycle] {name} smoother={smoother} rep={rep}")
            mvamg.kcycle_apply(S.h, _t(torch, r), z, smoother)
            zk = O.kcycle(r)
            err = _relinf(z.cpu().numpy(), zk)
            _say(f"  rel err {err:.2e}")
            assert err <= 1e-11
        if st["nlevels"] == 2:
            assert np.array_equal(z.cpu().numpy(), S.cycle(_t(torch, r), smoother=smoother).cpu().numpy())
    finally:
        S.close()


@pytest.mark.parametrize("name", ["jump16", "elast12", "aniso520", "aniso96_deep"])
def test_kcycle_pcg_parity(name, kcases, torch_gpu):
    torch = torch_gpu
    P, path, st = kcases[name]
    S = mvamg.Solver(path)
    O = oracle.Oracle(path)
    try:
        _say(f"[kcycle pcg] {name}")
        x, res = S.solve(_t(torch, P.b), rtol=1e-8, cycle=mvamg.CYCLE_K)
        xo, ho, nito, sto = O.pcg_kcycle(P.b, tol=1e-8)
        _, _, nitv, _ = O.pcg(P.b, tol=1e-8)
        _say(f"  gpu it {res.iterations}, oracle K it {nito}, oracle V it {nitv}")
        assert sto == 0 and res.converged and res.iterations == nito
        assert np.all(np.abs(res.history - ho) <= 1e-10 * ho)
        assert _relinf(x.cpu().numpy(), xo) <= 1e-9
        assert res.rel_res_true <= 1.01e-8
    finally:
        S.close()


def test_kcycle_argument_errors(kcases, torch_gpu):
    torch = torch_gpu
    P, path, st = kcases["jump16"]
    S = mvamg.Solver(path)
    try:
        b = _t(torch, P.b)
        with pytest.raises(mvamg.MvamgError) as ei:
            S.solve(b, precision=32, cycle=mvamg.CYCLE_K)
        assert ei.value.status == mvamg.ERR_ARG and "binary64" in str(ei.value)
        with pytest.raises(mvamg.MvamgError) as ei:
            S.solve(b, cycle=7)
        assert ei.value.status == mvamg.ERR_ARG
    finally:
        S.close()
