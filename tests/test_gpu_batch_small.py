"""Batches with problems on the one-launch small-problem path (one workgroup
runs a problem's whole CG and V-cycle over its own hierarchy) through the C
ABI, against the oracle problem by problem: history 1e-10 relative (1e-8
from the tolerance, as the other batch tests), solution 1e-9 relative, the
same iteration count.  The batch mixes sizes and level counts: problems
below the threshold and problems whose depth differs from the others' take
the small path, the rest the lockstep path, all in one call."""
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
def uneven(torch_gpu, setup_lib, tmp_path_factory):
    """batch6 (3 levels each, sides 32..64) plus problems with their own setups:
    a 2-level and a 4-level one, and two larger 3-level ones."""
    Ps, paths, stats = workloads.load_batch("batch6")
    Ps, paths = list(Ps), list(paths)
    d = tmp_path_factory.mktemp("uneven")
    extra = [(problems.aniso9(48, 1e-3, 0.3, seed=21), dict(boot_coarse_min=8, coarse_cap=400, compose=3)),
             (problems.aniso9(80, 1e-1, 1.1, seed=22), dict(boot_coarse_min=4, coarse_cap=60, compose=1)),
             (problems.aniso9(150, 1e-2, 0.7, seed=23), workloads.BATCH_SETUP),
             (problems.aniso9(170, 1e-3, 2.0, seed=24), workloads.BATCH_SETUP)]
    for P, sp in extra:
        path, st = make_hierarchy(d, P, 3, **sp)
        Ps.append(P)
        paths.append(path)
    depths = [oracle.Oracle(p).h.nlevels for p in paths]
    _say(f"[uneven] sizes {[P.n for P in Ps]} levels {depths}")
    assert len(set(depths)) >= 3
    return Ps, paths, depths


def _split(v, off):
    return [v[off[p]:off[p + 1]] for p in range(len(off) - 1)]


def _check(torch, Ps, paths, BS, smoother=mvamg.SMOOTH_GS):
    b = np.concatenate([P.b for P in Ps])
    x = torch.zeros(BS.offsets[-1], dtype=torch.float64, device="cuda")
    H = np.zeros((BS.nprob, 1001))
    infos = mvamg.batch_pcg_solve(BS.h, torch.from_numpy(b).cuda(), x, rtol=1e-8, history=H, smoother=smoother)
    xs_all = _split(x.cpu().numpy(), BS.offsets)
    for p, P in enumerate(Ps):
        O = oracle.Oracle(paths[p], smoother=oracle.GS_COLOUR if smoother == mvamg.SMOOTH_GS else oracle.L1_JACOBI)
        xo, ho, nito, sto = O.pcg(P.b, tol=1e-8)
        inf = infos[p]
        assert sto == 0 and inf.converged, p
        assert inf.iterations == nito, (p, inf.iterations, nito)
        h = H[p, :inf.iterations + 1]
        assert np.all(np.abs(h - ho) <= 1e-10 * ho), p
        assert np.abs(xs_all[p] - xo).max() <= 1e-9 * np.abs(xo).max(), p
        assert inf.rel_res_true <= 1.01e-8, p
    return [i.iterations for i in infos]


def test_all_on_the_small_path(uneven, torch_gpu):
    Ps, paths, depths = uneven
    BS = mvamg.BatchSolver(paths, mini_rows=1 << 30)
    try:
        flags = mvamg.batch_small_path(BS.h)
        _say(f"[small path] all: flags {flags}")
        assert all(flags) and BS.nprob == len(Ps)
        assert BS.offsets == list(np.cumsum([0] + [P.n for P in Ps]))
        its = _check(torch_gpu, Ps, paths, BS)
        _say(f"  iterations {its}")
    finally:
        BS.close()


def test_mixed_paths(uneven, torch_gpu):
    Ps, paths, depths = uneven
    BS = mvamg.BatchSolver(paths, mini_rows=3000)
    try:
        flags = mvamg.batch_small_path(BS.h)
        _say(f"[small path] mixed: flags {flags}")
        assert any(flags) and not all(flags)
        # the lockstep part has one depth; every problem of another depth is on the small path
        big = [p for p in range(len(Ps)) if not flags[p]]
        assert len({depths[p] for p in big}) == 1
        assert all(Ps[p].n > 3000 for p in big)
        for smoother in (mvamg.SMOOTH_GS, mvamg.SMOOTH_L1JACOBI):
            its = _check(torch_gpu, Ps, paths, BS, smoother)
            _say(f"  smoother {smoother}: iterations {its}")
    finally:
        BS.close()


def test_small_path_arguments(uneven, torch_gpu):
    torch = torch_gpu
    Ps, paths, depths = uneven
    BS = mvamg.BatchSolver(paths, mini_rows=1 << 30)
    try:
        b = torch.from_numpy(np.concatenate([P.b for P in Ps])).cuda()
        x = torch.zeros_like(b)
        with pytest.raises(mvamg.MvamgError) as ei:
            mvamg.batch_pcg_solve(BS.h, b, x, precision=32)
        assert ei.value.status == mvamg.ERR_ARG and "binary64" in str(ei.value)
        with pytest.raises(mvamg.MvamgError):
            mvamg.cycle_apply(BS.h, b, x)
        # not converged within maxit: reported per problem, x holds the last iterate
        infos = mvamg.batch_pcg_solve(BS.h, b, x, rtol=1e-8, maxit=3)
        assert all(i.iterations == 3 and not i.converged for i in infos)
    finally:
        BS.close()
