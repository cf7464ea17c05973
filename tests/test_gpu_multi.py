"""GPU parity of the multi-system paths against the CPU oracle.

Block right-hand sides: the method applied to each column is the
single-system method, so column c of every block result is compared with the
oracle's single-system result for that column (same tolerances as the
single-system parity tests: products 1e-13, binary64 cycle 1e-11, CG history
1e-10, solution 1e-9 relative; binary32 cycle element by element within
8 x the oracle's own binary32-versus-binary64 distance).

Batch of problems: the block-diagonal hierarchy's cycle is each problem's own
cycle, and every problem runs its own CG, so problem p is compared with the
oracle on problem p's own hierarchy file.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_1907_04417_amd import mvamg, problems, workloads
from tests.parity_util import fp32_cycle_bound

pytestmark = pytest.mark.gpu

BLOCK_CASES = ["aniso64", "jump16", "elast12"]


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _t(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _relinf(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def _hist_parity(hg, ho, tol):
    m = min(len(hg), len(ho))
    if len(hg) != len(ho):
        assert abs(len(hg) - len(ho)) == 1 and abs(ho[m - 1] / tol - 1) < 1e-8
    rel = np.abs(hg[:m] - ho[:m]) / ho[:m]
    assert rel.max() <= 1e-10, rel.max()


@pytest.fixture(scope="module")
def blk(torch_gpu):
    out = {}
    for name in BLOCK_CASES:
        P, path, st = workloads.load(name)
        _say(f"[block case] {name}: n={P.n} levels={st['n']}")
        out[name] = (P, path, mvamg.Solver(path, nrhs=32), oracle.Oracle(path))
    return out


# ------------------------------------------------------------ block columns

@pytest.mark.parametrize("m", [32, 7])
@pytest.mark.parametrize("name", BLOCK_CASES)
def test_spmv_block(name, m, blk, torch_gpu):
    P, path, S, O = blk[name]
    _say(f"[spmv_block] {name} m={m}")
    X = np.random.default_rng(11).standard_normal((P.n, m))
    Y = torch_gpu.empty((P.n, m), dtype=torch_gpu.float64, device="cuda")
    mvamg.spmv_block(S.h, _t(torch_gpu, X), Y)
    Y = Y.cpu().numpy()
    for c in range(m):
        assert _relinf(Y[:, c], oracle.spmv(P.rowptr, P.col, P.val, X[:, c])) <= 1e-13, c


@pytest.mark.parametrize("smoother", [mvamg.SMOOTH_GS, mvamg.SMOOTH_L1JACOBI])
@pytest.mark.parametrize("name", BLOCK_CASES)
def test_cycle_block(name, smoother, blk, torch_gpu):
    P, path, S, O = blk[name]
    _say(f"[cycle_block] {name} smoother={smoother}")
    Oc = O if smoother == mvamg.SMOOTH_GS else oracle.Oracle(path, smoother=oracle.L1_JACOBI)
    R = np.random.default_rng(12).standard_normal((P.n, 32))
    Z = torch_gpu.empty((P.n, 32), dtype=torch_gpu.float64, device="cuda")
    mvamg.cycle_apply_block(S.h, _t(torch_gpu, R), Z, smoother=smoother)
    Z = Z.cpu().numpy()
    for c in range(32):
        assert _relinf(Z[:, c], Oc.vcycle(R[:, c])) <= 1e-11, c


@pytest.mark.parametrize("name", BLOCK_CASES)
def test_cycle_block_fp32(name, blk, torch_gpu):
    P, path, S, O = blk[name]
    _say(f"[cycle_block32] {name}")
    R = np.random.default_rng(13).standard_normal((P.n, 32))
    Z = torch_gpu.empty((P.n, 32), dtype=torch_gpu.float64, device="cuda")
    mvamg.cycle_apply_block(S.h, _t(torch_gpu, R), Z, precision=32)
    Z = Z.cpu().numpy()
    for c in range(0, 32, 3):
        z32, z64, bound = fp32_cycle_bound(O, R[:, c])
        assert _relinf(Z[:, c], z32) <= bound and _relinf(Z[:, c], z64) <= bound, c


@pytest.mark.parametrize("m", [32, 5])
@pytest.mark.parametrize("name", BLOCK_CASES)
def test_pcg_block_fp64(name, m, blk, torch_gpu):
    P, path, S, O = blk[name]
    _say(f"[pcg_block64] {name} m={m}")
    B, _ = problems.block_rhs(P, m, seed=21)
    X = torch_gpu.zeros((P.n, m), dtype=torch_gpu.float64, device="cuda")
    H = np.zeros((m, 1001))
    infos = mvamg.pcg_solve_block(S.h, _t(torch_gpu, B), X, rtol=1e-8, history=H)
    X = X.cpu().numpy()
    for c in range(m):
        xo, ho, nito, sto = O.pcg(B[:, c], tol=1e-8)
        inf = infos[c]
        assert inf.converged and sto == 0, c
        _hist_parity(H[c, :inf.iterations + 1], ho, 1e-8)
        assert _relinf(X[:, c], xo) <= 1e-9, c
        assert inf.rel_res_true <= 1.01e-8, c


@pytest.mark.parametrize("name", BLOCK_CASES)
def test_pcg_block_mixed(name, blk, torch_gpu):
    """Binary32 cycle per column: every column meets the tolerance on the true
    residual, iteration counts close to the oracle's mixed run."""
    P, path, S, O = blk[name]
    _say(f"[pcg_block32] {name}")
    B, _ = problems.block_rhs(P, 32, seed=22)
    X = torch_gpu.zeros((P.n, 32), dtype=torch_gpu.float64, device="cuda")
    infos = mvamg.pcg_solve_block(S.h, _t(torch_gpu, B), X, rtol=1e-8, precision=32)
    X = X.cpu().numpy()
    for c in range(0, 32, 4):
        xo, ho, nito, sto, tro = O.pcg_mixed(B[:, c], tol=1e-8)
        x64, _, _, _ = O.pcg(B[:, c], tol=1e-8)
        inf = infos[c]
        assert inf.converged and inf.rel_res_true <= 1e-8, c
        assert abs(inf.iterations - nito) <= max(3, nito // 10), (c, inf.iterations, nito)
        assert _relinf(X[:, c], x64) <= 1e-5, c


def test_block_edge_cases(blk, torch_gpu):
    """m = 1; a zero column (stops at iteration 0 with x = 0) beside live
    ones; an iteration cap reached by every column; columns that start from
    a nonzero guess; block calls rejected on a batch handle and for m > 32."""
    torch = torch_gpu
    P, path, S, O = blk["jump16"]
    _say("[block edge] jump16")
    B, _ = problems.block_rhs(P, 4, seed=23)
    B[:, 2] = 0.0
    X0 = np.random.default_rng(24).standard_normal((P.n, 4)) * 0.1
    X0[:, 2] = 0.0
    X = _t(torch, X0)
    infos = mvamg.pcg_solve_block(S.h, _t(torch, B), X, rtol=1e-8)
    X = X.cpu().numpy()
    assert infos[2].iterations == 0 and infos[2].converged and np.all(X[:, 2] == 0.0)
    for c in (0, 1, 3):
        xo, ho, nito, _ = O.pcg(B[:, c], x0=X0[:, c], tol=1e-8)
        assert infos[c].converged and infos[c].iterations == nito, c
        assert _relinf(X[:, c], xo) <= 1e-9, c
    # one column (same start): each column's arithmetic does not depend on the others
    x1 = _t(torch, X0[:, :1])
    inf1 = mvamg.pcg_solve_block(S.h, _t(torch, B[:, :1]), x1, rtol=1e-8)
    assert inf1[0].iterations == infos[0].iterations
    assert _relinf(x1.cpu().numpy()[:, 0], X[:, 0]) <= 1e-12
    # cap
    Xc = torch.zeros((P.n, 4), dtype=torch.float64, device="cuda")
    infc = mvamg.pcg_solve_block(S.h, _t(torch, B), Xc, rtol=1e-12, maxit=3)
    assert [i.iterations for i in infc] == [3, 3, 0, 3]
    assert not infc[0].converged and infc[2].converged
    # width limits (checked by the library as well as the binding)
    lib = mvamg.load()
    st = lib.mvamg_pcg_solve_block(S.h, _t(torch, B).data_ptr(), Xc.data_ptr(), 33, None, None, None)
    assert st == mvamg.ERR_ARG


def test_block_full_size_aniso1024(torch_gpu):
    """C4b: 32 right-hand sides on the 1024^2 anisotropic problem.  Two
    columns against the oracle (history and solution); every column converged
    with the true residual within the tolerance."""
    torch = torch_gpu
    P, path, st = workloads.load("aniso1024")
    _say(f"[block full] aniso1024 levels={st['n']}")
    S = mvamg.Solver(path, nrhs=32)
    B, _ = problems.block_rhs(P, 32, seed=workloads.BLOCK_RHS_SEED)
    X = torch.zeros((P.n, 32), dtype=torch.float64, device="cuda")
    H = np.zeros((32, 1001))
    infos = mvamg.pcg_solve_block(S.h, _t(torch, B), X, rtol=1e-8, history=H)
    X = X.cpu().numpy()
    its = [i.iterations for i in infos]
    _say(f"  iterations {min(its)}..{max(its)}")
    for inf in infos:
        assert inf.converged and inf.rel_res_true <= 1.01e-8
    O = oracle.Oracle(path)
    for c in (0, 17):
        _say(f"  oracle column {c}")
        xo, ho, nito, sto = O.pcg(B[:, c], tol=1e-8)
        _hist_parity(H[c, :infos[c].iterations + 1], ho, 1e-8)
        assert _relinf(X[:, c], xo) <= 1e-9
    S.close()


# ------------------------------------------------------------ batch problems

@pytest.fixture(scope="module")
def batch6(torch_gpu):
    Ps, paths, stats = workloads.load_batch("batch6")
    _say(f"[batch case] batch6: {[s['n'] for s in stats]}")
    BS = mvamg.BatchSolver(paths)
    Os = [oracle.Oracle(p) for p in paths]
    return Ps, paths, BS, Os


def _split(v, offsets):
    return [v[offsets[p]:offsets[p + 1]] for p in range(len(offsets) - 1)]


def test_batch_layout(batch6):
    Ps, paths, BS, Os = batch6
    assert BS.nprob == len(Ps)
    assert BS.offsets == list(np.cumsum([0] + [P.n for P in Ps]))


def test_batch_spmv(batch6, torch_gpu):
    Ps, paths, BS, Os = batch6
    _say("[batch spmv]")
    x = np.random.default_rng(31).standard_normal(BS.offsets[-1])
    y = torch_gpu.empty(BS.offsets[-1], dtype=torch_gpu.float64, device="cuda")
    mvamg.spmv(BS.h, _t(torch_gpu, x), y)
    for P, xs, ys in zip(Ps, _split(x, BS.offsets), _split(y.cpu().numpy(), BS.offsets)):
        assert _relinf(ys, oracle.spmv(P.rowptr, P.col, P.val, xs)) <= 1e-13


@pytest.mark.parametrize("smoother", [mvamg.SMOOTH_GS, mvamg.SMOOTH_L1JACOBI])
def test_batch_cycle(batch6, smoother, torch_gpu):
    Ps, paths, BS, Os = batch6
    _say(f"[batch cycle] smoother={smoother}")
    r = np.random.default_rng(32).standard_normal(BS.offsets[-1])
    z = torch_gpu.empty(BS.offsets[-1], dtype=torch_gpu.float64, device="cuda")
    mvamg.cycle_apply(BS.h, _t(torch_gpu, r), z, smoother=smoother)
    for p, (rs, zs) in enumerate(zip(_split(r, BS.offsets), _split(z.cpu().numpy(), BS.offsets))):
        Oc = Os[p] if smoother == mvamg.SMOOTH_GS else oracle.Oracle(paths[p], smoother=oracle.L1_JACOBI)
        assert _relinf(zs, Oc.vcycle(rs)) <= 1e-11, p


def test_batch_pcg_fp64(batch6, torch_gpu):
    Ps, paths, BS, Os = batch6
    _say("[batch pcg64]")
    b = np.concatenate([P.b for P in Ps])
    x = torch_gpu.zeros(BS.offsets[-1], dtype=torch_gpu.float64, device="cuda")
    H = np.zeros((BS.nprob, 1001))
    infos = mvamg.batch_pcg_solve(BS.h, _t(torch_gpu, b), x, rtol=1e-8, history=H)
    for p, (P, xs) in enumerate(zip(Ps, _split(x.cpu().numpy(), BS.offsets))):
        xo, ho, nito, sto = Os[p].pcg(P.b, tol=1e-8)
        assert infos[p].converged and sto == 0, p
        _hist_parity(H[p, :infos[p].iterations + 1], ho, 1e-8)
        assert _relinf(xs, xo) <= 1e-9, p
        assert infos[p].rel_res_true <= 1.01e-8, p


def test_batch_pcg_mixed(batch6, torch_gpu):
    Ps, paths, BS, Os = batch6
    _say("[batch pcg32]")
    b = np.concatenate([P.b for P in Ps])
    x = torch_gpu.zeros(BS.offsets[-1], dtype=torch_gpu.float64, device="cuda")
    infos = mvamg.batch_pcg_solve(BS.h, _t(torch_gpu, b), x, rtol=1e-8, precision=32)
    for p, (P, xs) in enumerate(zip(Ps, _split(x.cpu().numpy(), BS.offsets))):
        xo, ho, nito, sto, tro = Os[p].pcg_mixed(P.b, tol=1e-8)
        x64, _, _, _ = Os[p].pcg(P.b, tol=1e-8)
        assert infos[p].converged and infos[p].rel_res_true <= 1e-8, p
        assert abs(infos[p].iterations - nito) <= max(3, nito // 10), (p, infos[p].iterations, nito)
        assert _relinf(xs, x64) <= 1e-5, p


def test_batch_handle_rules(batch6, torch_gpu):
    Ps, paths, BS, Os = batch6
    torch = torch_gpu
    b = torch.zeros(BS.offsets[-1], dtype=torch.float64, device="cuda")
    with pytest.raises(mvamg.MvamgError) as e:
        mvamg.pcg_solve(BS.h, b, torch.zeros_like(b))
    assert e.value.status == mvamg.ERR_ARG
    with pytest.raises(mvamg.MvamgError) as e:
        mvamg.spmv_block(BS.h, b.reshape(-1, 1), torch.zeros_like(b).reshape(-1, 1))
    assert e.value.status == mvamg.ERR_ARG
    # zero right-hand side: every problem stops at iteration 0
    infos = mvamg.batch_pcg_solve(BS.h, b, torch.zeros_like(b))
    assert all(i.iterations == 0 and i.converged for i in infos)


def test_batch64_full_size(torch_gpu):
    """C4a: 64 uneven problems in one batch.  Smallest, median and largest
    problem against the oracle; every problem converged with its true
    residual within the tolerance."""
    torch = torch_gpu
    Ps, paths, stats = workloads.load_batch("batch64")
    _say(f"[batch64] rows={sum(P.n for P in Ps)}")
    BS = mvamg.BatchSolver(paths)
    b = np.concatenate([P.b for P in Ps])
    x = torch.zeros(BS.offsets[-1], dtype=torch.float64, device="cuda")
    H = np.zeros((BS.nprob, 1001))
    infos = mvamg.batch_pcg_solve(BS.h, _t(torch, b), x, rtol=1e-8, history=H)
    xs = _split(x.cpu().numpy(), BS.offsets)
    its = [i.iterations for i in infos]
    _say(f"  iterations {min(its)}..{max(its)}")
    for inf in infos:
        assert inf.converged and inf.rel_res_true <= 1.01e-8
    order = np.argsort([P.n for P in Ps])
    for p in (order[0], order[len(order) // 2], order[-1]):
        _say(f"  oracle problem {p} n={Ps[p].n}")
        xo, ho, nito, sto = oracle.Oracle(paths[p]).pcg(Ps[p].b, tol=1e-8)
        _hist_parity(H[p, :infos[p].iterations + 1], ho, 1e-8)
        assert _relinf(xs[p], xo) <= 1e-9
    BS.close()
