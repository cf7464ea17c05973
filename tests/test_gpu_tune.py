"""Autotuner: every kernel variant it may choose keeps oracle parity, choices
round-trip as text, and invalid choices are rejected."""
import sys

import numpy as np
import pytest

import oracle
from paper_1907_04417_amd import mvamg, workloads

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


def _t(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _relinf(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def _hist_parity(hg, ho, tol):
    m = min(len(hg), len(ho))
    if len(hg) != len(ho):
        assert abs(len(hg) - len(ho)) == 1 and abs(ho[m - 1] / tol - 1) < 1e-8
    assert (np.abs(hg[:m] - ho[:m]) / ho[:m]).max() <= 1e-10


def _grouped_levels(text):
    return {int(k[1:]): int(v) for k, v in (i.split("=") for i in text.split(";") if i) if k.startswith("G")}


@pytest.mark.parametrize("name", ["jump16", "elast12"])
def test_every_group_lane_variant_keeps_parity(name, torch_gpu):
    """Every grouped-level kernel the tuner may choose (64 / G lanes per row,
    or one block per group) keeps oracle parity."""
    P, path, st = workloads.load(name)
    S = mvamg.Solver(path)
    O = oracle.Oracle(path)
    levels = _grouped_levels(mvamg.tune_get(S.h))
    _say(f"[tune lanes] {name} grouped levels {levels}")
    assert levels
    r = np.random.default_rng(41).standard_normal(P.n)
    zo = O.vcycle(r)
    text0 = mvamg.tune_get(S.h)
    xo, ho, nito, _ = O.pcg(P.b, tol=1e-8)
    for l, g0 in levels.items():
        # wave per group with 64 / g lanes per row, then one block per group
        variants = [(g, 0) for g in (1, 2, 4, 8) if g >= g0] + [(g0, 1)]
        for g, w in variants:
            mvamg.tune_set(S.h, f"G{l}={g};W{l}={w}")
            z = S.cycle(_t(torch_gpu, r)).cpu().numpy()
            assert _relinf(z, zo) <= 1e-11, (l, g, w)
            x, res = S.solve(_t(torch_gpu, P.b), rtol=1e-8)
            _hist_parity(res.history, ho, 1e-8)
            assert _relinf(x.cpu().numpy(), xo) <= 1e-9, (l, g, w)
        mvamg.tune_set(S.h, text0)
    assert mvamg.tune_get(S.h) == text0
    S.close()


def test_every_block_coarse_variant_keeps_parity(torch_gpu):
    P, path, st = workloads.load("jump16")
    S = mvamg.Solver(path, nrhs=32)
    O = oracle.Oracle(path)
    R = np.random.default_rng(42).standard_normal((P.n, 32))
    zo = [O.vcycle(R[:, c]) for c in range(0, 32, 5)]
    Z = torch_gpu.empty((P.n, 32), dtype=torch_gpu.float64, device="cuda")
    for v in range(6):
        _say(f"[tune gemm] variant {v}")
        mvamg.tune_set(S.h, f"gemm={v}")
        mvamg.cycle_apply_block(S.h, _t(torch_gpu, R), Z)
        Zc = Z.cpu().numpy()
        for i, c in enumerate(range(0, 32, 5)):
            assert _relinf(Zc[:, c], zo[i]) <= 1e-11, (v, c)
    S.close()


def test_autotune_report_roundtrip_and_rejects(torch_gpu, tmp_path):
    P, path, st = workloads.load("jump16")
    S = mvamg.Solver(path, nrhs=32)
    rep = mvamg.autotune(S.h)
    _say(f"[tune] {rep}")
    assert "chosen:" in rep and "gemm" in rep
    text = mvamg.tune_get(S.h)
    mvamg.tune_set(S.h, text)
    assert mvamg.tune_get(S.h) == text
    sig = mvamg.signature(S.h)
    assert sig.startswith("arch=") and f"n={P.n}," in sig
    for bad in ["G0=8", "W0=1", "W1=2", "gemm=99", "foo=1", "G1=3", "G1=16", "chunks=4", "G1"]:
        with pytest.raises(mvamg.MvamgError) as e:
            mvamg.tune_set(S.h, bad)
        assert e.value.status == mvamg.ERR_ARG, bad
    assert mvamg.tune_get(S.h) == text  # nothing applied by a rejected text
    cache = str(tmp_path / "tune.json")
    t1 = mvamg.tuned(S.h, cache)
    t2 = mvamg.tuned(S.h, cache)  # from the cache
    assert t1 == t2 == mvamg.tune_get(S.h)
    S.close()


def test_batch_chunk_variants_keep_parity(torch_gpu):
    """Every reduction chunking the tuner may choose for a batch keeps every
    problem's CG history and solution at oracle parity."""
    Ps, paths, stats = workloads.load_batch("batch6")
    BS = mvamg.BatchSolver(paths)
    rep = mvamg.autotune(BS.h, mvamg.TUNE_BATCH_CHUNKS | mvamg.TUNE_GROUP_LANES)
    _say(f"[tune batch] {rep}")
    assert "chunks" in rep
    b = np.concatenate([P.b for P in Ps])
    ref = [oracle.Oracle(p).pcg(P.b, tol=1e-8) for p, P in zip(paths, Ps)]
    for c in (4, 16, 64):
        _say(f"[tune batch] chunks={c}")
        mvamg.tune_set(BS.h, f"chunks={c}")
        x = torch_gpu.zeros(BS.offsets[-1], dtype=torch_gpu.float64, device="cuda")
        H = np.zeros((BS.nprob, 1001))
        infos = mvamg.batch_pcg_solve(BS.h, _t(torch_gpu, b), x, rtol=1e-8, history=H)
        xs = x.cpu().numpy()
        for p in range(BS.nprob):
            xo, ho, nito, sto = ref[p]
            assert infos[p].converged and sto == 0, (c, p)
            _hist_parity(H[p, :infos[p].iterations + 1], ho, 1e-8)
            assert _relinf(xs[BS.offsets[p]:BS.offsets[p + 1]], xo) <= 1e-9, (c, p)
    BS.close()
