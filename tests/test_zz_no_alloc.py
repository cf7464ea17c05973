"""The cycle entry point that allocates nothing (mvamg_cycle_apply_noalloc),
through the C ABI, against mvamg_cycle_apply on the same handle and input.

Both run the same kernels in the same order on the same data; only the
addresses of the work vectors differ, so the results must agree bit for bit.
Calls come in decreasing size on one shared static work array, so each later
call runs on what the previous one left there: a kernel that relied on
zeroed work memory would show up as a difference.
"""
import sys

import numpy as np
import pytest

from paper_1907_04417_amd import mvamg, workloads

pytestmark = pytest.mark.gpu

# decreasing fine sizes: 270,400 -> 5,184 -> 4,096 rows; aniso520 has
# sliced-ELL levels with 16- and 32-bit columns, elast12 a grouped fine level
SEQUENCE = ["aniso520", "elast12", "aniso64"]


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _pair(torch, S, r, precision, smoother):
    z_ref = torch.empty_like(r)
    z_na = torch.full_like(r, float("nan"))
    mvamg.cycle_apply(S.h, r, z_ref, precision, smoother)
    mvamg.cycle_apply_noalloc(S.h, r, z_na, precision, smoother)
    torch.cuda.synchronize()
    return z_ref.cpu().numpy(), z_na.cpu().numpy()


def test_noalloc_cycle_matches_cycle_apply(torch_gpu):
    torch = torch_gpu
    for name in SEQUENCE:
        P, path, st = workloads.load(name)
        S = mvamg.Solver(path)
        try:
            rng = np.random.default_rng(11)
            for precision in (64, 32):
                for smoother in (mvamg.SMOOTH_GS, mvamg.SMOOTH_L1JACOBI):
                    # two calls in a row on this handle, then the next (smaller) problem
                    for rep in range(2):
                        r = torch.from_numpy(rng.uniform(-1.0, 1.0, P.n)).cuda()
                        _say(f"[noalloc] {name} n={P.n} precision={precision} smoother={smoother} call={rep}")
                        a, b = _pair(torch, S, r, precision, smoother)
                        assert np.all(np.isfinite(a))
                        assert np.array_equal(a, b), (name, precision, smoother, float(np.abs(a - b).max()))
        finally:
            S.close()


def test_noalloc_cycle_rejects_too_large(torch_gpu):
    torch = torch_gpu
    P, path, st = workloads.load("jump128")
    S = mvamg.Solver(path)
    try:
        r = torch.ones(P.n, dtype=torch.float64, device="cuda")
        z = torch.zeros_like(r)
        _say(f"[noalloc] jump128 n={P.n}: above the static array, expect a rejection")
        with pytest.raises(mvamg.MvamgError) as ei:
            mvamg.cycle_apply_noalloc(S.h, r, z, 64, mvamg.SMOOTH_GS)
        assert ei.value.status == mvamg.ERR_ARG and "static scratch" in str(ei.value)
        # the handle still works afterwards
        mvamg.cycle_apply(S.h, r, z, 64, mvamg.SMOOTH_GS)
        torch.cuda.synchronize()
        assert torch.isfinite(z).all()
    finally:
        S.close()
