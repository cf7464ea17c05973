"""Differentiable solve on the GPU: gradients of L = ||x(g) - x_obs||^2 with
respect to g (through A(g), kappa = exp(g)) and b, via the adjoint AMG-PCG."""
import sys

import numpy as np
import pytest

from paper_1907_04417_amd import mvamg, problems, workloads
from paper_1907_04417_amd.autograd import amg_solve

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


def _observed(torch, S, fv, g, b, seed):
    with torch.no_grad():
        x = amg_solve(fv.values_torch(g), b, S, rtol=1e-12)
    rng = np.random.default_rng(seed + 1)
    rms = float(torch.sqrt((x * x).mean()))
    return x + torch.from_numpy(rng.normal(0.0, 0.01 * rms, x.shape[0])).to(x)


def test_gradient_matches_dense_float64(torch_gpu):
    """32 x 32 cells: the adjoint gradient equals the gradient of the same loss
    through a dense binary64 solve (torch on the CPU) to 1e-9."""
    torch = torch_gpu
    P, path, st = workloads.load("grf32")
    _say(f"[grad dense] grf32 levels={st['n']}")
    fv, g0 = P.meta["fv"], P.meta["g"].ravel()
    S = mvamg.Solver(path)
    b = torch.from_numpy(P.b).cuda()
    g = torch.from_numpy(g0.copy()).cuda().requires_grad_(True)
    bb = b.clone().requires_grad_(True)
    xobs = _observed(torch, S, fv, g.detach(), b, 3)
    x = amg_solve(fv.values_torch(g), bb, S, rtol=1e-13)
    L = ((x - xobs) ** 2).sum()
    L.backward()
    # dense reference
    gc = torch.from_numpy(g0.copy()).requires_grad_(True)
    bc = torch.from_numpy(P.b.copy()).requires_grad_(True)
    vc = fv.values_torch(gc)
    A = torch.zeros(P.n, P.n, dtype=torch.float64)
    rows = torch.from_numpy(np.repeat(np.arange(P.n), np.diff(fv.rowptr)))
    A = A.index_put((rows, torch.from_numpy(fv.col.astype(np.int64))), vc)
    xc = torch.linalg.solve(A, bc)
    Lc = ((xc - xobs.cpu()) ** 2).sum()
    Lc.backward()
    eg = (g.grad.cpu() - gc.grad).abs().max() / gc.grad.abs().max()
    eb = (bb.grad.cpu() - bc.grad).abs().max() / bc.grad.abs().max()
    _say(f"  dL/dg rel err {eg:.2e}, dL/db rel err {eb:.2e}")
    assert eg <= 1e-9 and eb <= 1e-9
    S.close()


def test_gradient_matches_central_differences_1024(torch_gpu):
    """1024^2 cells: dL/dg from the adjoint solve against central differences
    on 100 random cells, with steps h = 1e-6 and 1e-4 on the log-coefficient g.
    Each perturbed solve starts from x(g), so its tolerance (1e-11, relative to
    the initial residual) bounds the error of the small correction
    x(g +- h e_c) - x(g) itself; the difference of the losses is
    sum (x+ - x-)(x+ + x- - 2 x_obs), with no cancellation of L.

    Bound: 1e-4 |g_c| + 1e-6 max|g| + tau / h.  tau = 2e-16 covers the
    binary64 rounding floor of that loss difference, measured at up to
    6e-17 and independent of the solve tolerances between 1e-11 and 1e-14;
    at h = 1e-6 it is the dominant term.  The O(h^2) truncation error of
    central differences is below 1e-8 relative at h = 1e-4."""
    import time
    torch = torch_gpu
    t = time.time()
    P, path, st = workloads.load("grf1024")
    _say(f"[grad fd] grf1024 levels={st['n']} setup {time.time() - t:.1f}s")
    fv, g0 = P.meta["fv"], P.meta["g"].ravel()
    S = mvamg.Solver(path)
    b = torch.from_numpy(P.b).cuda()
    g = torch.from_numpy(g0.copy()).cuda().requires_grad_(True)
    xobs = _observed(torch, S, fv, g.detach(), b, 0)
    t = time.time()
    x = amg_solve(fv.values_torch(g), b, S, rtol=1e-13)
    ((x - xobs) ** 2).sum().backward()
    grad = g.grad.detach()
    x0 = x.detach()
    _say(f"  adjoint gradient {time.time() - t:.2f}s, max |g| {grad.abs().max().item():.3e}")
    cells = np.random.default_rng(7).choice(P.n, 100, replace=False)
    gmax = grad.abs().max().item()
    tau = 2e-16

    def perturbed(gv):
        mvamg.set_fine_values(S.h, fv.values_torch(gv))
        xs = x0.clone()
        inf = mvamg.pcg_solve(S.h, b, xs, rtol=1e-11)
        assert inf.converged
        return xs

    with torch.no_grad():
        for h in (1e-6, 1e-4):
            worst = 0.0
            for c in cells:
                gp = g.detach().clone()
                gm = g.detach().clone()
                gp[c] += h
                gm[c] -= h
                xp, xm = perturbed(gp), perturbed(gm)
                dL = ((xp - xm) * (xp + xm - 2 * xobs)).sum().item()
                fd = dL / (2 * h)
                ga = grad[c].item()
                bound = 1e-4 * abs(ga) + 1e-6 * gmax + tau / h
                worst = max(worst, abs(fd - ga) / bound)
                assert abs(fd - ga) <= bound, (h, c, fd, ga)
            _say(f"  h={h:.0e}, 100 cells: worst |fd - adj| / bound = {worst:.3f}")
    S.close()
