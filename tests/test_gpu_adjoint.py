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

    With x0 = x(g), the perturbed solutions are computed so that no two
    independently solved vectors are subtracted:
      x_- = x0 + d,  A(g - h e_c) d = b - A(g - h e_c) x0,
      D = x_+ - x_-, A(g + h e_c) D = (A(g - h e_c) - A(g + h e_c)) x_-,
    both from zero to rtol 1e-13.  The right-hand side of D is exactly zero
    away from cell c (both products are the same kernel on the same values
    there), so D carries its own relative accuracy.  Subtracting two
    separately solved x_+ and x_- instead leaves an absolute noise of about
    1e-17 on the loss difference, i.e. ~1e-3 of the smaller gradients at
    h = 1e-6 (measured: the error grows as 1/h and does not move with the
    solve tolerances, while the adjoint gradient agrees with itself to 10
    digits over tolerances 1e-12 .. 1e-15).
    L(x_+) - L(x_-) = sum D (D + 2 (x_- - x_obs)).  Even so the loss
    difference keeps an absolute noise of up to ~5e-16 (measured on the
    weakest cells; the same for solve tolerances 1e-13 .. 1e-16, while at
    h = 1e-4 the same cells agree with the adjoint to ~1e-5), i.e. up to
    ~2.5e-10 on the quotient at h = 1e-6.  Bound: 1e-4 |g_c| + 1e-6 max|g| +
    tau / (2 h) with tau = 2e-15 (4x that noise); at h = 1e-4 the tau term is
    5e-12.  The O(h^2) truncation error is below 1e-8 relative at h = 1e-4."""
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

    def matvec(gv, v):
        mvamg.set_fine_values(S.h, fv.values_torch(gv))
        y = torch.empty_like(b)
        mvamg.spmv(S.h, v, y)
        return y

    def solve(gv, rhs):
        mvamg.set_fine_values(S.h, fv.values_torch(gv))
        d = torch.zeros_like(b)
        inf = mvamg.pcg_solve(S.h, rhs, d, rtol=1e-13, maxit=2000)
        assert inf.converged
        return d

    with torch.no_grad():
        for h in (1e-6, 1e-4):
            worst = 0.0
            for c in cells:
                gp = g.detach().clone()
                gm = g.detach().clone()
                gp[c] += h
                gm[c] -= h
                xm = x0 + solve(gm, b - matvec(gm, x0))
                D = solve(gp, matvec(gm, xm) - matvec(gp, xm))
                dL = (D * (D + 2.0 * (xm - xobs))).sum().item()
                fd = dL / (2 * h)
                ga = grad[c].item()
                bound = 1e-4 * abs(ga) + 1e-6 * gmax + 2e-15 / (2 * h)
                worst = max(worst, abs(fd - ga) / bound)
                assert abs(fd - ga) <= bound, (h, c, fd, ga)
            _say(f"  h={h:.0e}, 100 cells: worst |fd - adj| / bound = {worst:.3f}")
    S.close()


def test_directional_derivative_1024(torch_gpu):
    """1024^2 cells: the adjoint gradient projected on a smooth direction v
    (a second Gaussian random field, all cells) against the central
    difference of L along v, with the difference solve of the cell test.
    The signal is spread over all cells, far above the loss-difference noise
    floor.  The O(h^2) term is large here (1.8e-5 relative at h = 1e-4,
    unchanged between solve tolerances 1e-13 and 1e-15), so the two central
    differences at h = 1e-4 and 2e-4 are combined by Richardson extrapolation
    (4 f(h) - f(2h)) / 3, which leaves O(h^4) ~ 3e-10.  Relative agreement
    1e-6."""
    torch = torch_gpu
    P, path, st = workloads.load("grf1024")
    fv, g0 = P.meta["fv"], P.meta["g"].ravel()
    S = mvamg.Solver(path)
    b = torch.from_numpy(P.b).cuda()
    g = torch.from_numpy(g0.copy()).cuda().requires_grad_(True)
    xobs = _observed(torch, S, fv, g.detach(), b, 0)
    x = amg_solve(fv.values_torch(g), b, S, rtol=1e-13)
    ((x - xobs) ** 2).sum().backward()
    v = torch.from_numpy(problems.grf(1024, seed=9).ravel()).cuda()
    dadj = float((g.grad * v).sum())
    x0 = x.detach()
    h = 1e-4

    def matvec(gv, u):
        mvamg.set_fine_values(S.h, fv.values_torch(gv))
        y = torch.empty_like(b)
        mvamg.spmv(S.h, u, y)
        return y

    def solve(gv, rhs):
        mvamg.set_fine_values(S.h, fv.values_torch(gv))
        d = torch.zeros_like(b)
        inf = mvamg.pcg_solve(S.h, rhs, d, rtol=1e-13, maxit=3000)
        assert inf.converged
        return d

    def central(step):
        gp = g.detach() + step * v
        gm = g.detach() - step * v
        xm = x0 + solve(gm, b - matvec(gm, x0))
        D = solve(gp, matvec(gm, xm) - matvec(gp, xm))
        return (D * (D + 2.0 * (xm - xobs))).sum().item() / (2 * step)

    with torch.no_grad():
        f1, f2 = central(h), central(2 * h)
    fd = (4.0 * f1 - f2) / 3.0
    _say(f"[grad dir] adjoint {dadj:.12e} central {f1:.12e} extrapolated {fd:.12e} "
         f"rel {abs(fd - dadj) / abs(dadj):.2e}")
    assert abs(fd - dadj) <= 1e-6 * abs(dadj)
    S.close()
