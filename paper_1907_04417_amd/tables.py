"""The paper's anisotropic test cases (Section 5.1, Tables 1 and 2) on this
GPU: setup statistics and CG solves for 3..10 smooth vectors.

    python -m paper_1907_04417_amd.tables [--sizes 410,820,1640] [--nsv 3..10]
                                          [--cases ANI1,ANI2]

For every case (ANI1: theta = 0, ANI2: theta = pi/8, eps = 1e-3), size and
number of smooth vectors nsv, it runs the host setup (Algorithm 1 and the
multiple-vector hierarchy of Section 4, TOL = 0.1, rho_des = 0.8, nu = 15,
at most 15 stages, three bootstrap levels composed into aggregates of at
most 64 nodes) and then CG with the binary64 V-cycle on the GPU from x0 = 0
with the unit vector as right-hand side, stopped at a 1e-6 reduction of the
residual norm (at most 1000 iterations), as the paper's runs are.  Reported
per row: nl, opc, the last bootstrap convergence estimate rho, cr (average
over the nl - 1 coarsening steps), the setup time tb (host), nit, and the GPU
solve time ts (median of 3).  The GPU parity tests check the same solves
against the CPU oracle at a test size (ANI1 and ANI2 on 160^2 nodes).

The matrices are linear finite elements on structured triangulations (the
paper's PDE-toolbox meshes are not available): m^2 interior nodes with
m = 410, 820, 1640 give n = 168,100, 672,400 and 2,689,600, close to the
paper's 168,577, 673,025 and 2,689,537.  Only trends can be compared.
"""
from __future__ import annotations

import argparse
import math
import os
import sys
import time

import numpy as np

PAPER_N = {410: 168577, 820: 673025, 1640: 2689537}


def _parse_range(s: str):
    if ".." in s:
        a, b = s.split("..")
        return list(range(int(a), int(b) + 1))
    return [int(v) for v in s.split(",")]


def run(cases, sizes, nsvs, steps: int = 3, out=sys.stdout):
    import torch

    from . import mvamg, problems, workloads
    from .setup import SetupParams, build_hierarchy

    assert torch.cuda.is_available(), "the table runs need a GPU"
    theta = {"ANI1": 0.0, "ANI2": math.pi / 8}
    rows = []
    tmpdir = os.environ.get("MVAMG_CACHE", "/tmp/mvamg_cache")
    os.makedirs(tmpdir, exist_ok=True)
    for case in cases:
        for m in sizes:
            P = problems.ani_p1(m, 1e-3, theta[case])
            b = torch.from_numpy(P.b).cuda()
            for nsv in nsvs:
                path = os.path.join(tmpdir, f"{case}_{m}_{nsv}.bin")
                t0 = time.perf_counter()
                x0 = problems.random_vectors(P.n, nsv - 1, workloads.BOOTSTRAP_SEED)
                st = build_hierarchy(P.rowptr, P.col, P.val, path, x0, SetupParams(nvec_max=nsv))
                tb = time.perf_counter() - t0
                S = mvamg.Solver(path)
                x = torch.zeros_like(b)
                times = []
                inf = None
                for _ in range(steps + 1):
                    x.zero_()
                    torch.cuda.synchronize()
                    t1 = time.perf_counter()
                    inf = mvamg.pcg_solve(S.h, b, x, rtol=1e-6, maxit=1000)
                    torch.cuda.synchronize()
                    times.append(time.perf_counter() - t1)
                ts = float(np.median(times[1:]))
                S.close()
                n = st["n"]
                cr = float(np.mean([n[k - 1] / n[k] for k in range(1, len(n))]))
                row = dict(case=case, m=m, n=P.n, nsv=nsv, nl=st["nlevels"], opc=st["opc"], rho=st["rho"][-1],
                           cr=cr, tb=tb, nit=inf.iterations, converged=bool(inf.converged), ts_ms=1e3 * ts,
                           levels=n)
                rows.append(row)
                print(f"{case} n={P.n} nsv={nsv}: nl={row['nl']} opc={row['opc']:.2f} rho={row['rho']:.2f} "
                      f"cr={cr:.2f} tb={tb:.1f}s nit={row['nit']} ts={row['ts_ms']:.2f}ms", file=out, flush=True)
    return rows


def markdown(rows) -> str:
    lines = ["| case | n | nsv | nl | opc | rho | cr | tb (s, host) | nit | ts (ms, GPU) |",
             "|---|---:|---:|---:|---:|---:|---:|---:|---:|---:|"]
    for r in rows:
        lines.append(f"| {r['case']} | {r['n']} | {r['nsv']} | {r['nl']} | {r['opc']:.2f} | {r['rho']:.2f} | "
                     f"{r['cr']:.2f} | {r['tb']:.1f} | {r['nit']}{'' if r['converged'] else ' (no conv.)'} | "
                     f"{r['ts_ms']:.2f} |")
    return "\n".join(lines)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--cases", default="ANI1,ANI2")
    ap.add_argument("--sizes", default="410,820,1640")
    ap.add_argument("--nsv", default="3..10")
    args = ap.parse_args()
    rows = run(args.cases.split(","), _parse_range(args.sizes), _parse_range(args.nsv))
    print(markdown(rows), flush=True)


if __name__ == "__main__":
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    main()
