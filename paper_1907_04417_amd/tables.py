"""The paper's anisotropic test cases (Section 5.1, Tables 1 and 2) on this
GPU: setup statistics and CG solves for 3..10 smooth vectors.

    python -m paper_1907_04417_amd.tables [--sizes 410,820,1640] [--nsv 3..8]
                                          [--cases ANI1,ANI2] [--bootstrap SIZES]

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

The GPU library relaxes the k_a coarse dofs of an aggregate together as one
Gauss-Seidel group of at most 8 rows, so nsv (which bounds k_a) stops at 8
here; the paper's tables go on to 10.

With --bootstrap SIZES, every case at those sizes also gets the paper's
comparison method (b-it, b-ts): the original composite bootstrap AMG, i.e.
stages built until the composite's estimate drops below rho_des = 0.8 or 15
stages exist, applied as the symmetrized multiplicative product of K-cycle
components (Section 5) -- and, for comparison, of V-cycle components -- as
the preconditioner of a flexible CG on the GPU.

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
                try:
                    st = build_hierarchy(P.rowptr, P.col, P.val, path, x0, SetupParams(nvec_max=nsv))
                except RuntimeError as e:  # the host setup's own limits (e.g. coarsening that stalls)
                    print(f"{case} n={P.n} nsv={nsv}: {e}", file=out, flush=True)
                    rows.append(dict(case=case, m=m, n=P.n, nsv=nsv, failed=str(e)))
                    continue
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
                           levels=n, composed=st["composed_stage"] + 1)
                rows.append(row)
                print(f"{case} n={P.n} nsv={nsv}: nl={row['nl']} opc={row['opc']:.2f} rho={row['rho']:.2f} "
                      f"cr={cr:.2f} tb={tb:.1f}s nit={row['nit']} ts={row['ts_ms']:.2f}ms "
                      f"(levels of stage {row['composed']} of {len(st['rho'])})", file=out, flush=True)
    return rows


def run_bootstrap(cases, sizes, steps: int = 3, out=sys.stdout):
    """b-it / b-ts rows: the original composite bootstrap AMG on the GPU."""
    import torch

    from . import mvamg, problems, workloads
    from .setup import SetupParams, build_hierarchy

    theta = {"ANI1": 0.0, "ANI2": math.pi / 8}
    rows = []
    tmpdir = os.environ.get("MVAMG_CACHE", "/tmp/mvamg_cache")
    os.makedirs(tmpdir, exist_ok=True)
    for case in cases:
        for m in sizes:
            P = problems.ani_p1(m, 1e-3, theta[case])
            prefix = os.path.join(tmpdir, f"{case}_{m}_boot")
            t0 = time.perf_counter()
            x0 = problems.random_vectors(P.n, 15, workloads.BOOTSTRAP_SEED)
            st = build_hierarchy(P.rowptr, P.col, P.val, prefix + "_main.bin", x0,
                                 SetupParams(nvec_max=16, rho_des=0.8, maxstage=15), boot_prefix=prefix)
            tb = time.perf_counter() - t0
            nst = len(st["rho"])
            Ss = [mvamg.Solver(f"{prefix}_b{r}.bin") for r in range(1, nst + 1)]
            C = mvamg.Composite(Ss)
            b = torch.from_numpy(P.b).cuda()
            out_c = {}
            for cyc in (mvamg.CYCLE_K, mvamg.CYCLE_V):
                times, res = [], None
                for _ in range(steps + 1 if cyc == mvamg.CYCLE_V else 2):
                    torch.cuda.synchronize()
                    t1 = time.perf_counter()
                    _, res = C.solve(b, rtol=1e-6, maxit=1000, cycle=cyc)
                    torch.cuda.synchronize()
                    times.append(time.perf_counter() - t1)
                out_c[cyc] = (res, 1e3 * float(np.median(times[1:])))
            # memory of the hierarchies relative to A: the sum of every stage's operator complexity
            nnz_all = sum(sum(S.info["nnz"]) for S in Ss)
            depths = [S.info["nlevels"] for S in Ss]
            for S in Ss:
                S.close()
            (rk, tk), (rv, tv) = out_c[mvamg.CYCLE_K], out_c[mvamg.CYCLE_V]
            row = dict(case=case, m=m, n=P.n, stages=nst, rho=st["rho"][-1], tb=tb, b_it=rk.iterations,
                       converged=bool(rk.converged and rv.converged), b_ts_ms=tk, b_it_v=rv.iterations,
                       b_ts_v_ms=tv, memory=nnz_all / P.nnz, depth=max(S_depth for S_depth in depths))
            rows.append(row)
            print(f"{case} n={P.n} original bootstrap: {nst} stages (up to {row['depth']} levels) rho={row['rho']:.2f} "
                  f"b-it={row['b_it']} b-ts={tk:.2f}ms (V-cycle components: {rv.iterations} it, {tv:.2f}ms) "
                  f"memory={row['memory']:.2f}x A tb={tb:.1f}s", file=out, flush=True)
    return rows


def markdown_bootstrap(rows) -> str:
    lines = ["| case | n | stages (levels) | rho | b-it | b-ts (ms, GPU, K-cycles) | it, ms with V-cycles | "
             "hierarchies' nnz / nnz(A) | tb (s, host) |",
             "|---|---:|---:|---:|---:|---:|---:|---:|---:|"]
    for r in rows:
        lines.append(f"| {r['case']} | {r['n']} | {r['stages']} ({r['depth']}) | {r['rho']:.2f} | {r['b_it']} | "
                     f"{r['b_ts_ms']:.1f} | {r['b_it_v']}, {r['b_ts_v_ms']:.1f} | {r['memory']:.2f} | {r['tb']:.1f} |")
    return "\n".join(lines)


def markdown(rows) -> str:
    lines = ["| case | n | nsv | nl | opc | rho | cr | tb (s, host) | nit | ts (ms, GPU) |",
             "|---|---:|---:|---:|---:|---:|---:|---:|---:|---:|"]
    for r in rows:
        if "failed" in r:
            lines.append(f"| {r['case']} | {r['n']} | {r['nsv']} | {r['failed']} | | | | | | |")
            continue
        lines.append(f"| {r['case']} | {r['n']} | {r['nsv']} | {r['nl']} | {r['opc']:.2f} | {r['rho']:.2f} | "
                     f"{r['cr']:.2f} | {r['tb']:.1f} | {r['nit']}{'' if r['converged'] else ' (no conv.)'} | "
                     f"{r['ts_ms']:.2f} |")
    return "\n".join(lines)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--cases", default="ANI1,ANI2")
    ap.add_argument("--sizes", default="410,820,1640")
    ap.add_argument("--nsv", default="3..8")
    ap.add_argument("--bootstrap", default="")
    args = ap.parse_args()
    cases, sizes = args.cases.split(","), _parse_range(args.sizes)
    brows = run_bootstrap(cases, _parse_range(args.bootstrap)) if args.bootstrap else []
    rows = run(cases, sizes, _parse_range(args.nsv))
    if brows:
        print(markdown_bootstrap(brows), flush=True)
    print(markdown(rows), flush=True)


if __name__ == "__main__":
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    main()
