"""Benchmark: AMG-PCG solves/s on one MI355X.

Workload (N = 1): 3-D jump-coefficient diffusion, 7-point finite differences
on 128^3 nodes (n = 2,097,152), coefficient 1e3 or 1e-3 on 8^3-node cubes
selected with p = 0.5, else 1; b = A x*, x* ~ U[-1, 1]; hierarchy with at most
4 smooth vectors (setup on the host, untimed).  One step = one preconditioned
CG solve from x_0 = 0 to ||r|| <= 1e-8 ||r_0|| with the binary64 cycle, all
inputs resident in HBM.  The binary32-cycle variant is timed in the same run
and reported beside it.

Prints one JSON line (see the keys below).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def counted_bytes_per_iteration(lv, tr_U, nvec_k):
    """Algorithmic HBM bytes of one binary64 CG iteration (values 8 B, indices 4 B):
    S_l = 12 nnz_l + 4 (n_l + 1) per pass over A_l, T_l = 8 sum(n_a k_a) + 4 n_l + 8 n_agg
    per pass over P_l, V_l = 8 n_l per vector pass."""
    n, nnz = lv["n"], lv["nnz"]
    L = len(n) - 1
    S = [12 * nnz[l] + 4 * (n[l] + 1) for l in range(L + 1)]
    V = [8 * n[l] for l in range(L + 1)]
    b = S[0] + 15 * V[0]  # CG: A p, dot products, vector updates
    for l in range(L):
        T = 8 * tr_U[l] + 4 * n[l] + 8 * n[l + 1]
        b += 3 * S[l] + 2 * T + 13 * V[l]
    b += 3 * 8 * n[L] * n[L]  # coarsest: two dense products with A_L^{-1} and one residual
    return b


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="jump128")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=40)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); this build has no multi-GPU path.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1907_04417_amd import mvamg, workloads
    from oracle.hierfile import read_hierarchy

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    t0 = time.time()
    P, path, st = workloads.load(args.workload)
    log(f"[bench] setup {args.workload}: n={P.n} nnz={P.nnz} levels={st['n']} opc={st['opc']:.3f} "
        f"({time.time() - t0:.1f}s)")
    S = mvamg.Solver(path)
    stream = torch.cuda.current_stream()
    b = torch.from_numpy(P.b).cuda()
    x = torch.zeros_like(b)
    hist = np.zeros(1001)

    def solve(precision):
        x.zero_()
        return mvamg.pcg_solve(S.h, b, x, rtol=1e-8, maxit=1000, precision=precision, history=hist,
                               stream=stream)

    results = {}
    for prec in (64, 32):
        for _ in range(args.warmup):
            solve(prec)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t_wall = time.perf_counter()
        e0.record(stream)
        its = []
        for _ in range(args.steps):
            inf = solve(prec)
            its.append(inf.iterations)
        e1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t_wall
        ms = e0.elapsed_time(e1) / args.steps
        xs = x.cpu().numpy()
        err = float(np.abs(xs - P.x_star).max() / np.abs(P.x_star).max())
        results[prec] = dict(ms=ms, wall_ms=1e3 * wall / args.steps, nit=its[-1], converged=bool(inf.converged),
                             rel_res_true=inf.rel_res_true, err_vs_xstar=err, x=xs)
        log(f"[bench] precision {prec}: {ms:.3f} ms/solve, nit={its[-1]}, true_res={inf.rel_res_true:.2e}")

    H = read_hierarchy(path)
    lv = mvamg.levels(S.h)
    tr_U = [int(T.U.shape[0]) for T in H.transfers]
    bpi = counted_bytes_per_iteration(lv, tr_U, H.nvec)
    r64 = results[64]
    gbs = bpi * r64["nit"] / (r64["ms"] * 1e-3) / 1e9

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        O = oracle.Oracle(H)
        tc = time.perf_counter()
        _, ho, nit_c, _ = O.pcg(P.b, tol=1e-8, maxit=args.cpu_iters)
        tcpu = time.perf_counter() - tc
        per_it = tcpu / max(nit_c, 1)
        est = per_it * r64["nit"]
        cpu = dict(value=1.0 / est, unit="solves/s", cores=1, kind="oracle",
                   sample=f"{nit_c} of the {r64['nit']} CG iterations of one solve of the same system "
                          f"({tcpu:.1f} s), scaled to the full iteration count")
        log(f"[bench] oracle: {per_it * 1e3:.1f} ms/iteration -> {est:.1f} s/solve")

    r32 = results[32]
    out = {
        "metric": "AMG-PCG solves/s to 1e-8 rel. residual (FP64 cycle)",
        "value": 1e3 / r64["ms"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r64["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "jump128: 3-D jump-coefficient diffusion, 7-point FD, 128^3 nodes, "
                               "coefficient 1e3/1e-3 on 8^3 cubes (p=0.5), <=4 smooth vectors, rtol 1e-8",
                   "n": P.n, "nnz": P.nnz, "levels": lv["n"], "level_nnz": lv["nnz"], "stages": lv["stages"],
                   "opc": st["opc"], "nit": r64["nit"]},
        "hbm_gbs_counted": gbs,
        "bytes_per_iteration": bpi,
        "mixed": {"value": 1e3 / r32["ms"], "unit": "solves/s", "ms_per_step": r32["ms"], "nit": r32["nit"],
                  "speedup_vs_fp64": r64["ms"] / r32["ms"], "rel_res_true": r32["rel_res_true"],
                  "err_vs_fp64_solution": float(np.abs(r32["x"] - r64["x"]).max() / np.abs(r64["x"]).max())},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
