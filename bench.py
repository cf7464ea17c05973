"""Benchmark: AMG-PCG solves/s on one MI355X.

Workload (N = 1): 3-D jump-coefficient diffusion, 7-point finite differences
on 128^3 nodes (n = 2,097,152), coefficient 1e3 or 1e-3 on 8^3-node cubes
selected with p = 0.5, else 1; b = A x*, x* ~ U[-1, 1]; hierarchy with at most
4 smooth vectors (host setup, untimed).  One step = one preconditioned CG
solve from x_0 = 0 to ||r|| <= 1e-8 ||r_0|| with the binary64 cycle, inputs
resident in HBM.  The binary32-cycle variant (binary64 CG outside) is timed in
the same run and reported beside it.

Timing: `value` comes from K uninstrumented steps.  A second pass of the same
K steps carries start/stop HIP events on every cycle kernel (the library's
measurement switch) and yields the per-kernel-class time and algorithmic
bytes; the dominant class gives the `roofline` object.  Measured HBM traffic
(rocprofv3 FETCH_SIZE + WRITE_SIZE, calibrated with a plain copy) is taken
from profiles/traffic.md when it was recorded for the current kernel source.

Also measured in the same run (unless --no-multi), at equal 1e-8 relative
residual per system:
  * multi_rhs: 32 right-hand sides B = A X* on the 1024^2 rotated anisotropic
    problem, one block solve against 32 single-system binary64 solves;
  * batch: 64 independent anisotropic problems (sides 32..512) in one batch
    against 64 separate binary64 solves;
  * elasticity: the 48^3-node linear elasticity problem, binary64 solves and
    binary32-cycle solves.
All with the binary64 and the binary32 cycle; kernel choices from the
project's autotuner.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import tempfile
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
WORKLOAD_DESC = {
    "jump128": "jump128: 3-D jump-coefficient diffusion, 7-point FD, 128^3 nodes, coefficient 1e3/1e-3 on 8^3 "
               "cubes (p=0.5), <=4 smooth vectors, rtol 1e-8",
    "aniso64": "aniso64: 2-D rotated anisotropic diffusion, 9-point FD, 64^2 interior nodes, eps=1e-2, "
               "theta=pi/4, <=3 smooth vectors, rtol 1e-8",
    "elast48": "elast48: 3-D linear elasticity, trilinear hexahedra, 48^3 free nodes x 3 dofs (n = 331,776), E=1, "
               "nu=0.3 with 10% nu=0.49 spherical inclusions, one face clamped; <=6 smooth vectors, node-grouped "
               "fine smoother, rtol 1e-8",
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    """Hash of what per-launch traffic depends on: the kernel and layout
    sources, and the setup source that writes the hierarchies (stage counts,
    aggregates)."""
    h = hashlib.sha1()
    d = os.path.join(ROOT, "paper_1907_04417_amd", "csrc")
    for f in sorted(os.listdir(d)):
        if f.endswith((".hpp", ".hip")):
            h.update(open(os.path.join(d, f), "rb").read())
    h.update(open(os.path.join(ROOT, "paper_1907_04417_amd", "setup", "mvsetup.cpp"), "rb").read())
    return h.hexdigest()[:12]


def recorded_traffic(kclass_name: str, workload: str):
    """Per-launch HBM bytes of a kernel class from profiles/traffic.md, or None
    when none was recorded for the current kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic.md")
    if not os.path.exists(path):
        return None
    src = kernel_source_hash()
    for line in open(path):
        m = re.match(r"\s*traffic:\s+(\S+)\s+(\S+)\s+bytes_per_launch=([0-9.eE+]+)\s+source=(\S+)", line)
        if m and m.group(1) == kclass_name and m.group(2) == workload and m.group(4) == src:
            return float(m.group(3))
    return None


def counted_bytes_per_iteration(lv, nu):
    """Algorithmic HBM bytes of one binary64 CG iteration: a pass over A_l is
    12 nnz_l + 4 (n_l + 1) bytes, a pass over P_l is 8 sum(n_a k_a) + 4 n_l + 8 n_{l+1},
    a vector pass 8 n_l; the coarsest solve reads its n_L^2 inverse once."""
    n, nnz = lv["n"], lv["nnz"]
    L = len(n) - 1
    S = [12 * nnz[l] + 4 * (n[l] + 1) for l in range(L + 1)]
    V = [8 * n[l] for l in range(L + 1)]
    b = S[0] + 15 * V[0]
    for l in range(L):
        T = 8 * nu[l] + 4 * n[l] + 8 * n[l + 1]
        b += 3 * S[l] + 2 * T + 13 * V[l]
    b += 8 * n[L] * n[L]
    return b


def host_cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def measured_copy_gbs(torch, mib=1024, reps=10):
    """Stream-copy bandwidth of this GPU: bytes read + written per second by a
    plain device-to-device copy of `mib` MiB."""
    a = torch.empty(mib << 17, dtype=torch.float64, device="cuda").fill_(1.0)
    c = torch.empty_like(a)
    c.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        c.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2.0 * a.numel() * 8 * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, c
    torch.cuda.empty_cache()
    return gbs


def _timed_ms(torch, fn, steps, warmup):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(steps):
        out = fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t) * 1e3 / steps, out


def _kernel_table(mvamg, h, nsolves):
    kernels = {}
    for kc, name in enumerate(mvamg.KC_NAMES):
        nl, ms, by = mvamg.kernel_stats(h, kc)
        if nl:
            kernels[name] = dict(launches=nl // nsolves, ms_per_solve=ms / nsolves, us_per_launch=1e3 * ms / nl,
                                 gbs=by / (ms * 1e-3) / 1e9 if ms > 0 else None)
    return kernels


def bench_latency(args, torch, mvamg, workloads, tune_cache):
    """The small 2-D case (64^2 rotated anisotropic): a solve is a chain of
    short launches, so this measures latency, not bandwidth."""
    P, path, st = workloads.load("aniso64")
    S = mvamg.Solver(path)
    tune = mvamg.tuned(S.h, tune_cache)
    b = torch.from_numpy(P.b).cuda()
    x = torch.zeros_like(b)
    res = {}
    for prec in (64, 32):
        def solve():
            x.zero_()
            return mvamg.pcg_solve(S.h, b, x, rtol=1e-8, maxit=1000, precision=prec)
        ms, inf = _timed_ms(torch, solve, max(3, args.steps), 2)
        res[prec] = dict(ms=ms, nit=inf.iterations, ok=bool(inf.converged) and inf.rel_res_true <= 1.01e-8)
        log(f"[bench] aniso64 precision {prec}: {ms:.3f} ms/solve, nit={inf.iterations}")
    S.close()
    r64, r32 = res[64], res[32]
    return {
        "workload": WORKLOAD_DESC["aniso64"], "value": 1e3 / r64["ms"], "unit": "solves/s",
        "ms_per_solve": r64["ms"], "us_per_iteration": 1e3 * r64["ms"] / r64["nit"], "nit": r64["nit"],
        "levels": st["n"], "all_converged": r64["ok"] and r32["ok"], "tuning": tune,
        "fp32_cycle": {"value": 1e3 / r32["ms"], "ms_per_solve": r32["ms"], "nit": r32["nit"]},
    }


def bench_adjoint(args, torch, mvamg, workloads, tune_cache):
    """The differentiable solve on 1024^2 cells (kappa = exp(g), g a Gaussian
    random field): one step is the forward solve, the adjoint solve for
    L = ||x - x_obs||^2 and the coefficient gradient -lambda_i x_j, all to
    1e-8 with the binary64 cycle."""
    P, path, st = workloads.load("grf1024")
    S = mvamg.Solver(path)
    tune = mvamg.tuned(S.h, tune_cache)
    b = torch.from_numpy(P.b).cuda()
    val = torch.from_numpy(P.val).cuda()
    A = (None, None, val)
    x = torch.zeros_like(b)
    lam = torch.zeros_like(b)
    dval = torch.empty_like(val)
    mvamg.pcg_solve(S.h, b, x, rtol=1e-12, maxit=2000, A=A)
    rng = np.random.default_rng(1)
    rms = float(torch.sqrt((x * x).mean()))
    x_obs = x + torch.from_numpy(rng.normal(0.0, 0.01 * rms, P.n)).cuda()
    out = {}

    def step():
        x.zero_()
        fi = mvamg.pcg_solve(S.h, b, x, rtol=1e-8, maxit=1000, A=A)
        gx = 2.0 * (x - x_obs)
        ai = mvamg.adjoint_solve(S.h, gx, lam, rtol=1e-8, maxit=1000, A=A)
        mvamg.grad_coeffs(S.h, lam, x, dval)
        out["f"], out["a"] = fi, ai
        return fi, ai
    ms, _ = _timed_ms(torch, step, max(1, min(args.steps, 5)), 1)

    def fwd():
        x.zero_()
        return mvamg.pcg_solve(S.h, b, x, rtol=1e-8, maxit=1000, A=A)
    ms_f, _ = _timed_ms(torch, fwd, max(1, min(args.steps, 5)), 1)
    fi, ai = out["f"], out["a"]
    ok = bool(fi.converged and ai.converged) and fi.rel_res_true <= 1.01e-8 and ai.rel_res_true <= 1.01e-8
    log(f"[bench] grf1024 forward + adjoint + gradient: {ms:.2f} ms (forward alone {ms_f:.2f} ms), "
        f"nit {fi.iterations} + {ai.iterations}")
    S.close()
    return {
        "workload": "grf1024: cell-centred 5-point finite volumes on 1024^2 cells, kappa = exp(g), g Gaussian random "
                    "field (squared-exponential covariance, length 0.05), b = h^2; L = ||x - x_obs||^2; forward and "
                    "adjoint solves to rtol 1e-8 (binary64 cycle) and the coefficient gradient",
        "value": 1e3 / ms, "unit": "gradients/s", "ms_per_gradient": ms, "ms_forward": ms_f,
        "nit_forward": fi.iterations, "nit_adjoint": ai.iterations, "levels": st["n"], "all_converged": ok,
        "tuning": tune,
    }


def bench_multi_rhs(args, torch, mvamg, workloads, tune_cache):
    """32 right-hand sides through one hierarchy (block solve) against 32
    single-system solves of the same columns."""
    from paper_1907_04417_amd import problems
    t0 = time.time()
    P, path, st = workloads.load("aniso1024")
    S = mvamg.Solver(path, nrhs=32)
    tune = mvamg.tuned(S.h, tune_cache)
    log(f"[bench] multi-rhs aniso1024: levels={st['n']} setup+upload {time.time() - t0:.1f}s tuning {tune}")
    B, _ = problems.block_rhs(P, 32, seed=workloads.BLOCK_RHS_SEED)
    Bd = torch.from_numpy(B).cuda()
    X = torch.zeros_like(Bd)
    steps = max(1, min(args.steps, 3))
    res = {}
    for prec in (64, 32):
        def blk():
            X.zero_()
            return mvamg.pcg_solve_block(S.h, Bd, X, rtol=1e-8, precision=prec)
        ms, infos = _timed_ms(torch, blk, steps, 1)
        its = [i.iterations for i in infos]
        ok = all(i.converged and i.rel_res_true <= 1.01e-8 for i in infos)
        cols = [Bd[:, c].contiguous() for c in range(32)]
        xs = torch.zeros(P.n, dtype=torch.float64, device="cuda")

        def singles():
            for c in range(32):
                xs.zero_()
                mvamg.pcg_solve(S.h, cols[c], xs, rtol=1e-8, precision=prec)
        ms1, _ = _timed_ms(torch, singles, 1, 0)
        res[prec] = dict(ms=ms, ms_single_total=ms1, its=(min(its), max(its)), ok=ok)
        log(f"[bench] multi-rhs precision {prec}: {ms:.1f} ms per 32-column solve, 32 single solves {ms1:.1f} ms")
    mvamg.profile(S.h, True)
    X.zero_()
    mvamg.pcg_solve_block(S.h, Bd, X, rtol=1e-8)
    torch.cuda.synchronize()
    kernels = _kernel_table(mvamg, S.h, 1)
    mvamg.profile(S.h, False)
    dom = max(kernels, key=lambda k: kernels[k]["ms_per_solve"])
    S.close()
    r64, r32 = res[64], res[32]
    return {
        "workload": "aniso1024 x 32: 2-D rotated anisotropic diffusion, 9-point FD, 1024^2 (n = 1,048,576), "
                    "eps=1e-2, theta=pi/4, <=3 smooth vectors; 32 right-hand sides B = A X*, X* ~ U[-1,1]; rtol 1e-8 "
                    "per column",
        "value": 32e3 / r64["ms"], "unit": "solves/s", "ms_per_block_solve": r64["ms"], "nit": r64["its"],
        "all_converged": r64["ok"] and r32["ok"],
        "single_fp64_ms_for_32": res[64]["ms_single_total"], "speedup_vs_single_fp64": res[64]["ms_single_total"] / r64["ms"],
        "fp32_cycle": {"value": 32e3 / r32["ms"], "ms_per_block_solve": r32["ms"], "nit": r32["its"],
                       "speedup_vs_single_fp64": res[64]["ms_single_total"] / r32["ms"]},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": kernels[dom]["gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": kernels[dom]["gbs"] / HBM_PEAK_GBS, "traffic": recorded_traffic(dom, "aniso1024x32")},
        "kernels": kernels,
    }


def bench_batch(args, torch, mvamg, workloads, tune_cache):
    """64 independent problems in one batch against 64 separate solves."""
    t0 = time.time()
    Ps, paths, stats = workloads.load_batch("batch64")
    BS = mvamg.BatchSolver(paths)
    tune = mvamg.tuned(BS.h, tune_cache)
    log(f"[bench] batch64: rows={sum(P.n for P in Ps)} setup+upload {time.time() - t0:.1f}s tuning {tune}")
    b = torch.from_numpy(np.concatenate([P.b for P in Ps])).cuda()
    x = torch.zeros_like(b)
    steps = max(1, min(args.steps, 3))
    Ss = [mvamg.Solver(p) for p in paths]
    for S1 in Ss:
        mvamg.tuned(S1.h, tune_cache)
    bs = [torch.from_numpy(P.b).cuda() for P in Ps]
    xs = [torch.zeros_like(v) for v in bs]
    res = {}
    for prec in (64, 32):
        def bat():
            x.zero_()
            return mvamg.batch_pcg_solve(BS.h, b, x, rtol=1e-8, precision=prec)
        ms, infos = _timed_ms(torch, bat, steps, 1)
        its = [i.iterations for i in infos]
        ok = all(i.converged and i.rel_res_true <= 1.01e-8 for i in infos)

        def seq():
            for S1, bb, xx in zip(Ss, bs, xs):
                xx.zero_()
                mvamg.pcg_solve(S1.h, bb, xx, rtol=1e-8, precision=prec)
        ms1, _ = _timed_ms(torch, seq, 1, 1)
        res[prec] = dict(ms=ms, ms_seq=ms1, its=(min(its), max(its)), ok=ok)
        log(f"[bench] batch precision {prec}: {ms:.1f} ms per batch, 64 separate solves {ms1:.1f} ms")
    mvamg.profile(BS.h, True)
    x.zero_()
    mvamg.batch_pcg_solve(BS.h, b, x, rtol=1e-8)
    torch.cuda.synchronize()
    kernels = _kernel_table(mvamg, BS.h, 1)
    mvamg.profile(BS.h, False)
    dom = max(kernels, key=lambda k: kernels[k]["ms_per_solve"])
    for S1 in Ss:
        S1.close()
    BS.close()
    # the one-launch small-problem path for the problems up to a size threshold
    # (every problem at the largest), the rest lockstep; binary64
    small = {}
    for thr in (16384, 65536, 1 << 30):
        BSm = mvamg.BatchSolver(paths, mini_rows=thr)
        nsmall = sum(mvamg.batch_small_path(BSm.h))

        def batm():
            x.zero_()
            return mvamg.batch_pcg_solve(BSm.h, b, x, rtol=1e-8)
        msm, infos = _timed_ms(torch, batm, steps, 1)
        ok = all(i.converged and i.rel_res_true <= 1.01e-8 for i in infos)
        small[str(thr)] = dict(problems_on_small_path=nsmall, ms_per_batch=msm, all_converged=ok)
        log(f"[bench] batch with problems up to {thr} rows on the small path ({nsmall} of 64): {msm:.1f} ms")
        BSm.close()
    r64, r32 = res[64], res[32]
    return {
        "workload": "batch64: 64 independent 2-D rotated anisotropic 9-point problems, sides U{32..512}, eps "
                    "log-uniform [1e-4, 1], theta U[0, pi), own 3-level hierarchies (<=3 smooth vectors); rtol 1e-8 "
                    "per problem",
        "value": 64e3 / r64["ms"], "unit": "problems/s", "ms_per_batch": r64["ms"], "nit": r64["its"],
        "rows": int(sum(P.n for P in Ps)), "all_converged": r64["ok"] and r32["ok"],
        "separate_fp64_ms_for_64": r64["ms_seq"], "speedup_vs_separate_fp64": r64["ms_seq"] / r64["ms"],
        "fp32_cycle": {"value": 64e3 / r32["ms"], "ms_per_batch": r32["ms"], "nit": r32["its"],
                       "speedup_vs_separate_fp64": r64["ms_seq"] / r32["ms"]},
        "small_path_fp64": small,
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": kernels[dom]["gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": kernels[dom]["gbs"] / HBM_PEAK_GBS, "traffic": recorded_traffic(dom, "batch64")},
        "kernels": kernels,
    }


def bench_elasticity(args, torch, mvamg, workloads, tune_cache):
    """3-D linear elasticity (48^3 nodes x 3 dofs, nearly incompressible
    inclusions): binary64 solves and binary32-cycle solves with binary64 CG,
    both to 1e-8."""
    t0 = time.time()
    P, path, st = workloads.load("elast48")
    S = mvamg.Solver(path)
    tune = mvamg.tuned(S.h, tune_cache)
    log(f"[bench] elast48: levels={st['n']} setup+upload {time.time() - t0:.1f}s tuning {tune}")
    b = torch.from_numpy(P.b).cuda()
    x = torch.zeros_like(b)
    steps = max(1, min(args.steps, 3))
    res = {}
    for prec in (64, 32):
        def solve():
            x.zero_()
            return mvamg.pcg_solve(S.h, b, x, rtol=1e-8, maxit=1000, precision=prec)
        ms, inf = _timed_ms(torch, solve, steps, 1)
        res[prec] = dict(ms=ms, nit=inf.iterations, ok=bool(inf.converged) and inf.rel_res_true <= 1.01e-8,
                         true=inf.rel_res_true, x=x.cpu().numpy())
        log(f"[bench] elast48 precision {prec}: {ms:.2f} ms/solve, nit={inf.iterations}, "
            f"true_res={inf.rel_res_true:.2e}")
    mvamg.profile(S.h, True)
    x.zero_()
    mvamg.pcg_solve(S.h, b, x, rtol=1e-8, maxit=1000)
    torch.cuda.synchronize()
    kernels = _kernel_table(mvamg, S.h, 1)
    mvamg.profile(S.h, False)
    dom = max(kernels, key=lambda k: kernels[k]["ms_per_solve"])
    S.close()
    r64, r32 = res[64], res[32]
    return {
        "workload": WORKLOAD_DESC.get("elast48", "elast48"),
        "value": 1e3 / r64["ms"], "unit": "solves/s", "ms_per_solve": r64["ms"], "nit": r64["nit"],
        "levels": st["n"], "all_converged": r64["ok"] and r32["ok"],
        "fp32_cycle": {"value": 1e3 / r32["ms"], "ms_per_solve": r32["ms"], "nit": r32["nit"],
                       "rel_res_true": r32["true"], "speedup_vs_fp64": r64["ms"] / r32["ms"],
                       "err_vs_fp64_solution": float(np.abs(r32["x"] - r64["x"]).max() / np.abs(r64["x"]).max())},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": kernels[dom]["gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": kernels[dom]["gbs"] / HBM_PEAK_GBS, "traffic": recorded_traffic(dom, "elast48")},
        "kernels": kernels,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="jump128")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile-pass", action="store_true")
    ap.add_argument("--no-multi", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}): the library has no multi-GPU path; "
              f"run it with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1907_04417_amd import mvamg, workloads

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    copy_gbs = measured_copy_gbs(torch)
    log(f"[bench] device copy: {copy_gbs:.0f} GB/s (read + write)")
    t0 = time.time()
    P, path, st = workloads.load(args.workload)
    log(f"[bench] setup {args.workload}: n={P.n} nnz={P.nnz} levels={st['n']} opc={st['opc']:.3f} "
        f"({time.time() - t0:.1f}s)")
    S = mvamg.Solver(path)
    tune_cache = os.environ.get("MVAMG_TUNE_CACHE", os.path.join(tempfile.gettempdir(), "mvamg_tune.json"))
    log(f"[bench] tuning: {mvamg.tuned(S.h, tune_cache)}")
    stream = torch.cuda.current_stream()
    b = torch.from_numpy(P.b).cuda()
    x = torch.zeros_like(b)
    hist = np.zeros(1001)
    # the matrix is passed to every solve (its pattern and values are checked
    # against the hierarchy's inside the timed call)
    A = (torch.from_numpy(P.rowptr.astype(np.int32)).cuda(), torch.from_numpy(P.col.astype(np.int32)).cuda(),
         torch.from_numpy(P.val).cuda())
    # at most 256 distinct off-diagonal values: the fine kernels read 1-byte codes
    offdiag = P.val[P.col != np.repeat(np.arange(P.n), np.diff(P.rowptr))]
    value_codes = bool(np.unique(offdiag).size <= 256)

    def solve(precision):
        x.zero_()
        return mvamg.pcg_solve(S.h, b, x, rtol=1e-8, maxit=1000, precision=precision, history=hist,
                               stream=stream, A=A)

    def timed(precision):
        for _ in range(args.warmup):
            solve(precision)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.steps):
            inf = solve(precision)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / args.steps, inf

    results = {}
    for prec in (64, 32):
        ms, inf = timed(prec)
        xs = x.cpu().numpy()
        results[prec] = dict(ms=ms, nit=inf.iterations, converged=bool(inf.converged),
                             rel_res_true=inf.rel_res_true, x=xs)
        log(f"[bench] precision {prec}: {ms:.3f} ms/solve, nit={inf.iterations}, true_res={inf.rel_res_true:.2e}")

    for prec, r in results.items():
        if not (r["converged"] and r["rel_res_true"] <= 1.01e-8):
            log(f"[bench] FAILED: precision {prec} did not reach 1e-8 (converged={r['converged']}, "
                f"true residual {r['rel_res_true']:.2e})")
            sys.exit(3)
    lv = mvamg.levels(S.h)
    bpi = counted_bytes_per_iteration(lv, mvamg.transfers(S.h)["nu"])
    r64 = results[64]

    roofline = None
    kernels = {}
    if not args.no_profile_pass:
        # two passes with per-launch events: bytes in the plain model (12 B per
        # stored binary64 entry, the figure `frac` uses) and in the compact forms
        # the kernels actually read
        booked = {}
        for booking in (mvamg.BOOK_PLAIN, mvamg.BOOK_COMPACT):
            mvamg.profile(S.h, True, booking)
            t_prof = time.perf_counter()
            for _ in range(args.steps):
                solve(64)
            torch.cuda.synchronize()
            t_prof = (time.perf_counter() - t_prof) * 1e3 / args.steps
            tab = {}
            for kc, name in enumerate(mvamg.KC_NAMES):
                nl, ms, by = mvamg.kernel_stats(S.h, kc)
                if nl:
                    tab[name] = dict(launches=nl // args.steps, ms_per_step=ms / args.steps,
                                     us_per_launch=1e3 * ms / nl, gbs=by / (ms * 1e-3) / 1e9 if ms > 0 else None,
                                     bytes_per_launch=by / nl)
            mvamg.profile(S.h, False)
            booked[booking] = (tab, t_prof)
        kernels, t_prof = booked[mvamg.BOOK_PLAIN]
        compact = booked[mvamg.BOOK_COMPACT][0]
        for name, k in kernels.items():
            k["gbs_compact"] = compact[name]["gbs"]
            k["bytes_per_launch_compact"] = compact[name]["bytes_per_launch"]
        dom = max(kernels, key=lambda k: kernels[k]["ms_per_step"])
        dl = kernels[dom]
        achieved = dl["gbs"]
        traffic = recorded_traffic(dom, args.workload)
        roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": dom,
                    "bytes_model": "plain: 12 B per stored binary64 entry + 4 B per row + 8 B per vector element "
                                   "touched (frac); compact: the forms the kernels read (frac_compact)",
                    "bytes_per_launch": dl["bytes_per_launch"],
                    "achieved_compact": dl["gbs_compact"], "frac_compact": dl["gbs_compact"] / HBM_PEAK_GBS,
                    "bytes_per_launch_compact": dl["bytes_per_launch_compact"],
                    "fine_value_codes": value_codes,
                    "measured_copy_gbs": copy_gbs, "frac_of_copy": achieved / copy_gbs,
                    "launches_per_step": dl["launches"], "us_per_launch": dl["us_per_launch"],
                    "profiled_ms_per_step": t_prof}
        log(f"[bench] dominant kernel class {dom}: {dl['ms_per_step']:.2f} ms/step over {dl['launches']} launches, "
            f"{achieved:.0f} GB/s plain, {dl['gbs_compact']:.0f} GB/s compact")

    # the same solves reading the stored values (no 1-byte value codes): a
    # refill with the same values retires the codes
    codes_off = None
    if value_codes:
        mvamg.set_fine_values(S.h, A[2])
        ms_off, inf_off = timed(64)
        codes_off = {"value": 1e3 / ms_off, "unit": "solves/s", "ms_per_step": ms_off, "nit": inf_off.iterations,
                     "rel_res_true": inf_off.rel_res_true}
        log(f"[bench] without value codes: {ms_off:.3f} ms/solve")

    cpu = None
    x_oracle = None
    if not args.no_cpu_baseline:
        import oracle
        tc = time.perf_counter()
        O = oracle.Oracle(path)
        tf = time.perf_counter() - tc
        tc = time.perf_counter()
        x_oracle, ho, nit_c, _ = O.pcg(P.b, tol=1e-8)
        tcpu = time.perf_counter() - tc
        cpu = dict(value=1.0 / tcpu, unit="solves/s", cores=1, kind="oracle",
                   host_cpu=host_cpu_model(), host_threads=os.cpu_count(),
                   sample=f"one complete solve of the same system ({nit_c} CG iterations, {tcpu:.1f} s on one host "
                          f"core; the oracle's own coarsest factorisation, {tf:.1f} s, is setup and not counted)")
        log(f"[bench] oracle: {tcpu:.1f} s/solve ({nit_c} iterations)")

    S.close()
    multi = batch = elast = latency = adjoint = None
    if not args.no_multi:
        latency = bench_latency(args, torch, mvamg, workloads, tune_cache)
        multi = bench_multi_rhs(args, torch, mvamg, workloads, tune_cache)
        batch = bench_batch(args, torch, mvamg, workloads, tune_cache)
        elast = bench_elasticity(args, torch, mvamg, workloads, tune_cache)
        adjoint = bench_adjoint(args, torch, mvamg, workloads, tune_cache)

    def err_vs(xa, xb):
        return None if xb is None else float(np.abs(xa - xb).max() / np.abs(xb).max())

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
        "config": {"workload": WORKLOAD_DESC.get(args.workload, args.workload), "n": P.n, "nnz": P.nnz,
                   "levels": lv["n"], "level_nnz": lv["nnz"], "stages": lv["stages"], "opc": st["opc"],
                   "nit": r64["nit"]},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "hbm_gbs_counted_whole_solve": bpi * r64["nit"] / (r64["ms"] * 1e-3) / 1e9,
        "bytes_per_iteration": bpi,
        "kernels": kernels,
        "rel_res_true": r64["rel_res_true"],
        "err_vs_oracle": err_vs(r64["x"], x_oracle),
        "value_codes_off": codes_off,
        "mixed": {"value": 1e3 / r32["ms"], "unit": "solves/s", "dtype": "f32 cycle, f64 CG",
                  "ms_per_step": r32["ms"], "nit": r32["nit"], "speedup_vs_fp64": r64["ms"] / r32["ms"],
                  "rel_res_true": r32["rel_res_true"],
                  "err_vs_oracle": err_vs(r32["x"], x_oracle),
                  "err_vs_fp64_solution": err_vs(r32["x"], r64["x"])},
        "latency": latency,
        "adjoint": adjoint,
        "multi_rhs": multi,
        "batch": batch,
        "elasticity": elast,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
