"""Measurement helpers for the profiles kept with the repository.

    python -m paper_1907_04417_amd.measure run [workload] [steps]
        a plain 256 MiB device copy (counter calibration) followed by `steps`
        binary64 solves; meant to run under rocprofv3.  Workload
        aniso1024x32: the 32-column block solve on aniso1024; batch64: one
        batch solve of the 64 anisotropic problems.
    python -m paper_1907_04417_amd.measure traffic <fetch.csv> <write.csv> <workload>
        per-launch HBM traffic of every kernel class from two rocprofv3 --pmc
        runs (FETCH_SIZE, WRITE_SIZE), each scaled by the ratio of the copy's
        true bytes to what the same counter read for the copy; prints lines for
        profiles/traffic.md.
    python -m paper_1907_04417_amd.measure stats <kernel_stats.csv>
        the rocprofv3 --stats summary reduced to the solve's kernels.
"""
from __future__ import annotations

import csv
import tempfile
import os
import re
import sys
from collections import defaultdict

COPY_BYTES = 256 << 20


def kernel_class(name: str) -> str | None:
    """Kernel class (as in mvamg_kernel_stats) of a binary64 cycle kernel symbol."""
    if "k_bgemm" in name or "k_bsum_splits" in name or "k_symv_" in name:
        return "coarse_solve"
    if "double" not in name and "k_gemv" not in name:
        return None
    if "k_bgs_sell" in name or "k_bstage0_point" in name:
        return "smooth_fine"
    if "k_bgs_grp" in name or "k_bzero_stage0_grp" in name:
        return "smooth_coarse"
    if "k_bresid_grps" in name:  # block per group: residual only
        return "residual"
    m = re.search(r"k_bresid_(sell|grp)<double,(?:\d,)?(\d)>", name.replace(" ", ""))
    if m:
        return "spmv" if m.group(2) == "1" else "residual"
    if "k_brestrict" in name:
        return "restrict"
    if "k_bprolong_rows" in name:
        return "prolong"
    if "k_resid_grp_wide" in name:
        return "residual"
    if "k_gs_sell" in name or "k_stage0_point" in name:
        return "smooth_fine"
    if "k_gs_grp" in name or "k_zero_stage0_grp" in name:
        return "smooth_coarse"
    m = re.search(r"k_resid_(sell|grp)<double,[^>]*?(\d)>", name.replace(" ", ""))
    if m:
        return "spmv" if m.group(2) == "1" else "residual"
    if "k_restrict" in name:
        return "restrict"
    if "k_prolong_rows" in name:
        return "prolong"
    if "k_gemv" in name:
        return "coarse_solve"
    return None


def classify_dispatches(names: dict) -> dict:
    """Kernel class of every cycle dispatch (dispatch id -> class).  A grouped
    smoother kernel can run on the fine level or on a coarse one, so the level
    is followed through the dispatch order: a restriction moves one level down,
    a prolongation one level up, and the CG product (which only the fine level
    has) marks the fine level again."""
    out = {}
    level = 0
    for d in sorted(names):
        k = kernel_class(names[d])
        if k is None:
            continue
        if k in ("smooth_fine", "smooth_coarse"):
            k = "smooth_fine" if level == 0 else "smooth_coarse"
        elif k == "spmv":
            level = 0
        elif k == "restrict":
            level += 1
        elif k == "prolong":
            level = max(level - 1, 0)
        out[d] = k
    return out


def run(workload: str = "jump128", steps: int = 3) -> None:
    import numpy as np
    import torch

    from . import mvamg, workloads
    a = torch.empty(COPY_BYTES // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    c = torch.empty_like(a)
    torch.cuda.synchronize()
    c.copy_(a)  # the calibration copy: reads and writes COPY_BYTES
    torch.cuda.synchronize()
    del a, c
    # kernel choices as bench.py makes them (same tuning cache)
    cache = os.environ.get("MVAMG_TUNE_CACHE", os.path.join(tempfile.gettempdir(), "mvamg_tune.json"))
    if workload == "aniso1024x32":
        from . import problems
        P, path, st = workloads.load("aniso1024")
        S = mvamg.Solver(path, nrhs=32)
        mvamg.tuned(S.h, cache)
        B, _ = problems.block_rhs(P, 32, seed=workloads.BLOCK_RHS_SEED)
        Bd = torch.from_numpy(B).cuda()
        for _ in range(steps):
            X = torch.zeros_like(Bd)
            mvamg.pcg_solve_block(S.h, Bd, X, rtol=1e-8)
    elif workload == "batch64":
        Ps, paths, stats = workloads.load_batch("batch64")
        S = mvamg.BatchSolver(paths)
        mvamg.tuned(S.h, cache)
        b = torch.from_numpy(np.concatenate([P.b for P in Ps])).cuda()
        for _ in range(steps):
            x = torch.zeros_like(b)
            mvamg.batch_pcg_solve(S.h, b, x, rtol=1e-8)
    else:
        P, path, st = workloads.load(workload)
        S = mvamg.Solver(path)
        mvamg.tuned(S.h, cache)
        b = torch.from_numpy(P.b).cuda()
        for _ in range(steps):
            x = torch.zeros_like(b)
            mvamg.pcg_solve(S.h, b, x, rtol=1e-8)
    torch.cuda.synchronize()
    print(f"measure run done: {workload} x{steps}", flush=True)


def _rows(path):
    with open(path) as f:
        yield from csv.DictReader(f)


def traffic(fetch_csv: str, write_csv: str, workload: str) -> None:
    from bench import kernel_source_hash  # the source hash bench.py checks against
    out = {}
    for counter, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        per = defaultdict(float)  # dispatch -> KiB (summed over counter dimensions)
        names = {}
        for r in _rows(path):
            if r["Counter_Name"] != counter:
                continue
            d = int(r["Dispatch_Id"])
            per[d] += float(r["Counter_Value"])
            names[d] = r["Kernel_Name"]
        # the calibration copy: the runtime's / torch's copy kernel, not the library's own k_copy
        copy = [d for d, n in names.items()
                if ("copy" in n.lower() or "elementwise" in n.lower()) and "mvamg" not in n]
        copy_kib = max((per[d] for d in copy), default=0.0)
        scale = (COPY_BYTES / 1024.0) / copy_kib if copy_kib > 0 else 1.0
        acc = defaultdict(lambda: [0, 0.0])
        for d, k in classify_dispatches(names).items():
            acc[k][0] += 1
            acc[k][1] += per[d] * 1024.0 * scale
        out[counter] = (scale, acc)
    src = kernel_source_hash()
    fs, fa = out["FETCH_SIZE"]
    ws, wa = out["WRITE_SIZE"]
    print(f"calibration: copy of {COPY_BYTES} bytes read as {COPY_BYTES / fs / 1024:.0f} KiB fetched "
          f"(scale {fs:.4f}) and {COPY_BYTES / ws / 1024:.0f} KiB written (scale {ws:.4f})")
    for k in sorted(fa):
        n, fb = fa[k]
        wb = wa.get(k, [n, 0.0])[1]
        print(f"traffic: {k} {workload} bytes_per_launch={(fb + wb) / n:.6e} source={src}  "
              f"(fetch {fb / n:.4e} + write {wb / n:.4e} bytes, {n} launches)")


def stats(path: str) -> None:
    rows = list(_rows(path))
    tot = sum(float(r["TotalDurationNs"]) for r in rows)
    print(f"{'kernel':60s} {'calls':>7s} {'avg_us':>9s} {'total_ms':>9s} {'pct':>6s}")
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"]))[:30]:
        name = re.sub(r"\(.*", "", r["Name"]).replace("void mvamg::", "").replace("mvamg::", "")
        print(f"{name[:60]:60s} {int(r['Calls']):7d} {float(r['AverageNs']) / 1e3:9.2f} "
              f"{float(r['TotalDurationNs']) / 1e6:9.3f} {100 * float(r['TotalDurationNs']) / tot:6.1f}")


if __name__ == "__main__":
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    cmd = sys.argv[1]
    if cmd == "run":
        run(sys.argv[2] if len(sys.argv) > 2 else "jump128", int(sys.argv[3]) if len(sys.argv) > 3 else 3)
    elif cmd == "traffic":
        traffic(sys.argv[2], sys.argv[3], sys.argv[4])
    elif cmd == "stats":
        stats(sys.argv[2])
