"""Named synthetic workloads: problem generator + setup parameters, with the
hierarchy file cached on disk (setup is the untimed input generator).

    aniso64   2-D rotated anisotropic diffusion, 9-point, 64 x 64 interior grid
              (eps = 1e-2, theta = pi/4), at most 3 smooth vectors
    jump128   3-D jump-coefficient diffusion, 7-point, 128^3 (coefficient 1e3
              or 1e-3 on 8^3 cubes selected with p = 0.5, else 1), at most 4
              smooth vectors
    jump32    the same family on 32^3 (test size)
    grf1024   cell-centred 5-point finite volumes on 1024^2 cells, conductivity
              exp(g), g a Gaussian random field (length 0.05, sigma 1), b = h^2 * 1
    aniso1024 the aniso64 operator on a 1024 x 1024 grid (32 right-hand sides
              B = A X* from block_rhs(seed 5) in the multi-RHS runs)
    aniso520  the aniso64 operator on 520 x 520 (test size: its colour blocks
              lie more than 65535 rows apart, so the fine level mixes 16-bit
              and 32-bit column slabs)
    elast48   3-D linear elasticity, trilinear hexahedra, 48^3 free nodes x 3
              dofs (node-based), E = 1, nu = 0.3 with 10 % nu = 0.49 spherical
              inclusions, one face clamped and the opposite face pushed down;
              at most 6 smooth vectors, smoother groups of the 3 dofs of a node
    elast12   the same family on 12^3 nodes (test size)
    ani1_410  the paper's ANI1 (Section 5.1: eps = 1e-3, theta = 0) with linear
              elements on a structured triangulation, 410^2 interior nodes
              (n = 168,100), unit right-hand side, 5 smooth vectors (the
              paper's best solve time at its n = 168,577)
    ani1_160 / ani2_160  ANI1 and ANI2 (theta = pi/8) on 160^2 nodes with 4
              and 5 smooth vectors (test size)

Batches (load_batch): independent problems, each with its own hierarchy, all
set up with three levels (bootstrap depth at most 6, three bootstrap levels
composed per level, no size cap on the coarse levels):
    batch64   64 aniso9 problems, sides 32..512, eps 1e-4..1, theta 0..pi
    batch6    6 problems, sides 32..64 (test size)
"""
from __future__ import annotations

import hashlib
import json
import math
import os

from . import problems
from .setup import SetupParams, build_hierarchy

CONFIGS = {
    "aniso64": dict(gen=lambda: problems.aniso9(64, 1e-2, math.pi / 4, seed=0), nvec=3, setup={}),
    "aniso128": dict(gen=lambda: problems.aniso9(128, 1e-2, math.pi / 4, seed=0), nvec=3, setup={}),
    "jump128": dict(gen=lambda: problems.jump7(128, 8, 0.5, seed=0), nvec=4, setup={}),
    "jump32": dict(gen=lambda: problems.jump7(32, 4, 0.5, seed=1), nvec=4, setup={}),
    "jump16": dict(gen=lambda: problems.jump7(16, 2, 0.5, seed=2), nvec=4,
                   setup=dict(boot_coarse_min=8, coarse_cap=64, compose=2)),
    "grf1024": dict(gen=lambda: problems.grf_fv5(1024, seed=0), nvec=3, setup={}),
    "grf32": dict(gen=lambda: problems.grf_fv5(32, seed=3), nvec=3, setup=dict(boot_coarse_min=8, coarse_cap=64)),
    "aniso1024": dict(gen=lambda: problems.aniso9(1024, 1e-2, math.pi / 4, seed=0), nvec=3, setup={}),
    "aniso520": dict(gen=lambda: problems.aniso9(520, 1e-2, math.pi / 4, seed=0), nvec=3, setup={}),
    "ani1_410": dict(gen=lambda: problems.ani_p1(410, 1e-3, 0.0), nvec=5, setup={}),
    "ani1_160": dict(gen=lambda: problems.ani_p1(160, 1e-3, 0.0), nvec=4, setup={}),
    "ani2_160": dict(gen=lambda: problems.ani_p1(160, 1e-3, math.pi / 8), nvec=5, setup={}),
    "elast48": dict(gen=lambda: problems.elast_q1(48, seed=0), nvec=6, setup=dict(fine_group=3)),
    "elast12": dict(gen=lambda: problems.elast_q1(12, seed=0), nvec=6,
                    setup=dict(fine_group=3, boot_coarse_min=8, coarse_cap=64)),
}

BLOCK_RHS_SEED = 5

BATCH_SETUP = dict(boot_coarse_min=8, coarse_cap=0, max_levels=7, compose=3)
BATCHES = {
    "batch64": dict(gen=lambda: problems.aniso_batch(64, 32, 512, seed=0), nvec=3, setup=BATCH_SETUP),
    "batch6": dict(gen=lambda: problems.aniso_batch(6, 32, 64, seed=1), nvec=3, setup=BATCH_SETUP),
}

BOOTSTRAP_SEED = 1000


def _setup_source_tag() -> str:
    """Hash of the setup library's source: cached hierarchies are keyed by it,
    so a change to the setup never reuses files an older setup wrote."""
    src = os.path.join(os.path.dirname(os.path.abspath(__file__)), "setup", "mvsetup.cpp")
    with open(src, "rb") as f:
        return hashlib.sha1(f.read()).hexdigest()[:12]


def cache_dir() -> str:
    d = os.environ.get("MVAMG_CACHE", "/tmp/mvamg_cache")
    os.makedirs(d, exist_ok=True)
    return d


def load(name: str, **setup_overrides):
    """Returns (problem, hierarchy_path, setup_stats)."""
    cfg = CONFIGS[name]
    P = cfg["gen"]()
    sp = dict(cfg["setup"])
    sp.update(setup_overrides)
    sp.setdefault("nvec_max", cfg["nvec"])
    params = SetupParams(**sp)
    key = hashlib.sha1(json.dumps([name, sorted(params.__dict__.items()), _setup_source_tag()],
                                  default=str).encode()).hexdigest()[:12]
    path = os.path.join(cache_dir(), f"{name}_{key}.bin")
    meta = path + ".json"
    if os.path.exists(path) and os.path.exists(meta):
        with open(meta) as f:
            return P, path, json.load(f)
    x0 = problems.random_vectors(P.n, max(params.nvec_max - 1, 1), BOOTSTRAP_SEED)
    st = build_hierarchy(P.rowptr, P.col, P.val, path + ".tmp", x0, params)
    os.replace(path + ".tmp", path)
    with open(meta, "w") as f:
        json.dump(st, f)
    return P, path, st


def load_bootstrap(name: str, **setup_overrides):
    """The workload's hierarchy together with the hierarchies of its bootstrap
    stages B_1..B_r (every stage tested, rho_des = 0 so that the nvec - 1
    stages are all built).  Returns (problem, hierarchy_path, setup_stats,
    stage_paths, x0), x0 the random starts of the stages' testing phases."""
    cfg = CONFIGS[name]
    P = cfg["gen"]()
    sp = dict(cfg["setup"])
    sp.update(setup_overrides)
    sp.setdefault("nvec_max", cfg["nvec"])
    sp.setdefault("rho_des", 0.0)
    params = SetupParams(**sp)
    key = hashlib.sha1(json.dumps([name, "boot", sorted(params.__dict__.items()), _setup_source_tag()],
                                  default=str).encode()).hexdigest()[:12]
    path = os.path.join(cache_dir(), f"{name}_boot_{key}.bin")
    meta = path + ".json"
    x0 = problems.random_vectors(P.n, max(params.nvec_max - 1, 1), BOOTSTRAP_SEED)
    prefix = path[:-4]
    if not (os.path.exists(path) and os.path.exists(meta)):
        st = build_hierarchy(P.rowptr, P.col, P.val, path + ".tmp", x0, params, boot_prefix=prefix)
        os.replace(path + ".tmp", path)
        with open(meta, "w") as f:
            json.dump(st, f)
    with open(meta) as f:
        st = json.load(f)
    stages = [f"{prefix}_b{r}.bin" for r in range(1, len(st["rho"]) + 1)]
    return P, path, st, stages, x0


def _hierarchy(tag: str, P, nvec: int, setup: dict):
    params = SetupParams(nvec_max=nvec, **setup)
    key = hashlib.sha1(json.dumps([tag, P.n, P.nnz, sorted(params.__dict__.items()), _setup_source_tag()],
                                  default=str).encode()).hexdigest()[:12]
    path = os.path.join(cache_dir(), f"{tag}_{key}.bin")
    meta = path + ".json"
    if os.path.exists(path) and os.path.exists(meta):
        with open(meta) as f:
            return path, json.load(f)
    x0 = problems.random_vectors(P.n, max(nvec - 1, 1), BOOTSTRAP_SEED)
    st = build_hierarchy(P.rowptr, P.col, P.val, path + ".tmp", x0, params)
    os.replace(path + ".tmp", path)
    with open(meta, "w") as f:
        json.dump(st, f)
    return path, st


def load_batch(name: str):
    """Returns (problems, hierarchy_paths, setup_stats) of a batch."""
    cfg = BATCHES[name]
    Ps = cfg["gen"]()
    paths, stats = [], []
    for p, P in enumerate(Ps):
        path, st = _hierarchy(f"{name}_p{p}", P, cfg["nvec"], cfg["setup"])
        paths.append(path)
        stats.append(st)
    return Ps, paths, stats
