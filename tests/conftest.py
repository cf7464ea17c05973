import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: full-size workload")


@pytest.fixture(scope="session")
def setup_lib():
    from paper_1907_04417_amd.setup import LIB_PATH
    if not os.path.exists(LIB_PATH):
        from paper_1907_04417_amd.build import build_setup
        build_setup()
    return LIB_PATH


def make_hierarchy(tmpdir, prob, nvec, seed=100, **kw):
    from paper_1907_04417_amd import problems
    from paper_1907_04417_amd.setup import SetupParams, build_hierarchy
    path = os.path.join(str(tmpdir), f"{prob.name}_{nvec}_{seed}_{abs(hash(tuple(sorted(kw.items()))))}.bin")
    x0 = problems.random_vectors(prob.n, max(nvec - 1, 1), seed)
    st = build_hierarchy(prob.rowptr, prob.col, prob.val, path, x0, SetupParams(nvec_max=nvec, **kw))
    return path, st


@pytest.fixture(scope="session")
def tiny_hier(setup_lib, tmp_path_factory):
    """12x12 rotated anisotropic problem with a 3-level hierarchy."""
    from paper_1907_04417_amd import problems
    P = problems.aniso9(12, seed=3)
    path, st = make_hierarchy(tmp_path_factory.mktemp("h"), P, 3, boot_coarse_min=4, coarse_cap=12, compose=1)
    return P, path, st


@pytest.fixture(scope="session")
def small3d_hier(setup_lib, tmp_path_factory):
    """6^3 jump-coefficient problem (cubes of 2^3) with a multi-level hierarchy."""
    from paper_1907_04417_amd import problems
    P = problems.jump7(6, cube=2, seed=5)
    path, st = make_hierarchy(tmp_path_factory.mktemp("h"), P, 4, boot_coarse_min=4, coarse_cap=20, compose=1)
    return P, path, st
