"""Error paths that need the device: invalid smoother stages and a non-s.p.d.
coarsest matrix are rejected at upload, an indefinite fine matrix stops CG
with a breakdown status.  Inputs are hierarchy files patched on the host."""
import os
import sys

import numpy as np
import pytest

from paper_1907_04417_amd import mvamg, workloads

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from hierpatch import patched_copy, read_chunk  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def test_upload_rejects_coupled_stage(torch_gpu, tmp_path):
    _, path, _ = workloads.load("jump16")
    bad = str(tmp_path / "stages.bin")
    patched_copy(path, bad, "A0.sptr", lambda v: np.where(np.arange(len(v)) == 0, 0, v[-1]))
    with pytest.raises(mvamg.MvamgError) as e:
        mvamg.Solver(bad)
    assert e.value.status == mvamg.ERR_FILE and "couples" in str(e.value)


def test_upload_rejects_indefinite_coarsest(torch_gpu, tmp_path):
    _, path, st = workloads.load("jump16")
    L = st["nlevels"] - 1
    bad = str(tmp_path / "coarsest.bin")
    patched_copy(path, bad, f"A{L}.val", lambda v: -v)
    with pytest.raises(mvamg.MvamgError) as e:
        mvamg.Solver(bad)
    assert e.value.status == mvamg.ERR_NOT_SPD


def test_indefinite_fine_matrix_is_a_breakdown(torch_gpu):
    torch = torch_gpu
    P, path, st = workloads.load("jump16")
    S = mvamg.Solver(path)
    mvamg.set_fine_values(S.h, torch.from_numpy(-P.val).cuda())
    b = torch.from_numpy(P.b).cuda()
    with pytest.raises(mvamg.MvamgError) as e:
        mvamg.pcg_solve(S.h, b, torch.zeros_like(b))
    assert e.value.status == mvamg.ERR_BREAKDOWN
    # the handle stays usable: original values, ordinary solve
    mvamg.set_fine_values(S.h, torch.from_numpy(P.val).cuda())
    x = torch.zeros_like(b)
    inf = mvamg.pcg_solve(S.h, b, x)
    assert inf.converged
    S.close()
