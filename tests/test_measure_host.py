"""Host logic of the profile tooling: kernel classes of rocprofv3 dispatches."""
from paper_1907_04417_amd.measure import classify_dispatches, kernel_class


def _cycle(fine_stage, coarse_stage, coarse_resid):
    """Kernel names of one PCG iteration on a three-level hierarchy with a
    grouped fine level, in launch order."""
    seq = ["void mvamg::k_zero_stage0_grp<double>(int)"] + [fine_stage.format(0)] * 3
    seq += ["void mvamg::k_resid_grp<double, 4, 0>(int)", "void mvamg::k_restrict<double, 8, 1, 64>(int)"]
    seq += ["void mvamg::k_zero_stage0_grp<double>(int)"] + [coarse_stage.format(0)] * 4
    seq += [coarse_resid, "void mvamg::k_restrict<double, 8, 0, 64>(int)", "void mvamg::k_symv_tiles(int)",
            "void mvamg::k_symv_sum(int)", "void mvamg::k_prolong_rows<double, 8>(int)"]
    seq += [coarse_stage.format(1)] * 5 + ["void mvamg::k_prolong_rows<double, 8>(int)"]
    seq += [fine_stage.format(1)] * 4 + ["void mvamg::k_resid_grp<double, 4, 1>(int)", "void mvamg::k_finish<1>(int)"]
    return seq


def test_grouped_smoothers_take_the_level_of_the_dispatch_order():
    # the same kernel name runs on the fine and on the coarse level
    names = _cycle("void mvamg::k_gs_grp<double, 4, {}>(int)", "void mvamg::k_gs_grp<double, 4, {}>(int)",
                   "void mvamg::k_resid_grp<double, 4, 0>(int)") * 2
    cls = classify_dispatches(dict(enumerate(names)))
    count = {}
    for k in cls.values():
        count[k] = count.get(k, 0) + 1
    assert count["smooth_fine"] == 2 * (1 + 3 + 4)
    assert count["smooth_coarse"] == 2 * (1 + 4 + 5)
    assert count["residual"] == 2 * 2 and count["spmv"] == 2
    assert count["restrict"] == 4 and count["prolong"] == 4 and count["coarse_solve"] == 4
    assert "k_finish" not in str(count)  # not a cycle kernel


def test_wide_kernels_are_classed():
    assert kernel_class("void mvamg::k_resid_grp_wide<double, 8>(int)") == "residual"
    assert kernel_class("void mvamg::k_bresid_grps<double, 4>(int)") == "residual"
    assert kernel_class("void mvamg::k_bgs_grps<double, 4>(int)") in ("smooth_fine", "smooth_coarse")
    assert kernel_class("void mvamg::k_gs_grp_wide<double, 8, 1>(int)") in ("smooth_fine", "smooth_coarse")
    names = _cycle("void mvamg::k_gs_grp<double, 4, {}>(int)", "void mvamg::k_gs_grp_wide<double, 8, {}>(int)",
                   "void mvamg::k_resid_grp_wide<double, 8>(int)")
    cls = classify_dispatches(dict(enumerate(names)))
    wide = [cls[d] for d, n in enumerate(names) if "k_gs_grp_wide" in n]
    assert wide and set(wide) == {"smooth_coarse"}
    assert [cls[d] for d, n in enumerate(names) if "k_gs_grp<" in n] == ["smooth_fine"] * 7


def test_binary32_kernels_are_not_classed():
    assert kernel_class("void mvamg::k_gs_grp<float, 4, 1>(int)") is None
    assert kernel_class("void mvamg::k_gs_sell<double, false>(int)") == "smooth_fine"


def test_bench_refuses_several_gpus():
    """bench.py measures one GPU: --gpus above 1 exits with a message before
    any GPU work."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=root)
    assert r.returncode == 2 and "one GPU only" in r.stderr
    assert r.stdout == ""


def test_recorded_traffic_matches_source_and_workload(tmp_path, monkeypatch):
    """bench.py takes a traffic line only for its kernel class, its workload and
    the current kernel-source hash (lines of other sources are stale)."""
    import bench
    src = bench.kernel_source_hash()
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "traffic.md").write_text(
        "```\n"
        f"traffic: smooth_coarse jump128 bytes_per_launch=1.5e+07 source={src}  (fetch ...)\n"
        "traffic: smooth_coarse jump128 bytes_per_launch=9.9e+07 source=000000000000  (older source)\n"
        f"traffic: spmv elast48 bytes_per_launch=3.0e+08 source={src}\n"
        "```\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: src)
    assert bench.recorded_traffic("smooth_coarse", "jump128") == 1.5e7
    assert bench.recorded_traffic("spmv", "elast48") == 3.0e8
    assert bench.recorded_traffic("spmv", "jump128") is None
    assert bench.recorded_traffic("residual", "elast48") is None


def test_block_path_dispatch_classes():
    """The block (several right-hand sides) kernels: a point fine level's
    stages are fine smoothing, the grouped coarse stages coarse smoothing, the
    block SpMV resets to the fine level."""
    seq = ["void mvamg::k_bstage0_point<double>(int)", "void mvamg::k_bgs_sell<double>(int)",
           "void mvamg::k_bresid_sell<double, 0>(int)", "void mvamg::k_brestrict<double, 4>(int)",
           "void mvamg::k_bgs_grp<double, 4>(int)", "void mvamg::k_bresid_grp<double, 4, 0>(int)",
           "void mvamg::k_brestrict<double, 4>(int)", "void mvamg::k_bgemm_mfma<0>(int)",
           "void mvamg::k_bprolong_rows<double, 4>(int)", "void mvamg::k_bgs_grp<double, 4>(int)",
           "void mvamg::k_bprolong_rows<double, 4>(int)", "void mvamg::k_bgs_sell<double>(int)",
           "void mvamg::k_bresid_sell<double, 1>(int)"]
    cls = [classify_dispatches(dict(enumerate(seq)))[d] for d in range(len(seq))]
    assert cls == ["smooth_fine", "smooth_fine", "residual", "restrict", "smooth_coarse", "residual", "restrict",
                   "coarse_solve", "prolong", "smooth_coarse", "prolong", "smooth_fine", "spmv"]
