"""C ABI checks that need no GPU: the library loads, exports every entry point
declared in include/mvamg.h, and its host-only file reader validates input."""
import ctypes
import os
import re

import pytest

from paper_1907_04417_amd import mvamg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "mvamg.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(mvamg_[a-z0-9_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(mvamg.LIB_PATH):
        from paper_1907_04417_amd.build import build_hip
        build_hip()
    return mvamg.load()


def test_header_declares_binding_names():
    assert _declared() == sorted(mvamg.EXPORTED)


def test_library_exports_every_declared_symbol(lib):
    for name in _declared():
        assert hasattr(lib, name), name


def test_hier_read_roundtrip(lib, tiny_hier):
    P, path, st = tiny_hier
    hh = mvamg.hier_read(path)
    try:
        nl, n, nnz = mvamg.hier_host_info(hh)
        assert (nl, n, nnz) == (st["nlevels"], P.n, P.nnz)
    finally:
        mvamg.hier_host_free(hh)


def test_hier_read_rejects_bad_files(lib, tiny_hier, tmp_path):
    _, path, _ = tiny_hier
    buf = open(path, "rb").read()
    cases = {"magic": b"NOTAHIER" + buf[8:], "truncated": buf[: len(buf) // 3], "empty": b""}
    for name, data in cases.items():
        f = tmp_path / f"{name}.bin"
        f.write_bytes(data)
        with pytest.raises(mvamg.MvamgError) as e:
            mvamg.hier_read(str(f))
        assert e.value.status == mvamg.ERR_FILE, name
    with pytest.raises(mvamg.MvamgError):
        mvamg.hier_read(str(tmp_path / "missing.bin"))


def test_null_handle_is_an_argument_error(lib):
    rc = lib.mvamg_levels(None, None, None, None, None)
    assert rc == mvamg.ERR_ARG
    assert "null" in mvamg.last_error()


def test_batch_upload_validates_on_the_host(lib, tiny_hier, tmp_path):
    """A batch needs at least one problem and no null entries; hierarchies of
    different depth are accepted (the odd ones take the small-problem path).
    Checked before any device work."""
    from paper_1907_04417_amd import problems
    from paper_1907_04417_amd.setup import SetupParams, build_hierarchy
    _, path3, st3 = tiny_hier
    P = problems.aniso9(10, seed=4)
    path2 = str(tmp_path / "two_levels.bin")
    st2 = build_hierarchy(P.rowptr, P.col, P.val, path2, problems.random_vectors(P.n, 1, 7),
                          SetupParams(nvec_max=2, boot_coarse_min=4, coarse_cap=40, compose=1))
    assert st2["nlevels"] != st3["nlevels"]
    hs = [mvamg.hier_read(path3), mvamg.hier_read(path2)]
    try:
        out = ctypes.c_void_p()
        nb = ctypes.c_size_t()
        arr = (ctypes.c_void_p * 2)(*hs)
        assert lib.mvamg_batch_arena_bytes(arr, 2, 0, ctypes.byref(nb)) == mvamg.OK and nb.value > 0
        assert lib.mvamg_batch_arena_bytes(arr, 0, 0, ctypes.byref(nb)) == mvamg.ERR_ARG
        assert lib.mvamg_batch_arena_bytes(arr, 2, -1, ctypes.byref(nb)) == mvamg.ERR_ARG
        nul = (ctypes.c_void_p * 2)(hs[0], None)
        assert lib.mvamg_batch_arena_bytes(nul, 2, 0, ctypes.byref(nb)) == mvamg.ERR_ARG
        # every problem on the small path, and a mixed split: both sized on the host
        assert lib.mvamg_batch_arena_bytes(arr, 2, 1 << 30, ctypes.byref(nb)) == mvamg.OK and nb.value > 0
        # no arena: rejected before any device work
        assert lib.mvamg_batch_upload(arr, 2, 0, None, nb.value, None, ctypes.byref(out)) == mvamg.ERR_ARG
        assert out.value is None
    finally:
        for hh in hs:
            mvamg.hier_host_free(hh)


def test_arena_bytes_on_the_host(lib, tiny_hier):
    """The arena size is computed on the host (no device work): it covers at
    least the stored matrices, grows with the block work space, and the
    upload rejects a missing or unaligned arena before touching the device."""
    P, path, st = tiny_hier
    hh = mvamg.hier_read(path)
    try:
        b1, b32 = mvamg.arena_bytes(hh, 1), mvamg.arena_bytes(hh, 32)
        # every level's values in binary64 and binary32 and its column indices
        assert b1 >= sum(12 * z + 4 * z for z in st["nnz"][:-1])
        # block work space: at least r, x in both precisions per row and level, 32 columns
        assert b32 - b1 >= sum(24 * 32 * n for n in st["n"])
        assert mvamg.arena_bytes(hh, 1) == b1  # deterministic
        nb = ctypes.c_size_t()
        for bad in (0, 33):
            assert lib.mvamg_arena_bytes(hh, bad, ctypes.byref(nb)) == mvamg.ERR_ARG
        out = ctypes.c_void_p()
        assert lib.mvamg_upload(hh, None, b1, None, ctypes.byref(out)) == mvamg.ERR_ARG
        assert lib.mvamg_upload(hh, ctypes.c_void_p(0x10000 + 8), b1, None, ctypes.byref(out)) == mvamg.ERR_ARG
        assert "aligned" in mvamg.last_error() and out.value is None
    finally:
        mvamg.hier_host_free(hh)


def test_single_level_hierarchy_is_rejected_on_the_host(lib, setup_lib, tmp_path):
    """A problem no larger than the bootstrap's coarsest size gives a one-level
    hierarchy (the whole solve would be the coarsest level's direct solve).
    The library needs a level to smooth and says so before any device work."""
    from paper_1907_04417_amd import problems
    from paper_1907_04417_amd import setup as mvs
    P = problems.aniso9(6, 1e-2, 0.5)
    path = str(tmp_path / "one.bin")
    st = mvs.build_hierarchy(P.rowptr, P.col, P.val, path, problems.random_vectors(P.n, 2, 1),
                             mvs.SetupParams(nvec_max=3))
    assert st["nlevels"] == 1
    hh = mvamg.hier_read(path)
    try:
        nb = ctypes.c_size_t()
        assert lib.mvamg_arena_bytes(hh, 1, ctypes.byref(nb)) == mvamg.ERR_ARG
        assert "two levels" in mvamg.last_error()
    finally:
        mvamg.hier_host_free(hh)
