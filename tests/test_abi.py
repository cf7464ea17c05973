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
