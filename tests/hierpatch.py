"""Test helper: read and rewrite the values of one chunk of a hierarchy file
in place (same length), to build invalid inputs for the error-path tests."""
import struct

import numpy as np

_DT = {1: np.int32, 2: np.float64, 3: np.int64}


def chunks(buf: bytes) -> dict:
    """name -> (dtype code, count, byte offset of the data)."""
    assert buf[:8] == b"MVAMGH01"
    nch = struct.unpack_from("<I", buf, 12)[0]
    out, off = {}, 16
    for _ in range(nch):
        name = buf[off:off + 48].split(b"\0", 1)[0].decode()
        dtype = struct.unpack_from("<I", buf, off + 48)[0]
        count = struct.unpack_from("<Q", buf, off + 56)[0]
        off += 64
        out[name] = (dtype, count, off)
        size = np.dtype(_DT[dtype]).itemsize * count
        off += size + (8 - size % 8) % 8
    return out


def read_chunk(path: str, name: str) -> np.ndarray:
    buf = open(path, "rb").read()
    dtype, count, off = chunks(buf)[name]
    return np.frombuffer(buf, dtype=_DT[dtype], count=count, offset=off).copy()


def patched_copy(src: str, dst: str, name: str, fn) -> None:
    """Copy src to dst with chunk `name` replaced by fn(values) (same length and type)."""
    buf = bytearray(open(src, "rb").read())
    dtype, count, off = chunks(bytes(buf))[name]
    v = np.frombuffer(bytes(buf), dtype=_DT[dtype], count=count, offset=off).copy()
    w = np.ascontiguousarray(fn(v), dtype=_DT[dtype])
    assert w.shape == v.shape
    buf[off:off + w.nbytes] = w.tobytes()
    open(dst, "wb").write(bytes(buf))
