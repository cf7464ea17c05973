"""Reader of the hierarchy file, written independently of the GPU library's
parser.  The file is a sequence of named little-endian arrays:

    magic "MVAMGH01", uint32 version, uint32 nchunks,
    per chunk: char name[48], uint32 dtype (1 int32, 2 float64, 3 int64),
               uint32 reserved, uint64 count, data, zero padding to 8 bytes.

Chunks: meta (int64: version, nlevels, nvec, n, nnz, nstages, stage used),
params, stats, rho; per level l: A{l}.rowptr/.col/.val (CSR of A^l),
W{l} (projected smooth vectors, row-major n_l x nvec); on a non-coarsest
level the Gauss-Seidel order: A{l}.order (the rows in relaxation order),
A{l}.gptr (groups: runs of `order`), A{l}.sptr (stages: runs of groups whose
rows are mutually uncoupled); per transfer l -> l+1: P{l}.aptr/.arows
(aggregate members), P{l}.coff (coarse offsets, k_a = coff[a+1] - coff[a]),
P{l}.uoff (offset of U_a), P{l}.U (U_a row-major n_a x k_a), P{l}.drop2
(sum of the squared dropped singular values).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

_DT = {1: np.int32, 2: np.float64, 3: np.int64}


def read_chunks(path: str) -> dict:
    with open(path, "rb") as f:
        buf = f.read()
    if buf[:8] != b"MVAMGH01":
        raise ValueError("not a hierarchy file (bad magic)")
    ver, nch = np.frombuffer(buf, dtype="<u4", count=2, offset=8)
    if ver != 1:
        raise ValueError(f"unsupported hierarchy file version {ver}")
    off = 16
    out = {}
    for _ in range(int(nch)):
        if off + 64 > len(buf):
            raise ValueError("truncated hierarchy file")
        name = buf[off:off + 48].split(b"\0", 1)[0].decode()
        dtype, _res = np.frombuffer(buf, dtype="<u4", count=2, offset=off + 48)
        count = int(np.frombuffer(buf, dtype="<u8", count=1, offset=off + 56)[0])
        off += 64
        dt = np.dtype(_DT[int(dtype)]).newbyteorder("<")
        nbytes = count * dt.itemsize
        if off + nbytes > len(buf):
            raise ValueError("truncated hierarchy file")
        out[name] = np.frombuffer(buf, dtype=dt, count=count, offset=off).copy()
        off += nbytes + (-nbytes) % 8
    return out


@dataclass
class Level:
    n: int
    rowptr: np.ndarray
    col: np.ndarray
    val: np.ndarray
    order: np.ndarray | None = None
    gptr: np.ndarray | None = None
    sptr: np.ndarray | None = None
    W: np.ndarray | None = None


@dataclass
class Transfer:
    aptr: np.ndarray
    arows: np.ndarray
    coff: np.ndarray
    uoff: np.ndarray
    U: np.ndarray
    drop2: np.ndarray

    @property
    def nagg(self) -> int:
        return int(self.aptr.shape[0] - 1)


@dataclass
class Hierarchy:
    levels: list
    transfers: list
    nvec: int
    rho: np.ndarray
    meta: np.ndarray
    params: np.ndarray = field(default=None)

    @property
    def nlevels(self) -> int:
        return len(self.levels)


def read_hierarchy(path: str) -> Hierarchy:
    c = read_chunks(path)
    meta = c["meta"]
    nl, nvec = int(meta[1]), int(meta[2])
    levels, transfers = [], []
    for l in range(nl):
        rp = c[f"A{l}.rowptr"]
        lev = Level(int(rp.shape[0] - 1), rp, c[f"A{l}.col"], c[f"A{l}.val"])
        if f"W{l}" in c:
            lev.W = c[f"W{l}"].reshape(lev.n, nvec)
        if l + 1 < nl:
            lev.order = c[f"A{l}.order"]
            lev.gptr = c[f"A{l}.gptr"]
            lev.sptr = c[f"A{l}.sptr"]
            transfers.append(Transfer(c[f"P{l}.aptr"], c[f"P{l}.arows"], c[f"P{l}.coff"],
                                      c[f"P{l}.uoff"], c[f"P{l}.U"], c[f"P{l}.drop2"]))
        levels.append(lev)
    return Hierarchy(levels, transfers, nvec, c.get("rho", np.zeros(0)), meta, c.get("params"))
