"""Build the native parts of the package in-tree.

* ``libmvamg.so``   -- the HIP library (C ABI declared in include/mvamg.h),
  compiled by hipcc for gfx950 only.
* ``setup/libmvsetup.so`` -- the host setup generator (g++ with OpenMP).
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

HIP_SOURCES = ["csrc/mvamg_lib.hip"]
HIP_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # vector FP32 code is compiled without packed-FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-fno-gpu-rdc", "-Wall", "-Wno-unused-result",
]


def _run(cmd, cwd=None):
    print("+", " ".join(cmd), flush=True)
    r = subprocess.run(cmd, cwd=cwd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        sys.stdout.write(r.stdout)
        raise RuntimeError(f"build step failed ({r.returncode}): {' '.join(cmd)}")
    # hipcc's host pass warns about the device-only target feature; keep real warnings visible
    out = "\n".join(l for l in r.stdout.splitlines() if "packed-fp32-ops" not in l and l.strip())
    if out:
        print(out)


def build_setup() -> str:
    src = os.path.join(PKG, "setup", "mvsetup.cpp")
    out = os.path.join(PKG, "setup", "libmvsetup.so")
    _run(["g++", "-O3", "-std=c++17", "-fopenmp", "-fPIC", "-shared", "-Wall", src, "-o", out + ".tmp"])
    os.replace(out + ".tmp", out)
    return out


def build_hip() -> str:
    out = os.path.join(PKG, "libmvamg.so")
    srcs = [os.path.join(PKG, s) for s in HIP_SOURCES]
    _run([HIPCC, *HIP_FLAGS, "-I", os.path.join(ROOT, "include"), *srcs, "-o", out + ".tmp"])
    os.replace(out + ".tmp", out)
    return out


def build_all() -> None:
    build_setup()
    build_hip()


if __name__ == "__main__":
    which = sys.argv[1:] or ["all"]
    for w in which:
        {"setup": build_setup, "hip": build_hip, "all": build_all}[w]()
