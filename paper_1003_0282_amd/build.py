"""Build step of the HIP library: ``liblbaxi.so`` for gfx950, in-tree.

    python -m paper_1003_0282_amd.build

Every call compiles (the build check must exercise the compiler even when a
library is already present).  Packed FP32 instructions are disabled for all
device code.
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
SRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "liblbaxi.so")
NNLIB = os.path.join(PKG, "liblbnn.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("LBAXI_ARCH", "gfx950")

COMMON = ["-O3", "--offload-arch=" + ARCH, "-std=c++17", "-fPIC",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I" + os.path.join(ROOT, "include")]


def _compile(out: str, sources: list[str], extra: list[str] | None = None) -> str:
    tmp = out + ".tmp%d" % os.getpid()
    cmd = [HIPCC] + COMMON + ["-shared", "-o", tmp] + sources + (extra or [])
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed for %s" % out)
    os.replace(tmp, out)
    return out


def build() -> list[str]:
    libs = [_compile(LIB, [os.path.join(SRC, "lbaxi.hip")]),
            _compile(NNLIB, [os.path.join(SRC, "lbnn.hip")])]
    return libs


if __name__ == "__main__":
    for p in build():
        print(p)
