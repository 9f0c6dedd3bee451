"""Build libmxr.so in-tree with hipcc for gfx950."""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
SOURCES = [os.path.join(PKG, "csrc", n) for n in ("mxr.hip", "mlp.hip", "stats.hip", "peaks.hip")]
HEADERS = [os.path.join(ROOT, "include", "mxr.h"), os.path.join(PKG, "csrc", "mxr_device.h")]
LIB = os.path.join(PKG, "libmxr.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # every expression rounds as written; FMA only where the source says so
    "-ffp-contract=off",
    # FP64 atomic adds compile to the hardware global_atomic_add_f64
    "-munsafe-fp-atomics",
    # no packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # keep loop-invariant constants (exp/sin/cos coefficients) where they are
    # used instead of hoisting them into registers for the whole kernel
    "-mllvm", "-disable-machine-licm",
    "-Wno-unused-command-line-argument",
]


def build(verbose: bool = False) -> str:
    cmd = [HIPCC, *FLAGS, "-I", os.path.join(ROOT, "include"), "-o", LIB + ".tmp", *SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(p) > t for p in SOURCES + HEADERS)


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
