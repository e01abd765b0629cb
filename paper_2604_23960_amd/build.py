"""Build libmrv.so (HIP, gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libmrv.so")
KERNELS = "mrv_kernels.hip"
HOST_SOURCES = ["mrv_host.cpp", "mrv_serve.cpp", "mrv_arena.cpp"]
SOURCES = [KERNELS, *HOST_SOURCES]
HEADERS = ["mrv_internal.hpp", "mrv_runtime.hpp", "mrv_tiles.hpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"


def _common() -> list[str]:
    return [HIPCC, f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
            # no packed FP32 instructions in any kernel
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wno-unused-command-line-argument", "-I", os.path.join(ROOT, "include")]


def commands(out: str) -> list[list[str]]:
    """Kernels compiled on their own, assuming no NaN (every floating-point value
    they read is checked finite and within MRV_MAX_COORD before any kernel uses
    it), so minima of matrix-core results need no NaN quieting; then the host
    code, without that assumption, linked into one library."""
    obj = out + ".kernels.o"
    return [[*_common(), "-fno-honor-nans", "-c", os.path.join(CSRC, KERNELS), "-o", obj],
            [*_common(), "-shared", "-o", out, obj, *[os.path.join(CSRC, s) for s in HOST_SOURCES], "-lpthread"]]


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    for cmd in commands(tmp):
        if verbose:
            print(" ".join(cmd), flush=True)
        res = subprocess.run(cmd, capture_output=True, text=True)
        if res.returncode != 0:
            sys.stderr.write(res.stdout + res.stderr)
            raise RuntimeError("hipcc failed building libmrv.so")
        warn = [ln for ln in res.stderr.splitlines() if "packed-fp32-ops" not in ln and ln.strip()]
        if verbose and warn:
            sys.stderr.write("\n".join(warn) + "\n")
    os.remove(tmp + ".kernels.o")
    os.replace(tmp, LIB)
    return LIB


def stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    deps = [os.path.join(CSRC, s) for s in SOURCES + HEADERS] + [os.path.join(ROOT, "include", "mrv.h")]
    return any(os.path.getmtime(d) > t for d in deps)


if __name__ == "__main__":
    print(build(verbose=True))
