"""Build the HIP library libpfc.so for gfx950 in-tree (hipcc, no JIT)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpfc.so")
SOURCES = ["mesh.hip", "solver.hip", "server.hip", "tune.hip"]
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # packed FP32 arithmetic off for all device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


# the instrumented build for phase_probe.py: wall-clock stamps of each solver launch (PFC_TICK_TIMING)
LIB_TIMING = os.path.join(HERE, "libpfc_timing.so")


def build(verbose: bool = False, timing: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    srcs = [os.path.join(CSRC, s) for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    lib = LIB_TIMING if timing else LIB
    tmp = lib + ".tmp"
    extra = ["-DPFC_TICK_TIMING"] if timing else []
    cmd = [hipcc, *FLAGS, *extra, "-I", os.path.join(HERE, "..", "include"), "-o", tmp, *srcs, "-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    out = "\n".join(l for l in (res.stdout + res.stderr).splitlines() if "packed-fp32-ops" not in l)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + out)
    if verbose and out.strip():
        print(out)
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, timing="--timing" in sys.argv))
