"""Builds the HIP library libwenomhd.so for gfx950 in-tree with hipcc.

Usage: ``python -m paper_1812_04278_amd.build [--verbose] [--clock]``; ``--clock``
builds the phase-clock measurement library libwenomhd_clock.so instead.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libwenomhd.so")
# measurement build with per-wave phase stamps in the sweep (include/wenomhd_clock.h)
CLOCK_LIB = os.path.join(HERE, "libwenomhd_clock.so")
SOURCES = [os.path.join(CSRC, "wenomhd.hip")]
HEADERS = [os.path.join(CSRC, f) for f in ("kernels.hpp", "mhd_device.hpp", "adjoint_device.hpp", "adjoint_kernels.hpp")] + [
    os.path.join(os.path.dirname(HERE), "include", "wenomhd.h"),
    os.path.join(os.path.dirname(HERE), "include", "wenomhd_clock.h")]

# Packed FP32 instructions are disabled for all device code; FMA contraction
# stays on (the default for HIP device code).
HIPCC_FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found (ROCm toolchain required to build libwenomhd.so)")


def build(verbose: bool = False, extra=(), clock: bool = False) -> str:
    """Builds libwenomhd.so, or with clock=True the phase-clock build."""
    out = CLOCK_LIB if clock else LIB
    tmp = out + ".tmp"
    cmd = [hipcc(), *HIPCC_FLAGS, *(["-DWM_SWEEP_CLOCK"] if clock else []), *extra, "-o", tmp, *SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed with code {r.returncode}")
    if verbose and (r.stdout or r.stderr):
        sys.stderr.write(r.stdout + r.stderr)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose="--verbose" in sys.argv,
                extra=["-Rpass-analysis=kernel-resource-usage"] if "--resources" in sys.argv else [],
                clock="--clock" in sys.argv))
