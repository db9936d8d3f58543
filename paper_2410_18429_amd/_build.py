"""Build the gfx950 shared library libwri.so in-tree with hipcc.

Usage: python -m paper_2410_18429_amd._build [-v]
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libwri.so")
SOURCES = ["kernels.hip", "capi.hip", "outer.hip", "fwi.hip", "resample.hip", "offgrid.hip", "probe.hip", "precond.hip"]
ARCH = os.environ.get("WRI_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared",
    f"--offload-arch={ARCH}",
    # bit-identical stencil arithmetic across tilings: no implicit FMA contraction
    "-ffp-contract=off",
    # no packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


# Host-sanitized variant for the CPU tests of the C ABI's host code
# (validation, planner, workspace layout, receiver column maps): AddressSanitizer
# and UndefinedBehaviorSanitizer on the host compilation only, device code as in
# the product build.  Loaded with the ASan runtime preloaded
# (tests/test_capi_host.py drives it in a subprocess).
LIB_HOSTSAN = os.path.join(PKG, "libwri_hostsan.so")
HOSTSAN_FLAGS = [
    "-Xarch_host", "-fsanitize=address",
    "-Xarch_host", "-fsanitize=undefined",
    "-Xarch_host", "-fno-sanitize-recover=undefined",
    "-Xarch_host", "-fno-omit-frame-pointer",
    "-Xarch_host", "-g",
]


def build(verbose: bool = False, host_sanitized: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    out_lib = LIB_HOSTSAN if host_sanitized else LIB
    tmp = out_lib + ".tmp"
    cmd = [hipcc, *FLAGS, *(HOSTSAN_FLAGS if host_sanitized else []), *srcs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    proc = subprocess.run(cmd, capture_output=True, text=True)
    out = "\n".join(l for l in (proc.stdout + proc.stderr).splitlines()
                    if "packed-fp32-ops" not in l and l.strip())
    if proc.returncode != 0:
        raise RuntimeError(f"hipcc failed ({proc.returncode}):\n{out}")
    if verbose and out:
        print(out)
    os.replace(tmp, out_lib)
    return out_lib


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, host_sanitized="--host-sanitized" in sys.argv))
