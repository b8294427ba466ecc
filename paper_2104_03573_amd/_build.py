"""Build step of the HIP library: one hipcc invocation -> paper_2104_03573_amd/libmcbte.so."""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libmcbte.so")
SOURCES = [os.path.join(CSRC, "mcbte_host.cpp"), os.path.join(CSRC, "mcbte_kernels.hip")]
HEADERS = [os.path.join(ROOT, "include", "mcbte.h"), os.path.join(CSRC, "mcbte_dev.h")]
ARCH = "gfx950"


def hipcc() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    return os.path.join(rocm, "bin", "hipcc")


def command(out: str = LIB) -> list[str]:
    return [hipcc(), f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
            # every step rounds as written (the FP64 form reproduces the method's event sequence)
            "-ffp-contract=off",
            # hardware FP64 atomic add for tally sums (ds_add_f64 / global_atomic_add_f64)
            "-munsafe-fp-atomics",
            # no packed FP32 instructions
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", os.path.join(ROOT, "include"), "-I", CSRC, *SOURCES, "-o", out]


def build(verbose: bool = False) -> str:
    """Compile the library for gfx950 (always recompiles)."""
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = command(tmp)
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed to build libmcbte.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
