"""Build the HIP library libadm1.so for gfx950 (in-tree).

Runs the Newton-matrix code generator, then one hipcc line over the HIP
sources.  All HIP code is compiled with packed-FP32 instructions disabled.
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(os.path.dirname(PKG), "include")
LIB = os.path.join(PKG, "libadm1.so")
ARCH = os.environ.get("ADM1_OFFLOAD_ARCH", "gfx950")
SOURCES = ["adm1_abi.hip", "adm1_kernels.hip", "adm1_step_sparse2.hip", "adm1_order.hip",
           "adm1_transport.hip", "adm1_mlp.hip", "adm1_surrogate.hip",
           "adm1_diffusion.hip", "adm1_snapshot.cpp"]


def hipcc() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    return os.path.join(rocm, "bin", "hipcc")


def build(verbose: bool = False) -> str:
    subprocess.check_call([sys.executable, os.path.join(CSRC, "gen_jac.py")])
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "-O3", "-std=c++17", "-fPIC", "-shared", f"--offload-arch={ARCH}",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-munsafe-fp-atomics", "-Wall", "-Wno-unused-function",
           f"-I{INCLUDE}", f"-I{CSRC}", "-o", tmp] + [os.path.join(CSRC, s) for s in SOURCES]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
