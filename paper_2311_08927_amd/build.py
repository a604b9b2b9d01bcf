"""Build the HIP library for gfx950 (in-tree).

Runs the Newton-matrix code generator over a model description, then one
hipcc line over the HIP sources.  All HIP code is compiled with packed-FP32
instructions disabled.  The standard ADM1 description generates into csrc/
and builds libadm1.so; another description generates into
_build/<model>/ (searched first for the generated includes) and builds
lib<model>.so beside it (model names start with "adm1_").
"""
from __future__ import annotations

import json
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
DATA = os.path.join(PKG, "data")
INCLUDE = os.path.join(os.path.dirname(PKG), "include")
LIB = os.path.join(PKG, "libadm1.so")
STANDARD_MODEL = os.path.join(DATA, "adm1_petersen.json")
# model descriptions built by default besides the standard one
VARIANT_MODELS = [os.path.join(DATA, "adm1_petersen_decay_to_particulates.json")]
ARCH = os.environ.get("ADM1_OFFLOAD_ARCH", "gfx950")
SOURCES = ["adm1_abi.hip", "adm1_kernels.hip", "adm1_step_sparse2.hip", "adm1_order.hip",
           "adm1_transport.hip", "adm1_mlp.hip", "adm1_surrogate.hip",
           "adm1_diffusion.hip", "adm1_train.hip", "adm1_snapshot.cpp"]


def hipcc() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    return os.path.join(rocm, "bin", "hipcc")


def model_name(path: str) -> str:
    with open(path) as fh:
        return json.load(fh)["model"]


def lib_path(name: str | None = None) -> str:
    """The library of a model description by its name (None: standard)."""
    if name is None or name == model_name(STANDARD_MODEL):
        return LIB
    return os.path.join(PKG, f"lib{name}.so")


def build(verbose: bool = False, model: str | None = None) -> str:
    model = model or STANDARD_MODEL
    name = model_name(model)
    standard = name == model_name(STANDARD_MODEL)
    gen = CSRC if standard else os.path.join(PKG, "_build", name)
    os.makedirs(gen, exist_ok=True)
    subprocess.check_call([sys.executable, os.path.join(CSRC, "gen_jac.py"), "--model", model,
                           "--out", gen])
    out = lib_path(name)
    tmp = out + ".tmp"
    cmd = [hipcc(), "-O3", "-std=c++17", "-fPIC", "-shared", f"--offload-arch={ARCH}",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-munsafe-fp-atomics", "-Wall", "-Wno-unused-function",
           f"-I{INCLUDE}", f"-I{gen}", f"-I{CSRC}", "-o", tmp] + \
        [os.path.join(CSRC, s) for s in SOURCES]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    return out


LU_BENCH_DIR = os.path.join(PKG, "_build", "lu_bench")
LU_BENCH = os.path.join(LU_BENCH_DIR, "lu_group_bench")


def build_lu_bench(verbose: bool = False) -> str:
    """The lanes-per-particle measurement of the sparse LU (a standalone
    program, csrc/lu_group_bench.hip; run it with [particles] [repeats])."""
    subprocess.check_call([sys.executable, os.path.join(CSRC, "gen_lu_groups.py"), "--out",
                           LU_BENCH_DIR])
    tmp = LU_BENCH + ".tmp"
    cmd = [hipcc(), "-O3", "-std=c++17", f"--offload-arch={ARCH}",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wall",
           f"-I{LU_BENCH_DIR}", "-o", tmp, os.path.join(CSRC, "lu_group_bench.hip")]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(tmp, LU_BENCH)
    return LU_BENCH


def build_all(verbose: bool = False) -> list[str]:
    return [build(verbose)] + [build(verbose, m) for m in VARIANT_MODELS] + \
        [build_lu_bench(verbose)]


if __name__ == "__main__":
    import argparse
    ap = argparse.ArgumentParser()
    ap.add_argument("--model", default=None, help="model description (default: standard)")
    ap.add_argument("--all", action="store_true",
                    help="standard and variant descriptions, and the LU lanes measurement")
    ap.add_argument("--lu-bench", action="store_true", help="only the LU lanes measurement")
    a = ap.parse_args()
    if a.lu_bench:
        print(build_lu_bench(True))
    else:
        print(build_all(True) if a.all else build(True, a.model))
