"""Operation counts of the oracle's right-hand side (measurement helper).

TEST/MEASUREMENT INFRASTRUCTURE ONLY.  Builds count_ops.cpp (the oracle's C
source compiled unchanged with a counting scalar type) and counts, per part
of one right-hand-side evaluation, the adds, multiplies, divides and the
exp / log / pow / sqrt calls at a few seeded states: the counted figures
behind the flop model of the step (rates and transfers, the eq.-2 assembly,
one eq.-7 residual with its derivative, one eq.-8 residual with its
derivative in the oracle's form, the ion write-back).

Run: python -m oracle.count_flops   (writes oracle/flop_counts.json)
"""
from __future__ import annotations

import ctypes
import json
import os
import subprocess

import numpy as np

from oracle.adm1 import Oracle

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "count_ops.cpp")
LIB = os.path.join(HERE, "libcount_ops.so")
OUT = os.path.join(HERE, "flop_counts.json")
PARTS = ["tconst", "rates", "assembly", "eq7_eval", "eq8_eval_oracle_form", "ions",
         "rhs_with_bracketed_solves"]
TALLIES = ["add", "mul", "div", "exp", "log", "pow", "sqrt"]


def build(force: bool = False) -> str:
    deps = [SRC, os.path.join(HERE, "adm1_oracle.c")]
    if force or not os.path.exists(LIB) or \
            os.path.getmtime(LIB) < max(os.path.getmtime(d) for d in deps):
        tmp = LIB + ".tmp"
        subprocess.check_call(["g++", "-O1", "-std=c++17", "-fPIC", "-shared", "-o", tmp, SRC,
                               "-lpthread"])
        os.replace(tmp, LIB)
    return LIB


def count(orc: Oracle, x, T, D, s_in) -> dict:
    L = ctypes.CDLL(build())
    L.orc_count_rhs.restype = ctypes.c_int
    L.orc_count_rhs.argtypes = [ctypes.c_void_p] * 3 + [ctypes.c_double] * 2 + \
        [ctypes.c_void_p] * 3
    x = np.ascontiguousarray(x, dtype=np.float64)
    s_in = np.ascontiguousarray(s_in, dtype=np.float64)
    out = np.zeros(7 * len(PARTS))
    it = ctypes.c_int(0)
    rc = L.orc_count_rhs(ctypes.byref(orc._p), ctypes.byref(orc._o), x.ctypes.data, T, D,
                         s_in.ctypes.data, out.ctypes.data, ctypes.byref(it))
    if rc != 0:
        raise RuntimeError("counting run failed")
    res = {p: {t: int(out[7 * k + j]) for j, t in enumerate(TALLIES)}
           for k, p in enumerate(PARTS)}
    for p in PARTS:
        res[p]["total"] = sum(res[p][t] for t in TALLIES)
    res["newton_iterations_of_that_rhs"] = int(it.value)
    return res


def states():
    """The nominal state (open reactor and closed particle) and two seeded
    perturbed states of the CSTR population."""
    from paper_2311_08927_amd import workloads as W  # input generators only
    nom = W.nominal()
    w = W.cstr_population(4, seed=3)
    return [("nominal, D = 178.45/3400", nom["state"], nom["T"], nom["D"], nom["feed"]),
            ("nominal, closed (D = 0)", nom["state"], nom["T"], 0.0, nom["feed"]),
            ("perturbed #1", w.X[:, 1], w.T[1], w.D[1], w.feed[w.fidx[1]]),
            ("perturbed #2", w.X[:, 2], w.T[2], w.D[2], w.feed[w.fidx[2]])]


def main():
    from paper_2311_08927_amd import workloads as W  # input generators only
    orc = Oracle(W.params_path())
    rows = []
    for label, x, T, D, s in states():
        c = count(orc, x, T, D, s)
        c["state"] = label
        rows.append(c)
        print(label, {p: c[p]["total"] for p in PARTS})
    with open(OUT, "w") as fh:
        json.dump({"about": __doc__.splitlines()[0], "tallies": TALLIES, "parts": PARTS,
                   "states": rows}, fh, indent=1)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
