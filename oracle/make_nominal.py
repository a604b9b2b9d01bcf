"""Write the nominal digester state and feed used to seed every workload.

Calls only the oracle.  The nominal state is the CSTR steady state of the
Case-1 reactor of the paper (Table 1: 3400 m3 liquid, 300 m3 gas,
178.45 m3/d in/out, 1.013 bar) at 35 C under a feed chosen for this code (the
BSM2 inflow the paper used is not available): particulates X_xc 20, X_ch 8,
X_pr 8, X_li 6, X_I 4; solubles S_I 1, S_su 1, S_aa 1, S_fa 1, each VFA 0.2
kg COD/m3; every biomass 0.05 kg COD/m3; S_IC 0.05, S_IN 0.02, S_an 0.02
kmol/m3; S_cat 0.04 kmol/m3, which puts the steady-state pH in 7.0-7.6.

The steady state is reached by integrating 200 days (about ten hydraulic
retention times) from a healthy start and then polishing f(x) = 0 with Newton
steps on the oracle's Jacobian.

Usage: python oracle/make_nominal.py   (rewrites the nominal data file)
"""
from __future__ import annotations

import json
import os
import sys

import numpy as np

sys.path[0] = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
from oracle.adm1 import DIFF, NLIQ, NX, Oracle  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "paper_2311_08927_amd", "data", "nominal.json")

NAMES = ["S_su", "S_aa", "S_fa", "S_va", "S_bu", "S_pro", "S_ac", "S_h2", "S_ch4", "S_IC",
         "S_IN", "S_I", "X_xc", "X_ch", "X_pr", "X_li", "X_su", "X_aa", "X_fa", "X_c4",
         "X_pro", "X_ac", "X_h2", "X_I", "S_cat", "S_an", "S_va_ion", "S_bu_ion",
         "S_pro_ion", "S_ac_ion", "S_hco3_ion", "S_nh3", "G_h2", "G_ch4", "G_co2"]

V_LIQ, V_GAS, Q = 3400.0, 300.0, 178.45
T_NOM = 308.15
S_CAT_FEED = 0.04


def nominal_feed() -> np.ndarray:
    feed = np.zeros(NLIQ)
    ix = {n: i for i, n in enumerate(NAMES)}
    vals = dict(X_xc=20, X_ch=8, X_pr=8, X_li=6, X_I=4, S_I=1, S_su=1, S_aa=1, S_fa=1,
                S_va=0.2, S_bu=0.2, S_pro=0.2, S_ac=0.2, S_IC=0.05, S_IN=0.02, S_an=0.02,
                S_cat=S_CAT_FEED)
    for n in ["X_su", "X_aa", "X_fa", "X_c4", "X_pro", "X_ac", "X_h2"]:
        vals[n] = 0.05
    for n, v in vals.items():
        feed[ix[n]] = v
    return feed


def healthy_start() -> np.ndarray:
    x = np.zeros(NX)
    ix = {n: i for i, n in enumerate(NAMES)}
    init = dict(S_su=0.01, S_aa=0.005, S_fa=0.1, S_va=0.01, S_bu=0.01, S_pro=0.02,
                S_ac=0.05, S_h2=2e-7, S_ch4=0.05, S_IC=0.1, S_IN=0.1, S_I=1, X_xc=2,
                X_ch=0.05, X_pr=0.05, X_li=0.05, X_su=1.0, X_aa=0.8, X_fa=0.3, X_c4=0.3,
                X_pro=0.1, X_ac=0.9, X_h2=0.4, X_I=10, S_cat=S_CAT_FEED, S_an=0.02,
                G_h2=1e-5, G_ch4=1.6, G_co2=0.014)
    for n, v in init.items():
        x[ix[n]] = v
    return x


def steady_state(o: Oracle, feed: np.ndarray, D: float, T: float):
    X = healthy_start().reshape(NX, 1).copy()
    H = np.array([-1.0])
    hl = np.array([-1.0])
    for _ in range(200):
        st, _ = o.step(X, [T], [D], [0], feed[None, :], 1.0, H=H, hlast=hl, nthreads=1)
        if st[0] & 0x7F:
            raise RuntimeError(f"integration failed: status {st[0]}")
    x = X[:, 0].copy()
    # Newton polish of f(y) = 0 in the 28 differential entries
    for _ in range(8):
        f, xa, _ = o.rhs(x, T, D, feed)
        J = o.jacobian(x, T, D, feed)
        dy = np.linalg.solve(J, -f)
        y = x[DIFF] + dy
        x[DIFF] = y
        if np.max(np.abs(dy) / np.maximum(np.abs(y), 1e-12)) < 1e-15:
            break
    f, xa, H = o.rhs(x, T, D, feed)
    return xa, f, H


def main():
    o = Oracle(rtol=1e-10)
    feed = nominal_feed()
    D = Q / V_LIQ
    x, f, H = steady_state(o, feed, D, T_NOM)
    assert np.all(x > 0.0), "nominal state must be positive"
    pH = -np.log10(H)
    assert 7.0 <= pH <= 7.6, pH
    doc = {
        "_about": "Nominal ADM1 state: CSTR steady state of the Case-1 reactor (paper "
                  "Table 1) at 308.15 K under the feed below, written by "
                  "oracle/make_nominal.py from the oracle alone.",
        "names": NAMES,
        "state": [float(v) for v in x],
        "feed": [float(v) for v in feed],
        "S_H": float(H),
        "pH": float(pH),
        "D": D,
        "T": T_NOM,
        "V_liq": V_LIQ,
        "V_gas": V_GAS,
        "max_abs_f": float(np.max(np.abs(f))),
    }
    with open(OUT, "w") as fh:
        json.dump(doc, fh, indent=1)
    print(f"pH {pH:.4f}  max|f| {np.max(np.abs(f)):.3e}  -> {OUT}")


if __name__ == "__main__":
    main()
