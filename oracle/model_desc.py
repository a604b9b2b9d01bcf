"""The oracle's reader of a model description (Petersen matrix as data).

TEST INFRASTRUCTURE ONLY.  A model description (JSON) lists, per biochemical
process of sec. 2.2, its rate form and its stoichiometric coefficients as
arithmetic expressions of the named parameters (the matrix of eq. 2); the
inorganic carbon and nitrogen rows are closures over carbon and nitrogen
contents that the description also lists.  This module evaluates such a
description with its own small expression parser into the numeric matrix
and content vectors the oracle integrates with; it shares nothing with the
kernel generator that reads the same files.

The oracle's rates (eqs. 3-6 and the uptake / decay forms) are hand-written
in adm1_oracle.c, so a description may change the matrix but not the rate
forms: `check_rates` refuses one whose rate forms differ from those.
"""
from __future__ import annotations

import json
import re

import numpy as np

NLIQ, NPROC = 26, 19

# liquid entries in the oracle's state order
LIQUID = ["S_su", "S_aa", "S_fa", "S_va", "S_bu", "S_pro", "S_ac", "S_h2", "S_ch4", "S_IC",
          "S_IN", "S_I", "X_xc", "X_ch", "X_pr", "X_li", "X_su", "X_aa", "X_fa", "X_c4",
          "X_pro", "X_ac", "X_h2", "X_I", "S_cat", "S_an"]

# The rate of each process as rates() in adm1_oracle.c writes it: form,
# rate constant, the entry it is first order in (or substrate, competitor,
# biomass), and the inhibition factors it multiplies in.
ORACLE_RATES = [
    ("dis", "first_order", "k_dis", "X_xc"),
    ("hch", "first_order", "k_hyd_ch", "X_ch"),
    ("hpr", "first_order", "k_hyd_pr", "X_pr"),
    ("hli", "first_order", "k_hyd_li", "X_li"),
    ("su", "monod", "k_m_su", "K_S_su", "S_su", None, "X_su", ("I_pH_aa", "I_IN_lim")),
    ("aa", "monod", "k_m_aa", "K_S_aa", "S_aa", None, "X_aa", ("I_pH_aa", "I_IN_lim")),
    ("fa", "monod", "k_m_fa", "K_S_fa", "S_fa", None, "X_fa",
     ("I_pH_aa", "I_IN_lim", "I_h2_fa")),
    ("va", "monod_competing", "k_m_c4", "K_S_c4", "S_va", "S_bu", "X_c4",
     ("I_pH_aa", "I_IN_lim", "I_h2_c4")),
    ("bu", "monod_competing", "k_m_c4", "K_S_c4", "S_bu", "S_va", "X_c4",
     ("I_pH_aa", "I_IN_lim", "I_h2_c4")),
    ("pro", "monod", "k_m_pro", "K_S_pro", "S_pro", None, "X_pro",
     ("I_pH_aa", "I_IN_lim", "I_h2_pro")),
    ("ac", "monod", "k_m_ac", "K_S_ac", "S_ac", None, "X_ac", ("I_pH_ac", "I_IN_lim", "I_nh3")),
    ("h2", "monod", "k_m_h2", "K_S_h2", "S_h2", None, "X_h2", ("I_pH_h2", "I_IN_lim")),
    ("dsu", "first_order", "k_dec_su", "X_su"),
    ("daa", "first_order", "k_dec_aa", "X_aa"),
    ("dfa", "first_order", "k_dec_fa", "X_fa"),
    ("dc4", "first_order", "k_dec_c4", "X_c4"),
    ("dpro", "first_order", "k_dec_pro", "X_pro"),
    ("dac", "first_order", "k_dec_ac", "X_ac"),
    ("dh2", "first_order", "k_dec_h2", "X_h2"),
]


def _rate_key(rate: dict) -> tuple:
    if rate["form"] == "first_order":
        return (rate["form"], rate["k"], rate["state"])
    return (rate["form"], rate["k"], rate["K"], rate["substrate"], rate.get("competitor"),
            rate["biomass"], tuple(rate.get("factors", ())))


def check_rates(desc: dict) -> None:
    """Raise ValueError unless the description's processes are the oracle's,
    in its order and with its rate forms."""
    procs = desc["processes"]
    if len(procs) != NPROC:
        raise ValueError(f"{len(procs)} processes, the oracle has {NPROC}")
    for j, (p, mine) in enumerate(zip(procs, ORACLE_RATES)):
        if p["name"] != mine[0]:
            raise ValueError(f"process {j} is {p['name']!r}, the oracle's is {mine[0]!r}")
        if _rate_key(p["rate"]) != tuple(mine[1:]):
            raise ValueError(f"process {p['name']!r}: rate form differs from the oracle's")


# -- expressions: numbers, parameter names, + - * / and parentheses ---------
_TOKEN = re.compile(r"\s*(?:(\d+\.\d*(?:[eE][-+]?\d+)?|\d*\.\d+(?:[eE][-+]?\d+)?|\d+(?:[eE][-+]?\d+)?)"
                    r"|([A-Za-z_][A-Za-z_0-9]*)|(.))")


def _tokens(text: str) -> list:
    out = []
    pos = 0
    text = text.strip()
    while pos < len(text):
        m = _TOKEN.match(text, pos)
        if m is None:
            break
        num, name, op = m.groups()
        if num is not None:
            out.append(("num", float(num)))
        elif name is not None:
            out.append(("name", name))
        elif op is not None and op.strip():
            if op not in "+-*/()":
                raise ValueError(f"unexpected {op!r} in {text!r}")
            out.append(("op", op))
        pos = m.end()
    return out


def evaluate(text: str, values: dict) -> float:
    """Value of an expression; grammar (usual precedence, left to right):
    sum := product (('+'|'-') product)*; product := unary (('*'|'/') unary)*;
    unary := '-' unary | '(' sum ')' | number | name."""
    toks = _tokens(text)
    k = 0

    def peek():
        return toks[k] if k < len(toks) else ("end", None)

    def take():
        nonlocal k
        tok = peek()
        k += 1
        return tok

    def unary():
        kind, v = take()
        if kind == "op" and v == "-":
            return -unary()
        if kind == "op" and v == "(":
            s = total()
            if take() != ("op", ")"):
                raise ValueError(f"unbalanced parentheses in {text!r}")
            return s
        if kind == "num":
            return v
        if kind == "name":
            if v not in values:
                raise ValueError(f"unknown parameter {v!r} in {text!r}")
            return float(values[v])
        raise ValueError(f"malformed expression {text!r}")

    def product():
        a = unary()
        while peek() in (("op", "*"), ("op", "/")):
            op = take()[1]
            b = unary()
            a = a * b if op == "*" else a / b
        return a

    def total():
        a = product()
        while peek() in (("op", "+"), ("op", "-")):
            op = take()[1]
            b = product()
            a = a + b if op == "+" else a - b
        return a

    val = total()
    if k != len(toks):
        raise ValueError(f"trailing input in {text!r}")
    return val


def load(path: str) -> dict:
    with open(path) as fh:
        return json.load(fh)


def tables(desc: dict, values: dict):
    """(nu[26][19], C[26], N[26]) of a description under a parameter set.  The
    rows the description closes (S_IC, S_IN) are left zero here: the oracle's
    closure fills them from C and N."""
    check_rates(desc)
    if desc.get("closures") != {"S_IC": "carbon", "S_IN": "nitrogen"}:
        raise ValueError("the oracle closes S_IC over carbon and S_IN over nitrogen")
    if desc.get("transfers") != {"S_h2": "T8", "S_ch4": "T9", "S_IC": "T10"}:
        raise ValueError("the oracle's gas transfers are T8 (S_h2), T9 (S_ch4), T10 (S_IC)")
    row = {name: i for i, name in enumerate(LIQUID)}
    nu = np.zeros((NLIQ, NPROC))
    for j, p in enumerate(desc["processes"]):
        for entry, expr in p["stoich"].items():
            if entry in ("S_IC", "S_IN"):
                raise ValueError(f"process {p['name']!r} sets the closed row {entry}")
            nu[row[entry], j] = evaluate(expr, values)
    C = np.zeros(NLIQ)
    N = np.zeros(NLIQ)
    for vec, key in ((C, "carbon"), (N, "nitrogen")):
        for entry, expr in desc["contents"][key].items():
            vec[row[entry]] = evaluate(expr, values)
    return nu, C, N
