"""Generate the Newton-matrix code of the ADM1 Rosenbrock step.

The Rosenbrock stage equations need (alpha I - J) u = r with J the total
derivative of the 28 differential right-hand sides, the algebraic unknowns
z = (S_H+, S_h2) being eliminated through eq. 7 and eq. 8.  Instead of the
dense reduced J, the kernels solve the equivalent sparse bordered system

    [ alpha I - f_y   -f_z ] [u]   [r]
    [   g_y            g_z ] [w] = [0]

(f_y, f_z partial derivatives at fixed z; g the eq. 7 and eq. 8 residuals),
whose 30x30 pattern is fixed by the model structure.  This script holds that
structure and emits:

  adm1_jac_dense.inc  -- fills a dense row-major M[30*30] (one lane per
                         particle, partial pivoting);
  adm1_jac_sparse1.inc -- one lane per particle: the static-order sparse LU
                         in named registers (emit_sparse1);
  adm1_jac_sparse1_lds.inc -- the same LU with the matrix in LDS
                         (emit_sparse1_lds);
  adm1_jac_sparse2.inc -- the two-lanes-per-particle kernel body pieces: the
                         static-order sparse LU, with rows split over a lane
                         pair (see emit_sparse2).

The Petersen matrix (stoichiometry and rate forms) is read from a model
description, data/adm1_petersen.json by default (see load_model).

Run: python gen_jac.py [--model JSON] [--out DIR]   (writes the .inc files
next to this script, or into DIR)
"""
from __future__ import annotations

import os
import re
import sys

HERE = os.path.dirname(os.path.abspath(__file__))

Y = ["Ssu", "Saa", "Sfa", "Sva", "Sbu", "Spro", "Sac", "Sch4", "SIC", "SIN", "SI", "Xxc",
     "Xch", "Xpr", "Xli", "Xsu", "Xaa", "Xfa", "Xc4", "Xpro", "Xac", "Xh2", "XI", "Scat",
     "San", "Gh2", "Gch4", "Gco2"]
Z = ["H", "Sh2"]
VARS = Y + Z
NV = len(VARS)  # 30
LIQ = Y[:25]
GAS = Y[25:]

# rate -> variables it depends on (partials named J_<rate>_<var> in struct Partials)
RATES = {
    "dis": ["Xxc"], "hch": ["Xch"], "hpr": ["Xpr"], "hli": ["Xli"],
    "su": ["Ssu", "Xsu", "SIN", "H"],
    "aa": ["Saa", "Xaa", "SIN", "H"],
    "fa": ["Sfa", "Xfa", "SIN", "H", "Sh2"],
    "va": ["Sva", "Sbu", "Xc4", "SIN", "H", "Sh2"],
    "bu": ["Sva", "Sbu", "Xc4", "SIN", "H", "Sh2"],
    "pro": ["Spro", "Xpro", "SIN", "H", "Sh2"],
    "ac": ["Sac", "Xac", "SIN", "H"],
    "h2": ["Sh2", "Xh2", "SIN", "H"],
    "dsu": ["Xsu"], "daa": ["Xaa"], "dfa": ["Xfa"], "dc4": ["Xc4"], "dpro": ["Xpro"],
    "dac": ["Xac"], "dh2": ["Xh2"],
    "T8": ["Sh2", "Gh2"], "T9": ["Sch4", "Gch4"], "T10": ["SIC", "H", "Gco2"],
    "QGh2": ["Gh2", "Gch4", "Gco2"], "QGch4": ["Gh2", "Gch4", "Gco2"],
    "QGco2": ["Gh2", "Gch4", "Gco2"],
    "E7": ["Scat", "San", "SIN", "SIC", "Sac", "Spro", "Sbu", "Sva", "H"],
}
PROCS = ["dis", "hch", "hpr", "hli", "su", "aa", "fa", "va", "bu", "pro", "ac", "h2", "dsu",
         "daa", "dfa", "dc4", "dpro", "dac", "dh2"]

# ---------------------------------------------------------------------------
# The Petersen matrix comes from a model description (data/adm1_petersen.json
# by default): per process its rate form and its stoichiometric coefficients
# as expressions of the named parameters.  The rate forms must be the ones the
# kernel implements (KERNEL_RATES); the stoichiometry is free (any pattern
# that conserves COD): it sets the generated eq.-2 assembly, the eq.-8
# coefficients, the host-side derivation of the coefficients and the pattern
# of the Newton matrix.
# ---------------------------------------------------------------------------
DATA = os.path.join(os.path.dirname(HERE), "data")
DEFAULT_MODEL = os.path.join(DATA, "adm1_petersen.json")
# 35-entry state names and the kernel's names of the 28 integrated entries
STATE = ["S_su", "S_aa", "S_fa", "S_va", "S_bu", "S_pro", "S_ac", "S_h2", "S_ch4", "S_IC",
         "S_IN", "S_I", "X_xc", "X_ch", "X_pr", "X_li", "X_su", "X_aa", "X_fa", "X_c4",
         "X_pro", "X_ac", "X_h2", "X_I", "S_cat", "S_an"]
KNAME = {s: s.replace("_", "") for s in STATE}  # S_su -> Ssu (enum YIdx / gen names)
KNAME["S_h2"] = "Sh2"
_fo = lambda k, s: {"form": "first_order", "k": k, "state": s}  # noqa: E731


def _monod(k, K, S, X, f, comp=None):
    d = {"form": "monod" if comp is None else "monod_competing", "k": k, "K": K,
         "substrate": S, "biomass": X, "factors": f}
    if comp is not None:
        d["competitor"] = comp
    return d


KERNEL_RATES = {
    "dis": _fo("k_dis", "X_xc"), "hch": _fo("k_hyd_ch", "X_ch"),
    "hpr": _fo("k_hyd_pr", "X_pr"), "hli": _fo("k_hyd_li", "X_li"),
    "su": _monod("k_m_su", "K_S_su", "S_su", "X_su", ["I_pH_aa", "I_IN_lim"]),
    "aa": _monod("k_m_aa", "K_S_aa", "S_aa", "X_aa", ["I_pH_aa", "I_IN_lim"]),
    "fa": _monod("k_m_fa", "K_S_fa", "S_fa", "X_fa", ["I_pH_aa", "I_IN_lim", "I_h2_fa"]),
    "va": _monod("k_m_c4", "K_S_c4", "S_va", "X_c4", ["I_pH_aa", "I_IN_lim", "I_h2_c4"],
                 "S_bu"),
    "bu": _monod("k_m_c4", "K_S_c4", "S_bu", "X_c4", ["I_pH_aa", "I_IN_lim", "I_h2_c4"],
                 "S_va"),
    "pro": _monod("k_m_pro", "K_S_pro", "S_pro", "X_pro", ["I_pH_aa", "I_IN_lim",
                                                          "I_h2_pro"]),
    "ac": _monod("k_m_ac", "K_S_ac", "S_ac", "X_ac", ["I_pH_ac", "I_IN_lim", "I_nh3"]),
    "h2": _monod("k_m_h2", "K_S_h2", "S_h2", "X_h2", ["I_pH_h2", "I_IN_lim"]),
    "dsu": _fo("k_dec_su", "X_su"), "daa": _fo("k_dec_aa", "X_aa"),
    "dfa": _fo("k_dec_fa", "X_fa"), "dc4": _fo("k_dec_c4", "X_c4"),
    "dpro": _fo("k_dec_pro", "X_pro"), "dac": _fo("k_dec_ac", "X_ac"),
    "dh2": _fo("k_dec_h2", "X_h2"),
}
# processes whose rate depends on S_h2 and the eq.-8 coefficient they feed
H2_DEPENDENT = {"fa": "c7", "va": "c8", "bu": "c8", "pro": "c10", "h2": "c12"}
TRANSFER_ROWS = {"S_h2": "T8", "S_ch4": "T9", "S_IC": "T10"}


def c_expr(text: str, names: set) -> str:
    """A coefficient expression of the description (numbers, parameter names,
    + - * / and parentheses) as C on the adm1_params struct p."""
    import ast

    def emit(n):
        if isinstance(n, ast.Expression):
            return emit(n.body)
        if isinstance(n, ast.BinOp) and type(n.op) in (ast.Add, ast.Sub, ast.Mult, ast.Div):
            op = {ast.Add: "+", ast.Sub: "-", ast.Mult: "*", ast.Div: "/"}[type(n.op)]
            return f"({emit(n.left)} {op} {emit(n.right)})"
        if isinstance(n, ast.UnaryOp) and isinstance(n.op, (ast.USub, ast.UAdd)):
            return f"({'-' if isinstance(n.op, ast.USub) else '+'}{emit(n.operand)})"
        if isinstance(n, ast.Constant) and isinstance(n.value, (int, float)):
            return repr(float(n.value))
        if isinstance(n, ast.Name):
            if n.id not in names:
                raise ValueError(f"unknown parameter {n.id!r} in {text!r}")
            return f"p.{n.id}"
        raise ValueError(f"unsupported expression {text!r}")
    return emit(ast.parse(text, mode="eval"))


def param_names() -> set:
    import json
    with open(os.path.join(DATA, "adm1_params.json")) as fh:
        return set(json.load(fh)["values"])


def load_model(path: str = DEFAULT_MODEL) -> dict:
    """Read and check a model description; returns it with, per process, the
    stoichiometry as {state: (C expression, unit coefficient or None)}."""
    import json
    with open(path) as fh:
        m = json.load(fh)
    names = param_names()
    procs = m["processes"]
    if [q["name"] for q in procs] != PROCS:
        raise ValueError(f"{path}: the processes must be {PROCS} in that order")
    for q in procs:
        if q["rate"] != KERNEL_RATES[q["name"]]:
            raise ValueError(f"{path}: rate form of {q['name']!r} is not the kernel's "
                             f"{KERNEL_RATES[q['name']]}")
        for st in q["stoich"]:
            if st not in STATE or st in m["closures"]:
                raise ValueError(f"{path}: process {q['name']!r} sets {st!r}, which is not "
                                 "an organic liquid entry")
        q["c"] = {}
        for st, e in q["stoich"].items():
            t = e.replace(" ", "")
            unit = 1.0 if t == "1" else (-1.0 if t == "-1" else None)
            q["c"][st] = (c_expr(e, names), unit)
    if m["closures"] != {"S_IC": "carbon", "S_IN": "nitrogen"}:
        raise ValueError(f"{path}: the closures must be S_IC (carbon) and S_IN (nitrogen)")
    if m.get("transfers") != TRANSFER_ROWS:
        raise ValueError(f"{path}: the liquid-gas transfers must be {TRANSFER_ROWS}")
    for kind in ("carbon", "nitrogen"):
        m["contents"][kind] = {st: c_expr(e, names) for st, e in m["contents"][kind].items()}
    # table of the distinct coefficients that are not +-1, in process order of
    # their first use (a coefficient shared by several processes is one slot)
    m["table"], m["slot"], first = [], {}, {}
    for j, q in enumerate(procs):
        for st, (e, u) in q["c"].items():
            if u is not None:
                continue
            if e not in first:
                first[e] = len(m["table"])
                m["table"].append((j, st))
            m["slot"][(j, st)] = first[e]
    return m


MODEL = None


def use_model(path: str = DEFAULT_MODEL):
    """Set the Petersen matrix NU (liquid row -> [(coefficient, rate)]) and the
    eq.-8 row NU_H2 from a description."""
    global MODEL, NU, NU_H2
    MODEL = load_model(path)
    NU = {KNAME[st]: [] for st in STATE if st not in ("S_h2",)}
    NU_H2 = []
    for j, q in enumerate(MODEL["processes"]):
        for st, (e, u) in q["c"].items():
            coef = ("1.0" if u == 1.0 else "-1.0") if u is not None else \
                f"p.nu_v[{MODEL['slot'][(j, st)]}]"
            if st == "S_h2":
                NU_H2.append((coef, q["name"]))
            else:
                NU[KNAME[st]].append((coef, q["name"]))
    NU["SIC"] = [(f"p.nuIC[{j}]", r) for j, r in enumerate(PROCS)] + [("-1.0", "T10")]
    NU["SIN"] = [(f"p.nuIN[{j}]", r) for j, r in enumerate(PROCS)]
    NU["Sch4"].append(("-1.0", "T9"))
    NU_H2.append(("-1.0", "T8"))
    # gas rows: f_G = inv_vg (-q G + T)
    NU["Gh2"] = [("-p.inv_vg", "QGh2"), ("p.inv_vg", "T8")]
    NU["Gch4"] = [("-p.inv_vg", "QGch4"), ("p.inv_vg", "T9")]
    NU["Gco2"] = [("-p.inv_vg", "QGco2"), ("p.inv_vg", "T10")]


def emit_stoich() -> str:
    """Host code of the coefficients (ADM1_PETERSEN_FILL: the organic rows of
    the Petersen matrix from the named parameters; ADM1_NU_VALUES: the table
    of the coefficients that are not +-1, as the kernels read it;
    ADM1_CONTENTS: carbon and nitrogen contents) and the device code of the
    eq.-2 assembly of the liquid rows and of the eq.-8 coefficients."""
    m = MODEL
    procs = m["processes"]
    e = lambda st: "e" + KNAME[st].replace("Sh2", "Sh2")  # noqa: E731
    out = [f"// Generated by gen_jac.py from the model description {m['model']!r}.",
           "#pragma once",
           f"#define ADM1_MODEL_NAME \"{m['model']}\"",
           f"#define ADM1_NU_COUNT {len(m['table'])}",
           "#define ADM1_PETERSEN_FILL(p, nu) \\"]
    for j, q in enumerate(procs):
        for st, (ex, u) in q["c"].items():
            out.append(f"    nu[{e(st)}][{j}] = {repr(u) if u is not None else ex}; \\")
    out.append("    (void)0")
    out.append("#define ADM1_NU_VALUES(nu, d) \\")
    for k, (j, st) in enumerate(m["table"]):
        out.append(f"    d.nu_v[{k}] = nu[{e(st)}][{j}]; \\")
    out.append("    (void)0")
    out.append("#define ADM1_CONTENTS(p, C, N) \\")
    for st, ex in m["contents"]["carbon"].items():
        out.append(f"    C[{e(st)}] = {ex}; \\")
    for st, ex in m["contents"]["nitrogen"].items():
        out.append(f"    N[{e(st)}] = {ex}; \\")
    out.append("    (void)0")
    # device: eq.-2 assembly of the organic liquid rows (rates rho[19], the
    # inflow term IN(k), transfers T9 / T10 in their rows)
    out.append("#define ADM1_ASSEMBLE_LIQUID(out, IN, rho, R, T9, T10) \\")
    for st in STATE:
        if st in ("S_h2", "S_IC", "S_IN"):
            continue
        k = KNAME[st]
        terms = []
        for j, q in enumerate(procs):
            if st in q["c"]:
                ex, u = q["c"][st]
                if u == 1.0:
                    terms.append(f" + rho[{j}]")
                elif u == -1.0:
                    terms.append(f" - rho[{j}]")
                else:
                    terms.append(f" + (R)p.nu_v[{m['slot'][(j, st)]}] * rho[{j}]")
        if st == "S_ch4":
            terms.append(" - T9")
        out.append(f"    out({k}, (double)(IN({k}){''.join(terms)})); \\")
    out.append("    (void)0")
    # device: eq.-8 coefficients from the S_h2 row
    base, groups = [], {"c7": [], "c8": [], "c10": [], "c12": []}
    rate_of = {"fa": "b7", "va": "b8", "bu": "b9", "pro": "b10", "h2": "b12"}
    for j, q in enumerate(procs):
        if "S_h2" not in q["c"]:
            continue
        ex, u = q["c"]["S_h2"]
        coef = repr(u) if u is not None else f"p.nu_v[{m['slot'][(j, 'S_h2')]}]"
        if q["name"] in H2_DEPENDENT:
            g = H2_DEPENDENT[q["name"]]
            sign = "-" if g == "c12" else ""
            groups[g].append(f"{sign}({coef}) * (double){rate_of[q['name']]}")
        else:
            base.append(f" + ({coef}) * (double)rho[{j}]")
    out.append("#define ADM1_H2_TERMS(t, h2in, rho, b7, b8, b9, b10, b12) \\")
    out.append(f"    t.base = h2in{''.join(base)}; \\")
    for g, terms in groups.items():
        out.append(f"    t.{g} = {' + '.join(terms) if terms else '0.0'}; \\")
    out.append("    (void)0")
    return "\n".join(out) + "\n"


def partial_names():
    return [f"J_{r}_{v}" for r, vs in RATES.items() for v in vs]


def entries():
    """Structural entries of the bordered matrix M as
    {(row, col): [terms]} with terms (sign, coef, rate) meaning
    sign * coef * J_rate_col, plus the diagonal constants."""
    M = {}

    def add(r, c, term):
        M.setdefault((r, c), []).append(term)

    for i, yname in enumerate(Y):
        # alpha I (and + D for the liquid dilution term)
        add(i, i, ("diag_liq" if yname in LIQ else "diag_gas",))
        for coef, rate in NU[yname]:
            for v in RATES[rate]:
                add(i, VARS.index(v), ("-", coef, rate))
    r7 = NV - 2
    for v in RATES["E7"]:
        add(r7, VARS.index(v), ("+", "1.0", "E7"))
    r8 = NV - 1
    # M row = -dE8/dv (+ D on the S_h2 column)
    add(r8, VARS.index("Sh2"), ("D",))
    for coef, rate in NU_H2:
        for v in RATES[rate]:
            add(r8, VARS.index(v), ("-", coef, rate))
    return M


def expr(terms, col):
    parts = []
    for t in terms:
        if t[0] == "diag_liq":
            parts.append("(alpha + D)")
        elif t[0] == "diag_gas":
            parts.append("alpha")
        elif t[0] == "D":
            parts.append("D")
        else:
            sign, coef, rate = t
            name = f"d.J_{rate}_{VARS[col]}"
            if coef == "1.0":
                parts.append(("-" if sign == "-" else "+") + name)
            elif coef == "-1.0":
                parts.append(("+" if sign == "-" else "-") + name)
            else:
                parts.append(f"{'-' if sign == '-' else '+'}({coef}) * {name}")
    s = " ".join(parts)
    return s[1:] if s.startswith("+") else s


def emit_partials_struct():
    lines = ["// partial derivatives of every rate in its inputs (generated list)",
             "struct Partials {"]
    names = partial_names()
    for k in range(0, len(names), 6):
        lines.append("    double " + ", ".join(names[k:k + 6]) + ";")
    lines.append("};")
    return "\n".join(lines)


def emit_dense():
    M = entries()
    out = ["// Generated by gen_jac.py: dense bordered Newton matrix, row-major 30x30.",
           "// Expects: Partials d, DevParams p, double alpha, double D, double* M",
           "// (zeroed by the caller).", f"// structural nonzeros: {len(M)}"]
    for (r, c) in sorted(M):
        out.append(f"M[{r * NV + c}] = {expr(M[(r, c)], c)};")
    return "\n".join(out) + "\n"


def analyze():
    """Static elimination order (greedy Markowitz on the pattern, the two
    constraint rows/columns last) and the resulting LU pattern with fill.
    Pivots stay on the diagonal of the bordered system (row E7 with column
    S_H+, row E8 with column S_h2)."""
    M = entries()
    pat = {(r, c) for (r, c) in M}
    remaining = list(range(NV - 2))
    order = []
    cur = set(pat)
    while remaining:
        best = None
        for k in remaining:
            rows = [i for i in remaining + [NV - 2, NV - 1] if i != k and (i, k) in cur]
            cols = [j for j in remaining + [NV - 2, NV - 1] if j != k and (k, j) in cur]
            score = (len(rows) * len(cols), len(rows) + len(cols), k)
            if best is None or score < best[0]:
                best = (score, k, rows, cols)
        _, k, rows, cols = best
        for i in rows:
            for j in cols:
                cur.add((i, j))
        order.append(k)
        remaining.remove(k)
    for k in (NV - 2, NV - 1):
        if k == NV - 2:
            rows = [NV - 1] if (NV - 1, k) in cur else []
            cols = [NV - 1] if (k, NV - 1) in cur else []
            for i in rows:
                for j in cols:
                    cur.add((i, j))
        order.append(k)
    pos = {v: p for p, v in enumerate(order)}
    L = {k: [i for i in order if pos[i] > pos[k] and (i, k) in cur] for k in order}
    U = {k: [j for j in order if pos[j] > pos[k] and (k, j) in cur] for k in order}
    return order, cur, L, U


def lu_counts():
    order, cur, L, U = analyze()
    nnzL = sum(len(v) for v in L.values())
    nnzU = sum(len(v) for v in U.values())
    factor = sum(1 + len(L[k]) + 2 * len(L[k]) * len(U[k]) for k in order)
    solve = 2 * nnzL + 2 * nnzU + NV
    return dict(nnz_struct=len(entries()), nnz_lu=len(cur), nnz_L=nnzL, nnz_U=nnzU,
                factor_flops=factor, solve_flops=solve, order=[VARIABLES_NAME(v) for v in order])


def VARIABLES_NAME(v):
    return VARS[v] if v < NY_ else ("E7/H" if v == NV - 2 else "E8/Sh2")


NY_ = 28


def assembly_flops():
    """Flops of the generated assembly expressions (unit coefficients: 1 add;
    others: 1 mul + 1 add)."""
    M = entries()
    n = 0
    for terms in M.values():
        for t in terms:
            if t[0] in ("diag_liq",):
                n += 1
            elif len(t) == 3:
                n += 1 if t[1] in ("1.0", "-1.0") else 2
    return n


def emit_sparse1():
    """One lane per particle: the bordered matrix as named scalars m_r_c, the
    static-order LU, and a solve on b[30] (original variable order)."""
    order, cur, L, U = analyze()
    M = entries()
    out = ["// Generated by gen_jac.py: sparse bordered Newton matrix, static-order LU.",
           f"// structural nonzeros {len(M)}, with fill {len(cur)}",
           "#define ADM1_SP_DECL \\"]
    names = sorted(cur)
    for k in range(0, len(names), 8):
        out.append("    double " + ", ".join(f"m_{r}_{c}" for r, c in names[k:k + 8]) + "; \\")
    out.append("    double " + ", ".join(f"iv_{k}" for k in range(NV)) + ";")
    out.append("#define ADM1_SP_BUILD(alpha, D) \\")
    for (r, c) in names:
        e = expr(M[(r, c)], c) if (r, c) in M else "0.0"
        e = e.replace("alpha", "(alpha)").replace("(alpha + D)", "((alpha) + (D))")
        out.append(f"    m_{r}_{c} = {e}; \\")
    out.append("    (void)0")
    # growth guard (the static order does not pivot): every pivot at least
    # `floor` times its row's scale, alpha = 1/(gamma h) for the
    # differential rows, the diagonal entry before elimination for the two
    # constraint rows
    out.append("#define ADM1_SP_FACTOR(ok, floor, alpha) \\")
    out.append("    const double gd_ = (alpha) * (floor); \\")
    for k in (NV - 2, NV - 1):
        out.append(f"    const double g_{k} = fabs(m_{k}_{k}) * (floor); \\")
    for k in order:
        g = f"g_{k}" if k >= NV - 2 else "gd_"
        out.append(f"    iv_{k} = 1.0 / m_{k}_{k}; "
                   f"ok = ok & (isfinite(iv_{k}) & !(fabs(iv_{k}) * {g} > 1.0)); \\")
        for i in L[k]:
            out.append(f"    m_{i}_{k} *= iv_{k}; \\")
        for i in L[k]:
            for j in U[k]:
                out.append(f"    m_{i}_{j} -= m_{i}_{k} * m_{k}_{j}; \\")
    out.append("    (void)0")
    out.append("#define ADM1_SP_SOLVE(b) \\")
    for k in order:
        for i in L[k]:
            out.append(f"    b[{i}] -= m_{i}_{k} * b[{k}]; \\")
    for k in reversed(order):
        terms = "".join(f" - m_{k}_{j} * b[{j}]" for j in U[k])
        out.append(f"    b[{k}] = (b[{k}]{terms}) * iv_{k}; \\")
    out.append("    (void)0")
    return "\n".join(out) + "\n"


def emit_sparse1_lds():
    """One lane per particle with the bordered matrix in LDS: entry e of the
    static-order LU (the 242 positions of emit_sparse1, in sorted order) of
    the lane's particle at ADM1_SPL_M(e), which the kernel maps to
    lds[e * 64 + lane] (consecutive lanes, consecutive banks); the inverse
    pivots stay in registers.  Same arithmetic as emit_sparse1."""
    order, cur, L, U = analyze()
    M = entries()
    names = sorted(cur)
    idx = {rc: e for e, rc in enumerate(names)}
    m = lambda r, c: f"ADM1_SPL_M({idx[(r, c)]})"  # noqa: E731
    out = ["// Generated by gen_jac.py: sparse bordered Newton matrix in LDS, static-order LU.",
           f"// structural nonzeros {len(M)}, with fill {len(cur)}",
           f"#define ADM1_SPL_NNZ {len(cur)}",
           "#define ADM1_SPL_DECL \\",
           "    double " + ", ".join(f"iv_{k}" for k in range(NV)) + ";",
           "#define ADM1_SPL_BUILD(alpha, D) \\"]
    for (r, c) in names:
        e = expr(M[(r, c)], c) if (r, c) in M else "0.0"
        e = e.replace("alpha", "(alpha)").replace("(alpha + D)", "((alpha) + (D))")
        out.append(f"    {m(r, c)} = {e}; \\")
    out.append("    (void)0")
    out.append("#define ADM1_SPL_FACTOR(ok, floor, alpha) \\")
    out.append("    const double gd_ = (alpha) * (floor); \\")
    for k in (NV - 2, NV - 1):
        out.append(f"    const double g_{k} = fabs({m(k, k)}) * (floor); \\")
    for k in order:
        g = f"g_{k}" if k >= NV - 2 else "gd_"
        out.append(f"    iv_{k} = 1.0 / {m(k, k)}; "
                   f"ok = ok & (isfinite(iv_{k}) & !(fabs(iv_{k}) * {g} > 1.0)); \\")
        for i in L[k]:
            out.append(f"    {m(i, k)} *= iv_{k}; \\")
        for i in L[k]:
            for j in U[k]:
                out.append(f"    {m(i, j)} -= {m(i, k)} * {m(k, j)}; \\")
    out.append("    (void)0")
    out.append("#define ADM1_SPL_SOLVE(b) \\")
    for k in order:
        for i in L[k]:
            out.append(f"    b[{i}] -= {m(i, k)} * b[{k}]; \\")
    for k in reversed(order):
        terms = "".join(f" - {m(k, j)} * b[{j}]" for j in U[k])
        out.append(f"    b[{k}] = (b[{k}]{terms}) * iv_{k}; \\")
    out.append("    (void)0")
    return "\n".join(out) + "\n"


def pairing(order, cur):
    """Rows (elimination positions) paired over the two lanes of a particle.
    The two constraint rows form the last pair; the others are paired greedily,
    longest pattern first, with the partner adding the fewest new columns."""
    pos = {v: p for p, v in enumerate(order)}
    rows = {p: set() for p in range(NV)}
    for (r, c) in cur:
        rows[pos[r]].add(pos[c])
    pairs = []
    remaining = list(range(NV - 2))
    while remaining:
        a = max(remaining, key=lambda q: (len(rows[q]), -q))
        remaining.remove(a)
        b = min(remaining, key=lambda q: (len(rows[a] | rows[q]) - len(rows[a]),
                                          -len(rows[q]), q))
        remaining.remove(b)
        pairs.append((min(a, b), max(a, b)))
    pairs.sort()
    pairs.append((NV - 2, NV - 1))
    return pairs, rows


def emit_sparse2():
    """Two lanes per particle.  Lane side h of pair m owns the row at
    elimination position pairs[m][h]; register w<m>_<c> holds, on each lane,
    its own row's entry in column position c (the union of the two rows'
    patterns, absent entries being zero).  `odd` is the lane side.  Pivot
    rows and solution components move between the two lanes with DPP
    broadcasts (bc<h>), so both lanes run the same instruction stream."""
    order, cur, L, U = analyze()
    M = entries()
    pos = {v: p for p, v in enumerate(order)}
    pairs, rows = pairing(order, cur)
    side = {}
    pair_of = {}
    for m, (a, b) in enumerate(pairs):
        side[a], side[b] = 0, 1
        pair_of[a], pair_of[b] = m, m
    slots = {m: sorted(rows[a] | rows[b]) for m, (a, b) in enumerate(pairs)}
    var = lambda p: order[p]  # noqa: E731
    out = ["// Generated by gen_jac.py: two-lanes-per-particle sparse bordered LU.",
           f"// pairs (elimination positions): {pairs}",
           f"// slots per lane: {sum(len(s) for s in slots.values())}"]

    def cexpr(p, c):
        r, cv = var(p), var(c)
        if (r, cv) in M:
            e = expr(M[(r, cv)], cv)
            return e.replace("(alpha + D)", "(alpha + D)")
        return "0.0"

    # declarations
    decl = []
    for m in range(len(pairs)):
        decl += [f"w{m}_{c}" for c in slots[m]]
    out.append("#define ADM1_SP2_DECL \\")
    for k in range(0, len(decl), 10):
        out.append("    double " + ", ".join(decl[k:k + 10]) + "; \\")
    out.append("    (void)0")
    # assembly.  The parameters are read into locals first: both sides of
    # each lane-dependent select then are plain values, so the select stays
    # a per-lane choice instead of becoming a branch around a memory load
    # (every wave holds both sides, so a branch runs both anyway).
    out.append("#define ADM1_SP2_BUILD(alpha, D) \\")
    body, hoist = [], {}

    def hoisted(e):
        def sub(mt):
            ref = mt.group(0)
            if ref not in hoist:
                hoist[ref] = f"q{len(hoist)}"
            return hoist[ref]
        return re.sub(r"\bp\.[A-Za-z_]\w*(?:\[\d+\])?", sub, e)
    for m, (a, b) in enumerate(pairs):
        for c in slots[m]:
            e0, e1 = hoisted(cexpr(a, c)), hoisted(cexpr(b, c))
            if e0 == e1:
                body.append(f"    w{m}_{c} = {e0}; \\")
            else:
                body.append(f"    w{m}_{c} = odd ? ({e1}) : ({e0}); \\")
    for ref, name in hoist.items():
        out.append(f"    const double {name} = {ref}; \\")
    out += body
    out.append("    (void)0")

    def role(q, k, structural):
        if q == k:
            return "P"
        if q < k:
            return "U"
        return "L" if structural else "Z"

    def roles(m, k):
        a, b = pairs[m]
        return (role(a, k, (var(a), var(k)) in cur), role(b, k, (var(b), var(k)) in cur))

    def masked(m, k, want):
        """Expression of slot (m, k) restricted to lanes whose role is in want
        ({'L','Z'} for the forward direction, {'U'} for the backward one)."""
        r = roles(m, k)
        ok = [x in want for x in r]
        if all(ok):
            return f"w{m}_{k}"
        if not any(ok):
            return None
        h = 0 if ok[0] else 1
        return f"({'odd' if h else '!odd'} ? w{m}_{k} : 0.0)"

    counts = dict(bcast=0, fma_factor=0, fma_solve=0, sel=0)
    # factorisation
    # growth guard: the pivots of the differential rows at least floor *
    # alpha, those of the two constraint rows (the last pair, one per side)
    # at least floor times their diagonal entries before elimination; every
    # pivot's reciprocal reaches both lanes, so both take the same decision
    out.append("#define ADM1_SP2_FACTOR(ok, floor, alpha) \\")
    out.append("    const double gd_ = (alpha) * (floor); \\")
    guard = {}
    for k in range(NV):
        if k >= NV - 2:
            mk, sk = pair_of[k], side[k]
            out.append(f"    const double g{k}_ = fabs(bc{sk}(w{mk}_{k})) * (floor); \\")
            guard[k] = f"g{k}_"
        else:
            guard[k] = "gd_"
    for k in range(NV):
        mk, sk = pair_of[k], side[k]
        out.append(f"    {{ const double iv = bc{sk}(1.0 / w{mk}_{k}); "
                   f"ok = ok & (isfinite(iv) & !(fabs(iv) * {guard[k]} > 1.0)); \\")
        counts["bcast"] += 1
        lpairs = []
        for m in range(len(pairs)):
            if k not in slots[m]:
                continue
            r0, r1 = roles(m, k)
            rr = (r0, r1)
            if "P" in rr:
                other = r1 if r0 == "P" else r0
                ps = 0 if r0 == "P" else 1
                pick = "odd" if ps == 1 else "!odd"
                if other in ("L", "Z"):
                    out.append(f"      w{m}_{k} = {pick} ? iv : w{m}_{k} * iv; \\")
                else:
                    out.append(f"      w{m}_{k} = {pick} ? iv : w{m}_{k}; \\")
                counts["sel"] += 1
                if other == "L":
                    lpairs.append(m)
            elif r0 in ("L", "Z") and r1 in ("L", "Z"):
                if "L" in rr:
                    out.append(f"      w{m}_{k} *= iv; \\")
                    lpairs.append(m)
            elif "L" in rr:
                h = 0 if r0 == "L" else 1
                pick = "odd" if h == 1 else "!odd"
                out.append(f"      w{m}_{k} = {pick} ? w{m}_{k} * iv : w{m}_{k}; \\")
                counts["sel"] += 1
                lpairs.append(m)
        if lpairs and U[var(k)]:
            ucols = [pos[j] for j in U[var(k)]]
            for c in ucols:
                out.append(f"      const double u{c} = bc{sk}(w{mk}_{c}); \\")
                counts["bcast"] += 1
            for m in lpairs:
                lx = masked(m, k, {"L", "Z"})
                out.append(f"      {{ const double l = {lx}; \\")
                for c in ucols:
                    if c in slots[m]:
                        out.append(f"        w{m}_{c} -= l * u{c}; \\")
                        counts["fma_factor"] += 1
                out.append("      } \\")
        out.append("    } \\")
    out.append("    (void)0")
    # forward / backward substitution on b<m> (own components)
    out.append("#define ADM1_SP2_SOLVE() \\")
    for k in range(NV):
        mk, sk = pair_of[k], side[k]
        targets = [m for m in range(len(pairs)) if k in slots[m] and masked(m, k, {"L"})
                   is not None and any(x == "L" for x in roles(m, k))]
        if not targets:
            continue
        out.append(f"    {{ const double z = bc{sk}(b{mk}); \\")
        counts["bcast"] += 1
        for m in targets:
            out.append(f"      b{m} -= {masked(m, k, {'L', 'Z'})} * z; \\")
            counts["fma_solve"] += 1
        out.append("    } \\")
    for k in reversed(range(NV)):
        mk, sk = pair_of[k], side[k]
        pick = "odd" if sk == 1 else "!odd"
        out.append(f"    b{mk} = {pick} ? b{mk} * w{mk}_{k} : b{mk}; \\")
        counts["sel"] += 1
        targets = [m for m in range(len(pairs)) if k in slots[m] and
                   any(x == "U" for x in roles(m, k)) and
                   (var(pairs[m][0]), var(k)) in cur | {(var(pairs[m][1]), var(k))} | set()]
        targets = [m for m in range(len(pairs)) if k in slots[m] and
                   any(roles(m, k)[h] == "U" and (var(pairs[m][h]), var(k)) in cur
                       for h in (0, 1))]
        if not targets:
            continue
        out.append(f"    {{ const double x = bc{sk}(b{mk}); \\")
        counts["bcast"] += 1
        for m in targets:
            out.append(f"      b{m} -= {masked(m, k, {'U'})} * x; \\")
            counts["fma_solve"] += 1
        out.append("    } \\")
    out.append("    (void)0")
    # which pair/side owns each differential variable's row
    out.append("// owner of each variable's row: pair and side")
    own_pair = [pair_of[pos[v]] for v in range(NV)]
    own_side = [side[pos[v]] for v in range(NV)]
    out.append(f"#define ADM1_SP2_NPAIR {len(pairs)}")
    out.append("#define ADM1_SP2_VAR_PAIR {" + ", ".join(map(str, own_pair)) + "}")
    out.append("#define ADM1_SP2_VAR_SIDE {" + ", ".join(map(str, own_side)) + "}")
    # variable held by side h of pair m
    pv0 = [var(a) for a, b in pairs]
    pv1 = [var(b) for a, b in pairs]
    out.append("#define ADM1_SP2_PAIR_VAR0 {" + ", ".join(map(str, pv0)) + "}")
    out.append("#define ADM1_SP2_PAIR_VAR1 {" + ", ".join(map(str, pv1)) + "}")
    out.append(f"// counts per lane: {counts}")
    return "\n".join(out) + "\n", counts, sum(len(s) for s in slots.values())


def main():
    import argparse
    import json
    ap = argparse.ArgumentParser()
    ap.add_argument("--model", default=DEFAULT_MODEL, help="model description (JSON)")
    ap.add_argument("--out", default=HERE, help="directory of the generated files")
    ap.add_argument("--stats", action="store_true")
    args = ap.parse_args()
    use_model(args.model)
    out = lambda name: os.path.join(args.out, name)  # noqa: E731
    with open(out("adm1_stoich.inc"), "w") as fh:
        fh.write(emit_stoich())
    with open(out("adm1_jac_sparse2.inc"), "w") as fh:
        txt, counts, nslots = emit_sparse2()
        fh.write(txt)
    if args.stats:
        print("sparse2 slots/lane", nslots, counts)
    with open(out("adm1_partials.inc"), "w") as fh:
        fh.write("// Generated by gen_jac.py -- do not edit.\n" + emit_partials_struct() + "\n")
    with open(out("adm1_jac_dense.inc"), "w") as fh:
        fh.write(emit_dense())
    with open(out("adm1_jac_sparse1.inc"), "w") as fh:
        fh.write(emit_sparse1())
    with open(out("adm1_jac_sparse1_lds.inc"), "w") as fh:
        fh.write(emit_sparse1_lds())
    stats = lu_counts()
    stats["assembly_flops"] = assembly_flops()
    stats["model"] = MODEL["model"]
    with open(out("adm1_lu_stats.json"), "w") as fh:
        json.dump(stats, fh, indent=1)
    if args.stats:
        print(json.dumps({k: v for k, v in stats.items() if k != "order"}))
        print("order:", " ".join(stats["order"]))


if __name__ == "__main__":
    main()
