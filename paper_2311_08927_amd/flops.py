"""Algorithmic flop and byte model of the per-particle ADM1 step.

Counts are of the method, not of any kernel's redundancy: one Rodas4 step
attempt needs six right-hand-side evaluations, one set of rate partials, the
assembly of the sparse bordered Newton matrix, its static-order sparse LU and
six forward/backward solves, plus the stage combinations and the error norm.

Where the FP64 oracle computes the same thing in the same form, the figure is
the oracle's own operation count: its C source built with a counting scalar
type (oracle/count_ops.cpp, oracle/count_flops.py -> oracle/flop_counts.json;
add, multiply, divide, exp, log, pow and sqrt are 1 each and also tallied
separately; multiplies by exact 0 or +-1 and adds of exact 0, i.e. the
Petersen matrix's structural zeros and unit coefficients, are not counted).
That covers the right-hand side (rates, transfers and gas flow: 124, of them
27 divides and 9 pow; the eq.-2 assembly and headspace balances: 224, 4
divides) and the temperature constants (8 exp).  The oracle has no
counterpart of the analytic partials and of the sparse LU (it differentiates
by complex steps and factors a dense 28x28 matrix), so those figures come
from the kernel source (partials) and from the generator's elimination
analysis (assembly, factor, solve: csrc/adm1_lu_stats.json).  Algebraic
Newton iterations are data dependent and counted from the kernel's own
per-particle tally at 50 flops each, below the oracle's 78 for an eq.-7
iteration (its residual and derivative with separate divisions) and 177 for
an eq.-8 iteration (which re-evaluates every rate), so the model does not
over-count them.
"""
from __future__ import annotations

import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))

# right-hand side without the Newton loops: the oracle's count of its rates,
# transfers and gas flow (124) and of the eq.-2 assembly with the headspace
# balances (224), nominal state of the open reactor
F_RHS_BASE = 124 + 224
# one algebraic Newton iteration (kernel count, averaged over eq. 7 and eq. 8)
F_NEWTON = 50
# analytic partial derivatives of all rates (pH/N/h2 inhibitions, Monod
# derivatives, transfers, valve, eq.-7 gradient), counted from the kernel
F_PARTIALS = 430
# stage arguments y0 + sum a_ij u_j and corrections sum c_ij/h u_j over six
# stages (2 x 15 multiply-adds per entry), the error norm (6 per entry) and
# the step-size control
F_VECTOR = 2 * 2 * 15 * 28 + 6 * 28 + 20
# temperature constants per particle and interval: 8 exponentials (oracle
# count) and the 11 products and differences around them
F_TCONST = 8 + 11
# bytes per particle and interval: state in and out (35 x 8 x 2), T, D,
# feed index, warm starts in and out (2 x 8 x 2), status, 3 counters
BYTES_PER_PARTICLE_STEP = 35 * 8 * 2 + 8 + 8 + 4 + 32 + 1 + 12


def lu_stats() -> dict:
    with open(os.path.join(HERE, "csrc", "adm1_lu_stats.json")) as fh:
        return json.load(fh)


def per_attempt() -> int:
    s = lu_stats()
    return (6 * F_RHS_BASE + F_PARTIALS + s["assembly_flops"] + s["factor_flops"] +
            6 * s["solve_flops"] + F_VECTOR)


def total_flops(attempts: int, newton: int, particles: int) -> float:
    """Algorithmic flops of `particles` particle-intervals that took
    `attempts` Rosenbrock attempts and `newton` algebraic iterations in all.
    Each interval also evaluates the right-hand side at its start and end."""
    return float(attempts) * per_attempt() + float(newton) * F_NEWTON + \
        particles * (F_TCONST + 2 * F_RHS_BASE)


# --- the fixed-step explicit scheme (sec. 2.3, sec. 4.3) --------------------
# explicit Euler update y + h f (one fused multiply-add per entry)
F_EULER_VECTOR = 2 * 28
# classical RK4: three stage arguments and the weighted sum (13 flops per
# entry as the kernel forms them)
F_RK4_VECTOR = 13 * 28
# the algebraic write-back at the end of the interval: inhibitions and the
# rate factors that enter eq. 8, then the six ion fractions
F_ALG_END = 220
# bytes per particle and interval: state in and out, T, D, feed index, the
# particle's feed row (26 entries), S_H+ in and out, status, Newton tally
BYTES_FIXED = 35 * 8 * 2 + 8 + 8 + 4 + 26 * 8 + 16 + 1 + 4


def fixed_flops(method: str, substeps: int, newton: int, particles: int) -> float:
    """Algorithmic flops of `particles` particle-intervals of the fixed-step
    scheme (`substeps` explicit steps each) that took `newton` algebraic
    iterations in all."""
    if method == "euler":
        per = F_RHS_BASE + F_EULER_VECTOR
    else:
        per = 4 * F_RHS_BASE + F_RK4_VECTOR
    return float(particles) * (F_TCONST + F_ALG_END + substeps * per) + float(newton) * F_NEWTON
