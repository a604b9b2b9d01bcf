"""Algorithmic flop and byte model of the per-particle ADM1 step.

Counts are of the method, not of any kernel's redundancy: one Rodas4 step
attempt needs six right-hand-side evaluations, one set of rate partials, the
assembly of the sparse bordered Newton matrix, its static-order sparse LU and
six forward/backward solves, plus the stage combinations and the error norm.
The LU and assembly counts come from the generator's elimination analysis
(csrc/adm1_lu_stats.json); the others were counted from csrc/adm1_model.h
and the step loop (add/sub/mul = 1, fused multiply-add = 2, divide = 1,
exp/pow = 1 each and also tallied separately).  Algebraic Newton iterations
are data dependent and counted from the kernel's own per-particle tally.
"""
from __future__ import annotations

import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))

# right-hand side without the Newton loops: inhibitions, 19 rates, 3
# transfers, gas flow, eq.-8 set-up, the eq.-2 assembly of 28 derivatives
F_RHS_BASE = 514
# one Newton iteration, averaged over eq. 7 (60 flops: 7 divides, the ion
# fractions and their derivatives) and eq. 8 (40 flops: 4 divides)
F_NEWTON = 50
# analytic partial derivatives of all rates (pH/N/h2 inhibitions, Monod
# derivatives, transfers, valve, eq.-7 gradient)
F_PARTIALS = 430
# stage arguments y0 + sum a_ij u_j and corrections sum c_ij/h u_j over six
# stages (2 x 15 fused multiply-adds per entry), the error norm (6 per entry)
# and the step-size control
F_VECTOR = 2 * 2 * 15 * 28 + 6 * 28 + 20
# temperature constants per particle and interval (9 exponentials)
F_TCONST = 40
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
