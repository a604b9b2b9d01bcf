"""The flop model of the step against operation counts of the oracle itself
(its C source built with a counting scalar type)."""
from __future__ import annotations

import json

from oracle import count_flops as C
from oracle.adm1 import Oracle
from paper_2311_08927_amd import flops as F
from paper_2311_08927_amd import workloads as W


def test_counts_reproduce_the_committed_table():
    """oracle/flop_counts.json is what the counting build reports now."""
    with open(C.OUT) as fh:
        stored = json.load(fh)
    orc = Oracle(W.params_path())
    for (label, x, T, D, s), row in zip(C.states(), stored["states"]):
        fresh = C.count(orc, x, T, D, s)
        for part in C.PARTS:
            assert fresh[part] == row[part], (label, part)


def test_flop_model_uses_the_oracle_counts():
    """The right-hand side of the model is the oracle's count of the same
    formulas (rates and transfers + eq.-2 assembly, open reactor); the
    temperature constants take the oracle's 8 exponentials; the Newton
    iteration figure stays at or below the oracle's own per-iteration
    counts, so the model never charges more than the oracle computes."""
    orc = Oracle(W.params_path())
    nom = W.nominal()
    c = C.count(orc, nom["state"], nom["T"], nom["D"], nom["feed"])
    assert F.F_RHS_BASE == c["rates"]["total"] + c["assembly"]["total"]
    assert c["tconst"]["exp"] == 8 and F.F_TCONST >= c["tconst"]["total"]
    eq7_iteration = c["eq7_eval"]["total"] + 2      # plus the update H - E/dE
    eq8_iteration = c["eq8_eval_oracle_form"]["total"] + 2
    assert F.F_NEWTON <= min(eq7_iteration, eq8_iteration)
    # divisions and transcendentals are tallied separately
    assert c["rates"]["div"] > 0 and c["rates"]["pow"] == 9


def test_counting_rules():
    """A closed particle (D = 0) drops only the dilution terms D (S_in - x)
    of the assembly (48 operations over the liquid rows: a multiply by an
    exact zero is free, and so is the add of its zero result) and nothing in
    the rates."""
    orc = Oracle(W.params_path())
    nom = W.nominal()
    a = C.count(orc, nom["state"], nom["T"], nom["D"], nom["feed"])
    b = C.count(orc, nom["state"], nom["T"], 0.0, nom["feed"])
    assert a["rates"] == b["rates"]
    assert a["assembly"]["total"] - b["assembly"]["total"] == 2 * 24
