"""The Petersen matrix as data (sec. 2.2, eq. 2; sec. 5 on other biokinetic
models): the model descriptions, the oracle's own reader of them, and the
kernel generator's checks.  CPU only."""
from __future__ import annotations

import copy
import importlib.util
import json
import os

import numpy as np
import pytest

from oracle import model_desc as MD
from oracle.adm1 import Oracle
from paper_2311_08927_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DATA = os.path.join(ROOT, "paper_2311_08927_amd", "data")
STANDARD = os.path.join(DATA, "adm1_petersen.json")
VARIANT = os.path.join(DATA, "adm1_petersen_decay_to_particulates.json")
DECAYS = list(range(12, 19))
DIS = 0
ROW = {n: i for i, n in enumerate(MD.LIQUID)}


def _gen():
    """The kernel generator as a module (it is a script beside the sources)."""
    path = os.path.join(ROOT, "paper_2311_08927_amd", "csrc", "gen_jac.py")
    spec = importlib.util.spec_from_file_location("gen_jac_under_test", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_standard_description_is_the_built_in_matrix():
    """The standard description, read by the oracle's parser, gives exactly
    the matrix and contents the oracle's hand-written formulas give (those
    are pinned elsewhere by COD, carbon and nitrogen continuity and by the
    textbook coefficients)."""
    a = Oracle(W.params_path())
    b = Oracle(W.params_path(), model=STANDARD)
    assert np.array_equal(a.petersen(), b.petersen())
    for u, v in zip(a.contents(), b.contents()):
        assert np.array_equal(u, v)


def test_variant_decay_is_decay_then_disintegration():
    """In the variant, biomass decays straight to the disintegration
    products: each decay column equals the standard decay column (biomass to
    composites) plus one unit of the standard disintegration column
    (composites to their fractions), closures included, since both are
    linear in the organic rows."""
    std = Oracle(W.params_path()).petersen()
    var = Oracle(W.params_path(), model=VARIANT).petersen()
    for j in DECAYS:
        want = std[:, j] + std[:, DIS]
        assert np.allclose(var[:, j], want, rtol=0, atol=1e-15), j
        assert var[ROW["X_xc"], j] == 0.0
    others = [j for j in range(MD.NPROC) if j not in DECAYS]
    assert np.array_equal(var[:, others], std[:, others])


def test_variant_conserves_cod_carbon_nitrogen():
    """COD over the COD rows (checked by the oracle's constructor), and
    carbon and nitrogen over all rows (the closures), hold column by column
    for the variant."""
    orc = Oracle(W.params_path(), model=VARIANT)     # raises on a COD violation
    nu = orc.petersen()
    C, N = orc.contents()
    Cf, Nf = C.copy(), N.copy()
    Cf[ROW["S_IC"]] = 1.0    # inorganic carbon is counted in kmol C
    Nf[ROW["S_IN"]] = 1.0
    assert np.abs(Cf @ nu).max() < 1e-15
    assert np.abs(Nf @ nu).max() < 1e-15


def test_cod_violation_is_refused(tmp_path):
    desc = MD.load(VARIANT)
    desc["processes"][12]["stoich"]["X_I"] = "f_xI_xc + 0.01"
    path = tmp_path / "bad_model.json"
    path.write_text(json.dumps(desc))
    with pytest.raises(ValueError, match="COD"):
        Oracle(W.params_path(), model=str(path))


@pytest.mark.parametrize("text,expect", [
    ("1 - a", lambda a, b, c: 1 - a),
    ("(1 - a) * b", lambda a, b, c: (1 - a) * b),
    ("1 - a * b", lambda a, b, c: 1 - a * b),
    ("a / b / c", lambda a, b, c: (a / b) / c),
    ("a - b - c", lambda a, b, c: (a - b) - c),
    ("-a * -b", lambda a, b, c: a * b),
    ("2.5e-1 * (a + .5)", lambda a, b, c: 0.25 * (a + 0.5)),
    ("-(a - (b - c))", lambda a, b, c: -(a - (b - c))),
])
def test_expression_evaluator(text, expect):
    """Precedence and associativity against hand-written values."""
    vals = {"a": 0.3, "b": 1.7, "c": 0.11}
    assert MD.evaluate(text, vals) == pytest.approx(expect(0.3, 1.7, 0.11), rel=1e-15)


@pytest.mark.parametrize("text", ["a +", "(a", "a)", "a ^ 2", "d", "a b", ""])
def test_expression_errors(text):
    with pytest.raises(ValueError):
        MD.evaluate(text, {"a": 1.0})


def _changed(mut):
    desc = MD.load(STANDARD)
    mut(desc)
    return desc


RATE_CHANGES = {
    "constant": lambda d: d["processes"][0]["rate"].__setitem__("k", "k_hyd_ch"),
    "factor": lambda d: d["processes"][4]["rate"]["factors"].append("I_nh3"),
    "order": lambda d: d["processes"].insert(0, d["processes"].pop(1)),
    "form": lambda d: d["processes"][5]["rate"].__setitem__("form", "monod_competing"),
}


@pytest.mark.parametrize("change", sorted(RATE_CHANGES))
def test_rate_form_changes_are_refused(change, tmp_path):
    """Rate forms are hand-written on both sides (the oracle's rates and the
    kernel's), so a description may change the matrix, not a rate form: the
    oracle's reader and the kernel generator both refuse."""
    desc = _changed(RATE_CHANGES[change])
    with pytest.raises(ValueError):
        MD.check_rates(desc)
    path = tmp_path / "m.json"
    path.write_text(json.dumps(desc))
    with pytest.raises(ValueError):
        _gen().load_model(str(path))


def test_generator_reads_both_descriptions():
    """The generator's table of non-unit coefficients: a coefficient shared by
    several processes is one slot, so the variant's decays reuse the
    disintegration fractions' slots; the matrix it fills equals the
    oracle's."""
    g = _gen()
    std = g.load_model(STANDARD)
    var = g.load_model(VARIANT)
    assert len(var["table"]) == len(std["table"])
    assert {var["slot"][(j, "X_ch")] for j in DECAYS} == {var["slot"][(DIS, "X_ch")]}
    vals = Oracle(W.params_path()).values
    for path, m in ((STANDARD, std), (VARIANT, var)):
        nu = Oracle(W.params_path(), model=path).petersen()
        for j, q in enumerate(m["processes"]):
            for st in q["stoich"]:
                assert nu[ROW[st], j] == pytest.approx(MD.evaluate(q["stoich"][st], vals),
                                                       rel=1e-15)


def test_closed_rows_and_transfers_are_fixed():
    for mut in (lambda d: d["processes"][4]["stoich"].__setitem__("S_IC", "0.1"),
                lambda d: d.__setitem__("transfers", {"S_h2": "T8"}),
                lambda d: d.__setitem__("closures", {"S_IC": "carbon"})):
        with pytest.raises(ValueError):
            MD.tables(_changed(mut), Oracle(W.params_path()).values)


def test_description_round_trip_copy_is_harmless():
    """Reading does not modify the description (the generator annotates its
    own copy)."""
    desc = MD.load(STANDARD)
    before = copy.deepcopy(desc)
    MD.tables(desc, Oracle(W.params_path()).values)
    assert desc == before
