"""The grouped-lane LU generator behind the lanes-per-particle measurement:
its row groups partition the 30 rows of the bordered matrix, and for two
lanes it keeps as many registers per lane as the step kernel's own split.
CPU only."""
from __future__ import annotations

import importlib.util
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2311_08927_amd", "csrc")


def _load(name):
    spec = importlib.util.spec_from_file_location(name, os.path.join(CSRC, name + ".py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_groups_partition_the_rows_and_slot_counts():
    gl = _load("gen_lu_groups")
    gl.GJ.use_model()
    for G in (2, 4):
        txt = gl.emit(G)
        groups = eval(re.search(r"// groups \(elimination positions\): (.*)", txt).group(1))
        rows = [q for g in groups for q in g if q is not None]
        assert sorted(rows) == list(range(30)) and all(len(g) == G for g in groups)
        slots = int(re.search(r"// slots per lane: (\d+)", txt).group(1))
        assert slots >= 242 / G          # at least the factor's nonzeros per lane
        if G == 2:
            with open(os.path.join(CSRC, "adm1_jac_sparse2.inc")) as fh:
                kernel = int(re.search(r"// slots per lane: (\d+)", fh.read()).group(1))
            assert slots == kernel
