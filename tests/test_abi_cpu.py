"""CPU-side checks of the C ABI: the library loads, exports every symbol the
header declares, and the ctypes mirrors match the C struct layouts.  No
compute calls (there is no GPU here)."""
from __future__ import annotations

import json
import os
import re
import subprocess

import pytest

from paper_2311_08927_amd import adm1 as A

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "adm1.h")


def header_text():
    with open(HEADER) as fh:
        return fh.read()


def declared_functions():
    txt = re.sub(r"/\*.*?\*/", "", header_text(), flags=re.S)
    return sorted(set(re.findall(r"\b(adm1_\w+)\s*\(", txt)))


def test_header_declares_the_boundary():
    fns = declared_functions()
    for f in ["adm1_init", "adm1_step_particles", "adm1_gas_flux", "adm1_rhs",
              "adm1_jacobian", "adm1_strerror", "adm1_destroy", "adm1_set_opts",
              "adm1_param_names", "adm1_solve_ph", "adm1_last_failures"]:
        assert f in fns


@pytest.mark.parametrize("model", [None, "adm1_decay_to_particulates"])
def test_library_exports_every_declared_symbol(model):
    """Each model description's library exports the whole boundary and
    reports the description it was generated from."""
    lib = A.lib(model)
    for f in declared_functions():
        assert hasattr(lib, f), f
    assert lib.adm1_model_name().decode() == (model or "adm1")


def test_param_names_match_header_and_data():
    txt = header_text()
    body = re.search(r"typedef struct adm1_params \{(.*?)\} adm1_params;", txt, re.S).group(1)
    fields = re.findall(r"\b([A-Za-z_][A-Za-z0-9_]*)\s*[,;]", body.replace("double", ""))
    assert fields == A.param_names()
    with open(os.path.join(ROOT, "paper_2311_08927_amd", "data", "adm1_params.json")) as fh:
        vals = json.load(fh)["values"]
    assert set(A.param_names()) == set(vals)


def test_strerror():
    assert A.strerror(0) == "ok"
    assert "n_max" in A.strerror(-2)
    assert "device" in A.strerror(-3)


def test_ctypes_layout_matches_c(tmp_path):
    src = tmp_path / "sz.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "adm1.h"\n'
                   'int main(void){printf("%zu %zu %zu %zu %zu %zu\\n", sizeof(adm1_opts),'
                   ' offsetof(adm1_opts, max_steps), offsetof(adm1_opts, variant),'
                   ' sizeof(adm1_feed), sizeof(adm1_aux), sizeof(adm1_params));return 0;}\n')
    exe = tmp_path / "sz"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o",
                           str(exe)])
    got = [int(v) for v in subprocess.check_output([str(exe)]).split()]
    import ctypes
    assert got[0] == ctypes.sizeof(A.adm1_opts)
    assert got[1] == A.adm1_opts.max_steps.offset
    assert got[2] == A.adm1_opts.variant.offset
    assert got[3] == ctypes.sizeof(A.adm1_feed)
    assert got[4] == ctypes.sizeof(A.adm1_aux)
    assert got[5] == 8 * len(A.param_names())


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(A, "_libs", {})
    monkeypatch.setattr(A, "LIB_PATH", str(tmp_path / "nope.so"))
    with pytest.raises(RuntimeError, match="not built"):
        A.lib()
    with pytest.raises(RuntimeError, match="not built"):
        A.lib("adm1_no_such_model")
