"""GPU parity for a second model description (sec. 5, other biokinetic
models): the library generated from the decay-to-particulates variant of the
Petersen matrix against the oracle reading the same description with its own
parser.  Every Newton-matrix variant of the step is checked, and the
standard oracle is shown to disagree, so the comparison sees the variant."""
from __future__ import annotations

import os

import numpy as np
import pytest

from oracle.adm1 import Oracle
from paper_2311_08927_amd import workloads as W
from tests.gpu_common import PARITY_TOL, run_side_by_side

pytestmark = pytest.mark.gpu

RTOL = 1e-8
MODEL = "adm1_decay_to_particulates"
DESC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                    "paper_2311_08927_amd", "data", "adm1_petersen_decay_to_particulates.json")


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _orc(model):
    return Oracle(W.params_path(), rtol=RTOL, atol=W.atol_vector(RTOL), model=model)


@pytest.mark.parametrize("variant", [0, 1, 2, 3])
def test_variant_model_step_parity(torch_cuda, variant):
    """700 CSTR particles (10 full tiles and a ragged 60), three coupling
    intervals with warm starts; FP64 parity and equal accepted-step counts."""
    from paper_2311_08927_amd.adm1 import Context
    w = W.cstr_population(700, seed=41)
    ctx = Context(w.ld, rtol=RTOL, atol=W.atol_vector(RTOL), model=MODEL, variant=variant)
    assert ctx.model == MODEL
    worst, xg, xo, st, st_o, cnt, cnt_o = run_side_by_side(ctx, _orc(DESC), w, 3)
    ctx.close()
    print(f"variant {variant}: parity {worst:.3e}, accepted steps GPU "
          f"{cnt[0, :w.n].sum()} oracle {cnt_o[0, :w.n].sum()}")
    assert (st & 0x7F == 0).all() and (st_o & 0x7F == 0).all()
    assert worst <= PARITY_TOL
    assert np.array_equal(cnt[0, :w.n], cnt_o[0, :w.n])


def test_variant_model_is_in_effect(torch_cuda):
    """The variant's result is far from the standard matrix's: the composite
    pool X_xc, fed only by the inflow in the variant, ends lower."""
    from paper_2311_08927_amd.adm1 import Context
    from tests.gpu_common import parity
    w = W.cstr_population(128, seed=42)
    ctx = Context(w.ld, rtol=RTOL, atol=W.atol_vector(RTOL), model=MODEL)
    _, xg, _, _, _, _, _ = run_side_by_side(ctx, _orc(DESC), w, 2)
    ctx.close()
    _, _, xs, _, _, _, _ = run_side_by_side(
        Context(w.ld, rtol=RTOL, atol=W.atol_vector(RTOL)), _orc(None), w, 2)
    gap = parity(xg, xs, w.n)
    print(f"variant vs standard matrix after two intervals: {gap:.3e}")
    assert gap > 1e3 * PARITY_TOL
    X_XC = 12
    assert (xg[X_XC, :w.n] < xs[X_XC, :w.n]).mean() > 0.9


def test_surrogate_refuses_other_models(torch_cuda):
    from paper_2311_08927_amd import surrogate as S
    from paper_2311_08927_amd.adm1 import Context
    ctx = Context(64, rtol=RTOL, atol=W.atol_vector(RTOL), model=MODEL)
    with pytest.raises(ValueError, match="standard"):
        S.Surrogate(ctx, 64)
    ctx.close()


def test_variant_model_with_mixed_phases(torch_cuda):
    """The second model's library with the mixed active / sediment / inert
    population: FP64 parity against the oracle reading the same description
    with the same phase factors, equal step counts."""
    import torch
    from paper_2311_08927_amd.adm1 import Context
    from tests.gpu_common import DeviceWorkload, parity
    w = W.cstr_population(300, seed=43)
    ph = W.mixed_phases(w.n, seed=43, ld=w.ld)
    ctx = Context(w.ld, rtol=RTOL, atol=W.atol_vector(RTOL), model=MODEL)
    ctx.set_phase_kinetics(W.PHASE_KIN)
    dw = DeviceWorkload(w)
    dph = torch.from_numpy(ph).cuda()
    orc = _orc(DESC)
    Xo = w.X.copy()
    Ho, hlo = np.full(w.ld, -1.0), np.full(w.ld, -1.0)
    worst = 0.0
    for s in range(2):
        D = w.D_at(s)
        dw.set_D(D)
        ctx.step(dw.X, dw.T, dw.D, dw.fidx, dw.S_in, w.dt, n=w.n, H=dw.H, hlast=dw.hlast,
                 status=dw.status, nsteps=dw.nsteps, phase=dph)
        st_o, cnt_o = orc.step(Xo, w.T, D, w.fidx, w.feed, w.dt, H=Ho, hlast=hlo, n=w.n,
                               phase=ph, phase_kin=W.PHASE_KIN)
        torch.cuda.synchronize()
        worst = max(worst, parity(dw.X.cpu().numpy(), Xo, w.n))
        assert (dw.status.cpu().numpy() & 0x7F == 0).all() and (st_o & 0x7F == 0).all()
        assert np.array_equal(dw.nsteps[0, :w.n].cpu().numpy(), cnt_o[0, :w.n])
    ctx.close()
    print(f"second model with phases: parity {worst:.3e}")
    assert worst <= PARITY_TOL
