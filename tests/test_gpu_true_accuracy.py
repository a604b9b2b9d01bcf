"""True accuracy of the FP64 step: the HIP path at rtol 1e-8 against the
oracle in its reference mode (rtol 1e-12), beside the oracle's own rtol-1e-8
result.  The parity tests show the two implementations agree; this shows
how far both are from the solution of the DAE (sec. 2.2, eqs. 2 and 7-8)
over a day's first four coupling intervals of the CSTR population, cold
start included."""
from __future__ import annotations

import numpy as np
import pytest

from oracle.adm1 import Oracle
from paper_2311_08927_amd import workloads as W
from tests.gpu_common import DeviceWorkload, parity

pytestmark = pytest.mark.gpu

RTOL = 1e-8
RTOL_REF = 1e-12


def test_true_error_against_tight_oracle():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2311_08927_amd.adm1 import Context
    w = W.cstr_population(128, seed=7)
    ctx = Context(w.ld, rtol=RTOL, atol=W.atol_vector(RTOL))
    dw = DeviceWorkload(w)
    orcs = {rt: Oracle(W.params_path(), rtol=rt, atol=W.atol_vector(rt)) for rt in (RTOL, RTOL_REF)}
    Xo = {rt: w.X.copy() for rt in orcs}
    Ho = {rt: np.full(w.ld, -1.0) for rt in orcs}
    hlo = {rt: np.full(w.ld, -1.0) for rt in orcs}
    for s in range(4):
        D = w.D_at(s)
        dw.set_D(D)
        ctx.step(dw.X, dw.T, dw.D, dw.fidx, dw.S_in, w.dt, n=w.n, H=dw.H, hlast=dw.hlast,
                 status=dw.status, nsteps=dw.nsteps)
        for rt, o in orcs.items():
            st, _ = o.step(Xo[rt], w.T, D, w.fidx, w.feed, w.dt, H=Ho[rt], hlast=hlo[rt], n=w.n)
            assert (st & 0x7F == 0).all()
        torch.cuda.synchronize()
        assert (dw.status.cpu().numpy() & 0x7F == 0).all()
        xg = dw.X.cpu().numpy()
        true_gpu = parity(xg, Xo[RTOL_REF], w.n)
        true_orc = parity(Xo[RTOL], Xo[RTOL_REF], w.n)
        par = parity(xg, Xo[RTOL], w.n)
        print(f"interval {s}: true error GPU {true_gpu:.3e}, oracle at rtol {RTOL:g} "
              f"{true_orc:.3e}; GPU vs that oracle {par:.3e}")
        # the integration error stays near the tolerance (proportionality),
        # and the GPU's is the oracle's up to their mutual agreement
        assert true_gpu <= 1e-7
        assert abs(true_gpu - true_orc) <= par + 1e-15
    ctx.close()
