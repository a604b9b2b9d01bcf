"""FP32-rate experiment: rates and assembly in FP32 while the eq. 7 / eq. 8
solves and the Newton-matrix LU stay in FP64.  The report is per state entry;
the test prints it and checks it against the FP64 oracle on a seeded sample
of the batched workload (a report, not a parity claim: the bounds are loose
sanity limits)."""
from __future__ import annotations

import numpy as np
import pytest

from oracle.adm1 import Oracle
from paper_2311_08927_amd import workloads as W
from tests.gpu_common import DeviceWorkload, parity

pytestmark = pytest.mark.gpu
RTOL = 1e-8


def test_fp32_rate_report():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2311_08927_amd.adm1 import Context
    from paper_2311_08927_amd import precision as P
    full = W.batched_population(1 << 14, seed=2)
    rng = np.random.default_rng(11)
    w = W.subset(full, np.sort(rng.choice(full.n, 1024, replace=False)))
    steps = 3
    atol = W.atol_vector(RTOL)
    c64 = Context(w.ld, rtol=RTOL, atol=atol)
    c32 = Context(w.ld, rtol=RTOL, atol=atol, rate_precision=1)
    dw = DeviceWorkload(w)

    def D_at(s):
        return torch.from_numpy(w.D_at(s)).cuda()

    rep = P.fp32_rate_report(c64, c32, dw.X, dw.T, dw.D, dw.fidx, dw.S_in, w.dt, w.n,
                             steps=steps, D_at=D_at)
    print()
    print(P.format_report(rep))
    rhs = np.array(rep["rhs"])
    st = np.array(rep["state"])
    assert np.all(np.isfinite(rhs)) and np.all(np.isfinite(st))
    # FP32 rates: the right-hand side carries single-precision rounding
    assert np.median(rhs[:, 2]) < 1e-4
    # the integrated states stay within single-precision-driven error levels
    assert st[-1, :, 2].max() < 1e-3

    # the FP32-rate path against the FP64 oracle on the same sample
    orc = Oracle(W.params_path(), rtol=RTOL, atol=atol)
    Xo = w.X.copy()
    Ho = np.full(w.ld, -1.0)
    hlo = np.full(w.ld, -1.0)
    X32 = dw.X.clone()
    H32 = torch.full((w.n,), -1.0, dtype=torch.float64, device="cuda")
    h32 = H32.clone()
    for s in range(steps):
        c32.step(X32, dw.T, D_at(s), dw.fidx, dw.S_in, w.dt, n=w.n, H=H32, hlast=h32)
        orc.step(Xo, w.T, w.D_at(s), w.fidx, w.feed, w.dt, H=Ho, hlast=hlo, n=w.n)
    torch.cuda.synchronize()
    e = parity(X32.cpu().numpy(), Xo, w.n)
    print("FP32-rate path vs FP64 oracle, worst relative error:", e)
    assert np.isfinite(e) and e < 1e-2
