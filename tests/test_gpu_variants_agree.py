"""The four Newton-matrix layouts of the FP64 step agree with one another at
a size the oracle cannot follow: 65,536 particles of the batched population
(feed-zone pulses, 30-40 C), the cold interval and two warm ones.  The dense
layout factorises with partial pivoting, the three others in the static
order; every pair of layouts must agree to well inside the oracle parity
bar, with (nearly) the same accepted-step counts, since they differ only in
the rounding of the linear algebra."""
from __future__ import annotations

import numpy as np
import pytest

from paper_2311_08927_amd import workloads as W
from tests.gpu_common import DeviceWorkload, parity

pytestmark = pytest.mark.gpu

RTOL = 1e-8


def _run(w, variant, steps):
    import torch
    from paper_2311_08927_amd.adm1 import Context
    ctx = Context(w.ld, rtol=RTOL, atol=W.atol_vector(RTOL), variant=variant)
    dw = DeviceWorkload(w)
    acc = np.zeros(w.n, dtype=np.int64)
    for s in range(steps):
        dw.set_D(w.D_at(s))
        ctx.step(dw.X, dw.T, dw.D, dw.fidx, dw.S_in, w.dt, n=w.n, H=dw.H, hlast=dw.hlast,
                 status=dw.status, nsteps=dw.nsteps)
        torch.cuda.synchronize()
        acc += dw.nsteps[0, :w.n].cpu().numpy()
    out = dw.X.cpu().numpy(), dw.status.cpu().numpy(), acc
    ctx.close()
    return out


def test_layouts_agree_on_65536_particles():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    w = W.subset(W.batched_population(1 << 20, seed=2), np.arange(0, 1 << 20, 16))
    res = {v: _run(w, v, 3) for v in (0, 1, 2, 3)}
    for v, (x, st, acc) in res.items():
        assert (st & 0x7F == 0).all(), v
    for a in (0, 1, 2):
        for b in range(a + 1, 4):
            xa, _, na = res[a]
            xb, _, nb = res[b]
            gap = parity(xa, xb, w.n)
            same = float(np.mean(na == nb))
            print(f"layouts {a} and {b}: max rel diff {gap:.2e}, equal step counts {same:.5f}")
            assert gap <= 1e-8
            assert same >= 0.999
