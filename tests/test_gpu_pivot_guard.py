"""Growth guard of the static-order factorisations of the bordered Newton
matrix (eqs. 7-8 bordering the eq. 2 rows).  The elimination order is fixed
at build time and does not pivot; the guard rejects an attempted step whose
factorisation has a pivot below `pivot_floor` times its row's diagonal
entry before elimination, so the step size shrinks (a smaller step makes
the matrix I/(gamma h) - J more diagonally dominant).  On the workloads the
pivots stay far above any such floor: the guard at 1e-2 never fires and the
results are bit-identical to the unguarded factorisation.  A floor no
pivot can meet rejects every attempt: the particles fail with status 2
(step underflow) and keep their input states."""
from __future__ import annotations

import numpy as np
import pytest

from paper_2311_08927_amd import workloads as W
from tests.gpu_common import DeviceWorkload

pytestmark = pytest.mark.gpu

RTOL = 1e-8
STATIC = [1, 2, 3]  # sparse LU one lane, two lanes, one lane with the matrix in LDS


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _run(w, variant, floor, steps):
    import torch
    from paper_2311_08927_amd.adm1 import Context
    ctx = Context(w.ld, rtol=RTOL, atol=W.atol_vector(RTOL), variant=variant, pivot_floor=floor)
    dw = DeviceWorkload(w)
    for s in range(steps):
        dw.set_D(w.D_at(s))
        ctx.step(dw.X, dw.T, dw.D, dw.fidx, dw.S_in, w.dt, n=w.n, H=dw.H, hlast=dw.hlast,
                 status=dw.status, nsteps=dw.nsteps)
    torch.cuda.synchronize()
    out = (dw.X.cpu().numpy(), dw.status.cpu().numpy(), dw.nsteps.cpu().numpy())
    ctx.close()
    return out


@pytest.mark.parametrize("variant", STATIC)
def test_guard_silent_on_the_batched_population(torch_cuda, variant):
    """4,096 particles of the batched population (feed-zone pulses, 30-40 C),
    the cold interval and two warm ones."""
    w = W.subset(W.batched_population(1 << 20, seed=2), np.arange(0, 1 << 20, 256))
    x0, s0, n0 = _run(w, variant, 0.0, 3)
    x1, s1, n1 = _run(w, variant, 1e-2, 3)
    assert (s0 & 0x7F == 0).all()
    assert np.array_equal(x0[:, :w.n], x1[:, :w.n])
    assert np.array_equal(n0[:, :w.n], n1[:, :w.n])


@pytest.mark.parametrize("variant", STATIC)
def test_guard_rejects_when_no_pivot_can_pass(torch_cuda, variant):
    w = W.cstr_population(200, seed=5)
    x, st, ns = _run(w, variant, 1e300, 1)
    assert ((st & 0x7F) == 2).all()
    assert (ns[0, :w.n] == 0).all() and (ns[1, :w.n] > 0).all()
    assert np.array_equal(x[:, :w.n], w.X[:, :w.n])


def test_default_floor_and_validation(torch_cuda):
    from paper_2311_08927_amd import adm1 as A
    assert A.make_opts().pivot_floor == A.PIVOT_FLOOR
    for bad in (-1.0, float("nan"), float("inf")):
        with pytest.raises(A.ADM1Error):
            A.Context(64, rtol=RTOL, atol=W.atol_vector(RTOL), pivot_floor=bad)


def test_floor_changed_on_a_live_context(torch_cuda):
    """adm1_set_opts updates the device copy the two-lane kernel reads: an
    impossible floor fails every particle, the default one restores the
    normal step on the same inputs."""
    import torch
    from paper_2311_08927_amd import adm1 as A
    w = W.cstr_population(128, seed=6)
    ctx = A.Context(w.ld, rtol=RTOL, atol=W.atol_vector(RTOL), variant=2)
    for floor, want in ((1e300, 2), (A.PIVOT_FLOOR, 0)):
        ctx.set_opts(pivot_floor=floor)
        assert ctx.opts.pivot_floor == floor
        dw = DeviceWorkload(w)
        ctx.step(dw.X, dw.T, dw.D, dw.fidx, dw.S_in, w.dt, n=w.n, H=dw.H, hlast=dw.hlast,
                 status=dw.status, nsteps=dw.nsteps)
        torch.cuda.synchronize()
        assert ((dw.status.cpu().numpy() & 0x7F) == want).all(), floor
    ctx.close()
