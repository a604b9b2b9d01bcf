"""GPU parity of the paper's fixed-step explicit scheme (adm1_step_fixed,
sec. 2.3 and 4.3) against the oracle's fixed-step integrator, particle by
particle, through the C ABI; argument errors and failure handling."""
from __future__ import annotations

import numpy as np
import pytest

from oracle.adm1 import Oracle
from paper_2311_08927_amd import workloads as W
from tests.gpu_common import PARITY_TOL, DeviceWorkload, parity

pytestmark = pytest.mark.gpu

SEC = 1.0 / 86400.0
RTOL = 1e-8


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def orc():
    return Oracle(W.params_path(), rtol=RTOL, atol=W.atol_vector(RTOL))


def make_ctx(n_max):
    from paper_2311_08927_amd.adm1 import Context
    return Context(n_max, rtol=RTOL, atol=W.atol_vector(RTOL))


def oracle_fixed(orc, w, X, D, dt, substeps, method, idx):
    """Oracle result per particle of idx (None where the oracle fails)."""
    out = {}
    for i in idx:
        try:
            out[i] = orc.fixed(X[:, i], w.T[i], D[i], w.feed[w.fidx[i]], dt, substeps, method)
        except RuntimeError:
            out[i] = None
    return out


def method_code(method):
    from paper_2311_08927_amd import adm1 as A
    return {"euler": A.FIXED_EULER, "rk4": A.FIXED_RK4}[method]


@pytest.mark.parametrize("method,dt,substeps", [
    ("euler", 0.5 * SEC, 10),     # the paper's coupling interval (sec. 4.3)
    ("rk4", 0.5 * SEC, 10),
    ("euler", 60 * SEC, 600),
    ("rk4", 900 * SEC, 90),       # one 1/96-d interval in 10 s steps
])
def test_fixed_parity_cstr(torch_cuda, orc, method, dt, substeps):
    """CSTR population, 200 particles (three full 64-particle tiles and a
    ragged tail)."""
    w = W.cstr_population(200, seed=13)
    ctx = make_ctx(w.ld)
    dw = DeviceWorkload(w)
    newton = torch_cuda.zeros(w.n, dtype=torch_cuda.int32, device="cuda")
    ctx.step_fixed(dw.X, dw.T, dw.D, dw.fidx, dw.S_in, dt, substeps, method_code(method),
                   n=w.n, H=dw.H, status=dw.status, newton=newton)
    torch_cuda.cuda.synchronize()
    st = dw.status.cpu().numpy()
    assert (st == 0).all(), np.unique(st)
    assert (newton.cpu().numpy() > 0).all()
    ref = oracle_fixed(orc, w, w.X, w.D, dt, substeps, method, range(w.n))
    Xo = w.X.copy()
    for i, y in ref.items():
        assert y is not None
        Xo[:, i] = y
    p = parity(dw.X.cpu().numpy(), Xo, w.n)
    print(f"fixed {method} dt={dt / SEC:g} s x{substeps}: parity {p:.2e}")
    assert p < PARITY_TOL
    # the roots handed back are those of the final state
    H = dw.H.cpu().numpy()
    assert np.all(np.isfinite(H)) and np.all(H > 0)


def test_fixed_intervals_with_warm_start(torch_cuda, orc):
    """Batched population (per-particle temperature, pulsed feed zone): three
    coupling intervals of the paper's shape, S_H+ carried between them."""
    w = W.batched_population(1000, seed=7)
    ctx = make_ctx(w.ld)
    dw = DeviceWorkload(w)
    Xo = w.X.copy()
    dt, sub = 0.5 * SEC, 10
    for s in range(3):
        D = w.D_at(s)
        dw.set_D(D)
        ctx.step_fixed(dw.X, dw.T, dw.D, dw.fidx, dw.S_in, dt, sub, method_code("euler"),
                       n=w.n, H=dw.H, status=dw.status)
        ref = oracle_fixed(orc, w, Xo, D, dt, sub, "euler", range(w.n))
        for i, y in ref.items():
            Xo[:, i] = y
        torch_cuda.cuda.synchronize()
        assert (dw.status.cpu().numpy() == 0).all()
    p = parity(dw.X.cpu().numpy(), Xo, w.n)
    print(f"three intervals: parity {p:.2e}")
    assert p < PARITY_TOL


def test_fixed_paper_workload_sampled(torch_cuda, orc):
    """The paper's parallel benchmark shape (sec. 4.3): 110,929 CSTR
    particles, Dt = 0.5 s in ten explicit steps; 64 seeded particles
    recomputed by the oracle."""
    n = 110_929
    w = W.cstr_population(n, seed=1)
    ctx = make_ctx(w.ld)
    dw = DeviceWorkload(w)
    ctx.step_fixed(dw.X, dw.T, dw.D, dw.fidx, dw.S_in, 0.5 * SEC, 10, method_code("euler"),
                   n=n, H=dw.H, status=dw.status)
    torch_cuda.cuda.synchronize()
    st = dw.status.cpu().numpy()
    assert (st == 0).all()
    idx = np.sort(np.random.default_rng(5).choice(n, 64, replace=False))
    idx[-1] = n - 1
    ref = oracle_fixed(orc, w, w.X, w.D, 0.5 * SEC, 10, "euler", idx)
    xg = dw.X.cpu().numpy()
    Xo = np.stack([ref[i] for i in idx], axis=1)
    p = parity(xg[:, idx], Xo, len(idx))
    print(f"paper workload, 64 sampled: parity {p:.2e}")
    assert p < PARITY_TOL


def test_fixed_too_long_step_fails_and_keeps_input(torch_cuda, orc):
    """One explicit step over a whole day drives particles out of the
    model's domain (negative concentrations).  A particle that fails on the
    GPU keeps its input; where both sides advance a particle the results
    agree.  On negative totals the eq.-7 solves of the two independent
    implementations may draw the failure line differently (either side may
    still find a root where the other gives up), so only the particles both
    advance are compared."""
    w = W.cstr_population(16, seed=13)
    ctx = make_ctx(w.ld)
    dw = DeviceWorkload(w)
    ctx.step_fixed(dw.X, dw.T, dw.D, dw.fidx, dw.S_in, 1.0, 1, method_code("euler"), n=w.n,
                   status=dw.status)
    torch_cuda.cuda.synchronize()
    st = dw.status.cpu().numpy()
    xg = dw.X.cpu().numpy()
    ref = oracle_fixed(orc, w, w.X, w.D, 1.0, 1, "euler", range(w.n))
    n_both = n_fail = 0
    for i, y in ref.items():
        if (st[i] & 0x7F) != 0:
            n_fail += 1
            assert (st[i] & 0x7F) in (1, 2), (i, st[i])
            assert np.array_equal(xg[:, i], w.X[:, i])
        elif y is not None:
            n_both += 1
            assert parity(xg[:, i:i + 1], y[:, None], 1) < PARITY_TOL
            assert bool(st[i] & 0x80) == bool((y[:26] < 0).any() or (y[32:] < 0).any())
    print(f"one-day Euler step: GPU failed {n_fail}, oracle failed "
          f"{sum(y is None for y in ref.values())}, both advanced {n_both} of {w.n}")
    assert n_fail > 0 and n_both > 0


def test_fixed_invalid_input_and_arguments(torch_cuda):
    from paper_2311_08927_amd import adm1 as A
    w = W.cstr_population(100, seed=3)
    ctx = make_ctx(w.ld)
    dw = DeviceWorkload(w)
    dw.X[5, 3] = float("nan")
    dw.T[7] = -1.0
    x0 = dw.X.cpu().numpy()
    ctx.step_fixed(dw.X, dw.T, dw.D, dw.fidx, dw.S_in, 0.5 * SEC, 10, n=w.n, status=dw.status)
    torch_cuda.cuda.synchronize()
    st = dw.status.cpu().numpy()
    assert st[3] == 4 and st[7] == 4
    ok = np.ones(w.n, bool)
    ok[[3, 7]] = False
    assert (st[ok] == 0).all()
    x1 = dw.X.cpu().numpy()
    assert np.array_equal(x1[:, [3, 7]], x0[:, [3, 7]], equal_nan=True)
    feed = A.feed_struct(dw.D, dw.fidx, dw.S_in)
    h, ld = ctx.handle, w.ld

    def rc(**kw):
        a = dict(dt=0.5 * SEC, sub=10, method=0, n=w.n, status=dw.status)
        a.update(kw)
        return A.adm1_step_fixed(h, dw.X, ld, dw.T, feed, a["dt"], a["sub"], a["method"],
                                 a["n"], None, a["status"], None, None, check=False)

    assert rc(sub=0) == -5 and rc(sub=(1 << 20) + 1) == -5
    assert rc(method=2) == -5 and rc(method=-1) == -5
    assert rc(dt=0.0) == -9 and rc(dt=float("inf")) == -9
    assert rc(status=None) == -1
    assert rc(n=w.ld + 1) == -2
    assert rc(n=0) == 0
    x2 = dw.X.cpu().numpy()
    assert np.array_equal(x2, x1, equal_nan=True)
