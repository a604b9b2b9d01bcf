"""The no-allocation step (adm1_step_particles_static) against the step with
context scratch (adm1_step_particles): two calls in a row on one device, the
second smaller and warm-started (cost-ordered queue), through the C ABI."""
from __future__ import annotations

import numpy as np
import pytest

from paper_2311_08927_amd import workloads as W
from tests.gpu_common import PARITY_TOL, parity

pytestmark = pytest.mark.gpu

RTOL = 1e-8


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _run(A, ctx, fn, X, T, D, fidx, S_in, H, hl, n, dt):
    import torch
    status = torch.zeros(n, dtype=torch.uint8, device="cuda")
    nsteps = torch.zeros((3, X.shape[1]), dtype=torch.int32, device="cuda")
    feed = A.feed_struct(D, fidx, S_in)
    aux = A.adm1_aux(H.data_ptr(), hl.data_ptr())
    fn(ctx.handle, X, X.shape[1], T, feed, dt, n, aux, status, nsteps)
    torch.cuda.synchronize()
    return status, nsteps, A.adm1_last_failures(ctx.handle)


def test_static_step_matches_context_step(torch_cuda):
    torch = torch_cuda
    from paper_2311_08927_amd import adm1 as A
    w = W.batched_population(1000, seed=2, steps=2)
    ctx = A.Context(w.ld, rtol=RTOL, atol=W.atol_vector(RTOL))
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda")  # noqa: E731
    T, fidx, S_in = t(w.T), t(w.fidx), t(w.feed)
    sides = {}
    for name, fn in [("ctx", A.adm1_step_particles), ("static", A.adm1_step_particles_static)]:
        X = t(w.X)
        H = torch.full((w.ld,), -1.0, dtype=torch.float64, device="cuda")
        hl = torch.full((w.ld,), -1.0, dtype=torch.float64, device="cuda")
        out = []
        # first call: 1000 particles, cold start; second call: the first 600
        # of them, warm-started (the queue is cost ordered from h_last)
        for k, n in enumerate([w.n, 600]):
            st, ns, fails = _run(A, ctx, fn, X, T, t(w.D_at(k)), fidx, S_in, H, hl, n, w.dt)
            out.append((X.clone(), st, ns, H.clone(), hl.clone(), fails))
        sides[name] = out
    for k, n in enumerate([w.n, 600]):
        Xc, stc, nsc, Hc, hlc, fc = sides["ctx"][k]
        Xs, sts, nss, Hs, hls, fs = sides["static"][k]
        err = parity(Xs.cpu().numpy(), Xc.cpu().numpy(), n)
        print(f"call {k}: n={n}, parity static vs context {err:.3e}, failures {fs}")
        assert err <= PARITY_TOL
        # same kernels on the same inputs: the results are bit for bit equal
        assert torch.equal(Xs, Xc) and torch.equal(Hs, Hc) and torch.equal(hls, hlc)
        assert torch.equal(sts, stc) and torch.equal(nss, nsc)
        assert fs == fc and fs["counted"] == n and fs["failed"] == 0
        assert int(nss[0, :n].min()) > 0


def test_static_step_rejects_more_than_its_capacity(torch_cuda):
    torch = torch_cuda
    from paper_2311_08927_amd import adm1 as A
    n = A.STATIC_MAX_N + 1
    ld = W.pad_ld(n, 64)
    ctx = A.Context(ld, rtol=RTOL, atol=W.atol_vector(RTOL))
    X = torch.zeros((35, ld), dtype=torch.float64, device="cuda")
    T = torch.full((ld,), 308.15, dtype=torch.float64, device="cuda")
    D = torch.zeros(ld, dtype=torch.float64, device="cuda")
    fidx = torch.zeros(ld, dtype=torch.int32, device="cuda")
    S_in = torch.zeros((1, 26), dtype=torch.float64, device="cuda")
    status = torch.full((ld,), 7, dtype=torch.uint8, device="cuda")
    feed = A.feed_struct(D, fidx, S_in)
    rc = A.adm1_step_particles_static(ctx.handle, X, ld, T, feed, 1.0 / 96, n, None, status,
                                      None, check=False)
    assert rc == -11 and "ADM1_STATIC_MAX_N" in A.strerror(rc)
    torch.cuda.synchronize()
    assert int(status.min()) == 7  # nothing was enqueued
