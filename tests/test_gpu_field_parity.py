"""FP64 parity on the lab-digester field (sec. 3.2, Table 2 case): the
coupling loop of sec. 2.3 as the coupling driver runs it on the GPU (inlet feed mask,
adaptive step with warm starts, advection between intervals), and a seeded
sample of particles, inlet ones included, recomputed by the oracle with the
feed each of them received in each interval.  Also one cold interval of the
2^24-particle field (the size of the gated-surrogate comparison)."""
from __future__ import annotations

import numpy as np
import pytest

from oracle.adm1 import Oracle
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


@pytest.fixture(scope="module")
def orc():
    return Oracle(W.params_path(), rtol=RTOL, atol=W.atol_vector(RTOL))


def inlet(pos: np.ndarray) -> np.ndarray:
    """Inlet membership of float32 positions [3][n] (the recipe's region)."""
    r = np.hypot(pos[0].astype(np.float64), pos[1].astype(np.float64))
    return (pos[2] >= W.INLET_Z) & (r <= W.INLET_R)


def sample(n: int, pos: np.ndarray, seed: int, n_inlet=24, n_other=70) -> np.ndarray:
    rng = np.random.default_rng(seed)
    ins = np.flatnonzero(inlet(pos[:, :n]))
    idx = np.concatenate([rng.choice(ins, min(n_inlet, ins.size), replace=False),
                          rng.choice(n, n_other, replace=False), [0, n - 1]])
    return np.unique(idx)


def run_field(torch, w, intervals, idx):
    """The coupling loop on the GPU over the whole field; returns per interval
    the sampled particles' states after the step, their D and feed rows
    during it, and their accepted-step counts."""
    from paper_2311_08927_amd import adm1 as A
    dev = "cuda"
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)  # noqa: E731
    ctx = A.Context(w.ld, rtol=RTOL, atol=W.atol_vector(RTOL))
    X, T, S_in, pos = t(w.X), t(w.T), t(w.feed), t(w.extra["pos"])
    flow = A.make_flow(w.extra["flow"])
    D = torch.zeros(w.n, dtype=torch.float64, device=dev)
    fidx = torch.zeros(w.n, dtype=torch.int32, device=dev)
    H = torch.full((w.n,), -1.0, dtype=torch.float64, device=dev)
    hl = torch.full((w.n,), -1.0, dtype=torch.float64, device=dev)
    status = torch.zeros(w.n, dtype=torch.uint8, device=dev)
    nsteps = torch.zeros((3, w.ld), dtype=torch.int32, device=dev)
    it = t(idx)
    dt_s = w.dt * 86400.0
    out = []
    for k in range(intervals):
        A.adm1_feed_mask(pos, w.ld, w.n, W.INLET_Z, W.INLET_R, 1.0, 1, 0, D, fidx)
        Dk, fk = D.index_select(0, it).cpu().numpy(), fidx.index_select(0, it).cpu().numpy()
        ctx.step(X, T, D, fidx, S_in, w.dt, n=w.n, H=H, hlast=hl, status=status,
                 nsteps=nsteps)
        if k + 1 < intervals:
            A.adm1_advect(pos, w.ld, w.n, flow, dt_s, W.advect_substeps(dt_s))
        torch.cuda.synchronize()
        st = status.cpu().numpy()
        out.append(dict(X=X.index_select(1, it).cpu().numpy(), D=Dk, fidx=fk,
                        acc=nsteps[0].index_select(0, it).cpu().numpy(),
                        status_counts=np.bincount(st & 0x7F, minlength=5),
                        fed=int((D > 0).sum())))
    ctx.close()
    return out


def test_field_2e22_three_intervals_sampled(torch_cuda, orc):
    """2^22 field particles, three coupling intervals (cold, then warm starts,
    particles moved by the flow in between, inlet membership re-evaluated at
    every interval start); 96 sampled particles, a quarter of them in the
    inlet at the start, integrated by the oracle with the same per-interval
    feed: parity at every interval end and equal accepted-step counts."""
    torch = torch_cuda
    w = W.digester_field(1 << 22, seed=3, steps=3)
    idx = sample(w.n, w.extra["pos"], seed=31)
    gpu = run_field(torch, w, 3, idx)
    sub = W.subset(w, idx)
    Xo = sub.X.copy()
    Ho = np.full(sub.ld, -1.0)
    hlo = np.full(sub.ld, -1.0)
    fed_sampled = 0
    for k, g in enumerate(gpu):
        assert (g["status_counts"][1:] == 0).all(), g["status_counts"]
        st_o, cnt_o = orc.step(Xo, sub.T, g["D"], g["fidx"], sub.feed, sub.dt, H=Ho,
                               hlast=hlo, n=sub.n)
        assert (st_o & 0x7F == 0).all()
        err = parity(g["X"], Xo, sub.n)
        same = np.array_equal(g["acc"], cnt_o[0, :sub.n])
        fed_sampled += int((g["D"] > 0).sum())
        print(f"interval {k}: {g['fed']} particles fed ({int((g['D'] > 0).sum())} sampled), "
              f"parity {err:.3e}, accepted steps GPU {g['acc'].sum()} oracle "
              f"{cnt_o[0, :sub.n].sum()}")
        assert err <= PARITY_TOL
        assert same
        assert g["fed"] > 0
    assert fed_sampled >= 20  # the inlet particles were really fed


def test_field_2e24_cold_interval_sampled(torch_cuda, orc):
    """The 2^24-particle field (the gated-surrogate comparison's size), one
    cold coupling interval with the inlet feed; 96 sampled particles
    recomputed by the oracle."""
    torch = torch_cuda
    w = W.digester_field(1 << 24, seed=3, steps=1)
    idx = sample(w.n, w.extra["pos"], seed=32)
    g = run_field(torch, w, 1, idx)[0]
    assert (g["status_counts"][1:] == 0).all(), g["status_counts"]
    sub = W.subset(w, idx)
    Xo = sub.X.copy()
    st_o, cnt_o = orc.step(Xo, sub.T, g["D"], g["fidx"], sub.feed, sub.dt, n=sub.n)
    assert (st_o & 0x7F == 0).all()
    err = parity(g["X"], Xo, sub.n)
    print(f"2^24 field, cold interval: {g['fed']} fed, parity {err:.3e}, accepted steps "
          f"GPU {g['acc'].sum()} oracle {cnt_o[0, :sub.n].sum()}")
    assert err <= PARITY_TOL
    assert np.array_equal(g["acc"], cnt_o[0, :sub.n])
    assert int((g["D"] > 0).sum()) >= 20
