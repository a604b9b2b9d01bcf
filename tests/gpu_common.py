"""Helpers shared by the GPU tests: device copies of a workload, running the
HIP step and the oracle side by side, and the parity metric.

Parity metric (one number per comparison): max over particles and entries of
|x_gpu - x_oracle| / max(|x_oracle|, 1e-4 x_nom), x_nom the nominal state.
"""
from __future__ import annotations

import numpy as np

from paper_2311_08927_amd import workloads as W

PARITY_TOL = 1e-6


def parity(xg: np.ndarray, xo: np.ndarray, n: int) -> float:
    nom = W.nominal()["state"][:, None]
    den = np.maximum(np.abs(xo[:, :n]), 1e-4 * nom)
    return float(np.max(np.abs(xg[:, :n] - xo[:, :n]) / den))


class DeviceWorkload:
    """torch device copies of a workload's arrays."""

    def __init__(self, w: W.Workload, device="cuda:0"):
        import torch
        self.w = w
        self.dev = device
        self.X = torch.from_numpy(np.ascontiguousarray(w.X)).to(device)
        self.T = torch.from_numpy(np.ascontiguousarray(w.T)).to(device)
        self.D = torch.from_numpy(np.ascontiguousarray(w.D)).to(device)
        self.fidx = torch.from_numpy(np.ascontiguousarray(w.fidx)).to(device)
        self.S_in = torch.from_numpy(np.ascontiguousarray(w.feed)).to(device)
        self.H = torch.full((w.n,), -1.0, dtype=torch.float64, device=device)
        self.hlast = torch.full((w.n,), -1.0, dtype=torch.float64, device=device)
        self.status = torch.zeros(w.n, dtype=torch.uint8, device=device)
        self.nsteps = torch.zeros((3, w.ld), dtype=torch.int32, device=device)

    def set_D(self, D: np.ndarray):
        self.D.copy_(__import__("torch").from_numpy(np.ascontiguousarray(D)))


def run_side_by_side(ctx, orc, w: W.Workload, steps: int, nthreads=None, check_each=True):
    """Advance w on the GPU and on the oracle for `steps` coupling intervals;
    returns (worst parity, GPU state, oracle state, GPU status, oracle status,
    GPU counts, oracle counts)."""
    import torch
    dw = DeviceWorkload(w)
    Xo = w.X.copy()
    Ho = np.full(w.ld, -1.0)
    hlo = np.full(w.ld, -1.0)
    worst = 0.0
    st_o = None
    cnt_o = None
    for s in range(steps):
        D = w.D_at(s)
        dw.set_D(D)
        ctx.step(dw.X, dw.T, dw.D, dw.fidx, dw.S_in, w.dt, n=w.n, H=dw.H, hlast=dw.hlast,
                 status=dw.status, nsteps=dw.nsteps)
        st_o, cnt_o = orc.step(Xo, w.T, D, w.fidx, w.feed, w.dt, H=Ho, hlast=hlo, n=w.n,
                               nthreads=nthreads)
        torch.cuda.synchronize()
        if check_each or s == steps - 1:
            xg = dw.X.cpu().numpy()
            worst = max(worst, parity(xg, Xo, w.n))
    return (worst, dw.X.cpu().numpy(), Xo, dw.status.cpu().numpy(), st_o,
            dw.nsteps.cpu().numpy(), cnt_o)
