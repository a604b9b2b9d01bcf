"""Timing of the coupling driver's kernels on the digester field.

Between two coupling steps every particle is displaced by the flow (it
follows its fluid particle, sec. 2.3), the inlet feed mask is rebuilt from
the new positions, and (optionally) the soluble entries diffuse between
neighbouring particles.  `python -m paper_2311_08927_amd.coupling` times
adm1_advect (one coupling interval of 1/96 d in the field's 0.25 s substeps),
adm1_feed_mask and adm1_diffuse (grid build plus one explicit step of
molecular diffusion, h = 1.3 x the mean particle spacing) on the field's
seeded positions and states with HIP events on the launching stream, and
prints one line per call.
"""
from __future__ import annotations

import argparse

import numpy as np

from . import adm1 as A
from . import workloads as W


def main():
    import torch
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--n", type=int, default=1 << 24)
    ap.add_argument("--reps", type=int, default=3)
    args = ap.parse_args()
    n = args.n
    pos = W.cylinder_positions(n, seed=3)
    ld = pos.shape[1]
    d = torch.from_numpy(np.ascontiguousarray(pos)).cuda()
    flow = A.make_flow(W.flow_field(3))
    D = torch.empty(n, dtype=torch.float64, device="cuda")
    fidx = torch.empty(n, dtype=torch.int32, device="cuda")
    dt_s = W.DT * 86400.0
    sub = W.advect_substeps(dt_s)
    stream = torch.cuda.current_stream()

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.reps):
            fn()
        e1.record(stream)
        e1.synchronize()
        return e0.elapsed_time(e1) / args.reps

    ms = timed(lambda: A.adm1_advect(d, ld, n, flow, dt_s, sub))
    print(f"adm1_advect: {n} particles, {sub} RK4 substeps: {ms:.2f} ms per call, "
          f"{n * sub / ms / 1e6:.1f} G particle-substeps/s", flush=True)
    ms = timed(lambda: A.adm1_feed_mask(d, ld, n, W.INLET_Z, W.INLET_R, 1.0, 1, 0, D, fidx))
    print(f"adm1_feed_mask: {n} particles: {ms:.3f} ms per call, "
          f"{n * 24 / ms / 1e6:.1f} GB/s (12 B read, 12 B written per particle)", flush=True)
    del D, fidx
    V_p = np.pi * W.TANK_R ** 2 * W.TANK_H / n
    h = 1.3 * V_p ** (1.0 / 3.0)
    grid = A.Grid(A.make_diffusion(h, 1e-9 * 86400.0, V_p, [-W.TANK_R, -W.TANK_R, 0.0],
                                   [W.TANK_R, W.TANK_R, W.TANK_H]), ld)
    X = torch.from_numpy(W.perturbed_states(n, 3, ld=ld)).cuda()
    cnt = torch.zeros(n, dtype=torch.int32, device="cuda")
    grid.diffuse(X, d, n, W.DT / 8, 1, cnt)
    nb = cnt.double().mean().item()
    ms = timed(lambda: grid.diffuse(X, d, n, W.DT / 8, 1))
    print(f"adm1_diffuse: {n} particles, h = {h * 1e3:.2f} mm, {nb:.1f} neighbours per "
          f"particle: {ms:.2f} ms per call (grid build + one explicit step), "
          f"{n * nb / ms / 1e6:.1f} G neighbour pairs/s", flush=True)
    grid.close()


if __name__ == "__main__":
    main()
