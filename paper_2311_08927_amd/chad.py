"""The CHAD coupling loop on one GPU (sec. 2.3), end to end.

Every coupling interval: the inlet feed mask is rebuilt from the particle
positions, every particle's ADM1 state is advanced (the adaptive FP64 step,
or the paper's fixed-step explicit scheme), the soluble entries optionally
diffuse between neighbouring particles, the tank gas flows are reduced, and
the particles move with the flow to their next positions (the seeded
analytic field standing in for the SPH solver).  Optionally a binary
snapshot of positions and states is written per interval, and a run can
resume from one (`--resume`).  All arrays stay
in HBM; only the four gas totals come back to the host.

    python -m paper_2311_08927_amd.chad --n 4194304 --steps 10 \\
        [--scheme adaptive|fixed] [--diffusion 1e-9] [--snapshot-dir DIR] [--resume FILE]

prints the time of every stage per interval and the tank methane flow.
"""
from __future__ import annotations

import argparse
import os
import sys

import numpy as np

from . import adm1 as A
from . import workloads as W


class Loop:
    """State and kernels of one coupled run on the digester field."""

    def __init__(self, n, seed=3, scheme="adaptive", rtol=1e-8, substeps=10,
                 diffusion=0.0, diffusion_substeps=None):
        import torch
        self.torch = torch
        w = W.digester_field(n, seed=seed, steps=1)
        self.w, self.n, self.ld = w, n, w.ld
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
        self.X, self.T, self.S_in = t(w.X), t(w.T), t(w.feed)
        self.pos = t(w.extra["pos"])
        self.V = torch.full((n,), w.extra["V_p"], dtype=torch.float64, device="cuda")
        self.D = torch.zeros(n, dtype=torch.float64, device="cuda")
        self.fidx = torch.zeros(n, dtype=torch.int32, device="cuda")
        self.H = torch.full((n,), -1.0, dtype=torch.float64, device="cuda")
        self.hl = torch.full((n,), -1.0, dtype=torch.float64, device="cuda")
        self.status = torch.zeros(n, dtype=torch.uint8, device="cuda")
        self.tot = torch.zeros(4, dtype=torch.float64, device="cuda")
        self.flow = A.make_flow(w.extra["flow"])
        self.ctx = A.Context(w.ld, rtol=rtol, atol=W.atol_vector(rtol))
        self.scheme, self.substeps = scheme, substeps
        self.grid = None
        if diffusion > 0.0:
            V_p = w.extra["V_p"]
            self.grid = A.Grid(A.make_diffusion(1.3 * V_p ** (1 / 3), diffusion * 86400.0, V_p,
                                                [-W.TANK_R, -W.TANK_R, 0.0],
                                                [W.TANK_R, W.TANK_R, W.TANK_H]), w.ld)
        self.dt = w.dt
        if self.grid is not None:
            # explicit diffusion substeps within the stability bound unless given
            self.diffusion_substeps = (diffusion_substeps if diffusion_substeps
                                       else self.grid.stable_substeps(self.dt))

    def interval(self, events=None):
        """One coupling interval; `events` (optional dict name -> (start,
        end) CUDA events) brackets each stage."""

        def stage(name, fn):
            if events is not None:
                events[name][0].record()
            fn()
            if events is not None:
                events[name][1].record()

        stage("feed mask", lambda: A.adm1_feed_mask(self.pos, self.ld, self.n, W.INLET_Z,
                                                     W.INLET_R, 1.0, 1, 0, self.D, self.fidx))
        if self.scheme == "fixed":
            stage("reaction", lambda: self.ctx.step_fixed(
                self.X, self.T, self.D, self.fidx, self.S_in, self.dt, self.substeps,
                A.FIXED_EULER, n=self.n, H=self.H, status=self.status))
        else:
            stage("reaction", lambda: self.ctx.step(
                self.X, self.T, self.D, self.fidx, self.S_in, self.dt, n=self.n, H=self.H,
                hlast=self.hl, status=self.status))
        if self.grid is not None:
            stage("diffusion", lambda: self.grid.diffuse(self.X, self.pos, self.n, self.dt,
                                                         self.diffusion_substeps))
        stage("gas flux", lambda: A.adm1_gas_flux(self.ctx.handle, self.X, self.ld, self.T,
                                                  self.V, self.n, None, None, self.tot))
        dt_s = self.dt * 86400.0
        stage("advection", lambda: A.adm1_advect(self.pos, self.ld, self.n, self.flow, dt_s,
                                                 W.advect_substeps(dt_s)))

    def save(self, path, time_s):
        """Write the particle positions and ADM1 states to a binary snapshot."""
        from . import snapshot as S
        S.adm1_snapshot_write(path, self.n, self.ld, time_s, pos=self.pos.cpu(),
                              state=self.X.cpu())

    def load(self, path):
        """Restore positions and states from a snapshot of the same particle
        count and return its time (s).  The per-particle warm starts (the
        S_H+ guess of the charge-balance solve and the adaptive scheme's
        last step size) are not part of a snapshot and restart from their
        defaults, so a resumed run agrees with an uninterrupted one to the
        solver tolerances, not bit for bit (positions do agree bit for
        bit)."""
        from . import snapshot as S
        torch = self.torch
        n, _, time_s = S.adm1_snapshot_info(path)
        if n != self.n:
            raise ValueError(f"snapshot holds {n} particles, the loop {self.n}")
        pos_h = torch.empty(self.pos.shape, dtype=self.pos.dtype)
        X_h = torch.empty(self.X.shape, dtype=self.X.dtype)
        S.adm1_snapshot_read(path, self.ld, pos=pos_h, state=X_h)
        self.pos.copy_(pos_h)
        self.X.copy_(X_h)
        self.H.fill_(-1.0)
        self.hl.fill_(-1.0)
        return time_s

    def close(self):
        if self.grid is not None:
            self.grid.close()
        self.ctx.close()


def main():
    import time

    import torch
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--n", type=int, default=1 << 22)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--scheme", choices=["adaptive", "fixed"], default="adaptive")
    ap.add_argument("--substeps", type=int, default=900,
                    help="fixed scheme: explicit steps per 1/96-d interval (1 s each)")
    ap.add_argument("--diffusion", type=float, default=0.0,
                    help="diffusivity of the soluble entries in m2/s (0: off)")
    ap.add_argument("--snapshot-dir", default="",
                    help="write positions and states after every interval")
    ap.add_argument("--resume", default="",
                    help="start from the positions and states of this snapshot")
    args = ap.parse_args()
    from . import snapshot as S
    loop = Loop(args.n, scheme=args.scheme, substeps=args.substeps, diffusion=args.diffusion)
    t0_s = loop.load(args.resume) if args.resume else 0.0
    names = ["feed mask", "reaction"] + (["diffusion"] if loop.grid is not None else []) + \
        ["gas flux", "advection"]
    if args.snapshot_dir:
        names.append("snapshot")
        pos_h = torch.empty_like(loop.pos, device="cpu").pin_memory()
        X_h = torch.empty_like(loop.X, device="cpu").pin_memory()
    extra = (f" in {loop.diffusion_substeps} explicit substeps" if loop.grid is not None
             else "")
    print(f"CHAD loop: {args.n} particles, {args.scheme} reaction step, "
          f"diffusion {args.diffusion:g} m2/s{extra}; times in ms per interval", flush=True)
    print("interval " + " ".join(f"{m:>10s}" for m in names) + "   CH4 flow (m3/d)",
          flush=True)
    for k in range(args.steps):
        ev = {m: (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for m in names}
        loop.interval(ev)
        if args.snapshot_dir:
            ev["snapshot"][0].record()
            pos_h.copy_(loop.pos, non_blocking=True)
            X_h.copy_(loop.X, non_blocking=True)
            torch.cuda.current_stream().synchronize()
            t0 = time.perf_counter()
            S.adm1_snapshot_write(os.path.join(args.snapshot_dir, f"chad_{k:04d}.bin"),
                                  args.n, loop.ld, t0_s + (k + 1) * loop.dt * 86400.0, pos=pos_h,
                                  state=X_h)
            snap_ms = (time.perf_counter() - t0) * 1e3
            ev["snapshot"][1].record()
        torch.cuda.synchronize()
        ms = [a.elapsed_time(b) for a, b in ev.values()]
        if args.snapshot_dir:
            ms[-1] += snap_ms
        bad = int((loop.status & 0x7F).count_nonzero())
        print(f"{k:8d} " + " ".join(f"{v:10.2f}" for v in ms) +
              f"   {float(loop.tot[2]):.6e}" + (f"  ({bad} failed)" if bad else ""),
              flush=True)
    loop.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
