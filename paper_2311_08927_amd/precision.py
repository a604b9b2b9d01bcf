"""Reduced-precision experiment: rate evaluation in FP32.

The eq. 7 and eq. 8 Newton solves and the Newton-matrix LU stay in FP64;
only the inhibitions, the 19 rates, the transfers and the eq. 2 assembly run
in FP32 (adm1_opts.rate_precision = 1).  The report gives, per state entry,
the max / 99th percentile / median of the relative error
|x_32 - x_64| / max(|x_64|, 1e-4 x_nom) of (a) the right-hand side at the
start states and (b) the integrated states after each coupling step, the
FP64 reference being the FP64 HIP path (itself checked against the FP64
oracle); callers add an oracle sample where they can afford one.
"""
from __future__ import annotations

import sys

import numpy as np

from . import workloads as W

NAMES = ["S_su", "S_aa", "S_fa", "S_va", "S_bu", "S_pro", "S_ac", "S_h2", "S_ch4", "S_IC",
         "S_IN", "S_I", "X_xc", "X_ch", "X_pr", "X_li", "X_su", "X_aa", "X_fa", "X_c4",
         "X_pro", "X_ac", "X_h2", "X_I", "S_cat", "S_an", "S_va_ion", "S_bu_ion",
         "S_pro_ion", "S_ac_ion", "S_hco3_ion", "S_nh3", "G_h2", "G_ch4", "G_co2"]


def rel_err_stats(a, b, scale):
    """Per row: (max, p99, median) of |a - b| / max(|b|, scale) over columns.
    a, b: torch tensors [rows][n]; scale: [rows] tensor."""
    import torch
    den = torch.maximum(b.abs(), scale[:, None])
    e = (a - b).abs() / den
    e = e.float()
    q = torch.quantile(e[:, :min(e.shape[1], 1 << 24)],
                       torch.tensor([0.99, 0.5], device=e.device), dim=1)
    return torch.stack([e.max(dim=1).values, q[0], q[1]], dim=1).cpu().numpy()


def fp32_rate_report(ctx64, ctx32, X, T, D, fidx, S_in, dt, n, steps=1, D_at=None):
    """Run the FP64 and FP32-rate paths side by side from X (device tensor,
    not modified).  Returns {"rhs": [28][3], "state": [steps][35][3]}."""
    import torch
    nom = torch.from_numpy(W.nominal()["state"]).to(X.device)
    d64, _, _ = ctx64.rhs(X, T, D, fidx, S_in, n=n, rate_precision=0)
    d32, _, _ = ctx64.rhs(X, T, D, fidx, S_in, n=n, rate_precision=1)
    fscale = d64[:, :n].abs().amax(dim=1) * 1e-3 + 1e-300
    out = {"rhs": rel_err_stats(d32[:, :n], d64[:, :n], fscale).tolist(), "state": []}
    X64, X32 = X.clone(), X.clone()
    H64 = torch.full((n,), -1.0, dtype=torch.float64, device=X.device)
    H32, h64, h32 = H64.clone(), H64.clone(), H64.clone()
    for s in range(steps):
        Ds = D if D_at is None else D_at(s)
        ctx64.step(X64, T, Ds, fidx, S_in, dt, n=n, H=H64, hlast=h64)
        ctx32.step(X32, T, Ds, fidx, S_in, dt, n=n, H=H32, hlast=h32)
        out["state"].append(rel_err_stats(X32[:, :n], X64[:, :n], 1e-4 * nom).tolist())
    return out


def format_report(rep) -> str:
    rows = ["entry        rhs max    rhs p99   state max  state p99 state med"]
    last = np.array(rep["state"][-1])
    rhs = np.array(rep["rhs"])
    diff_rows = list(W.DIFF)
    for i, name in enumerate(NAMES):
        r = rhs[diff_rows.index(i)] if i in diff_rows else [np.nan] * 3
        rows.append(f"{name:10s} {r[0]:10.2e} {r[1]:10.2e} {last[i][0]:10.2e} "
                    f"{last[i][1]:10.2e} {last[i][2]:10.2e}")
    return "\n".join(rows)


def main():
    """Per-state FP32-rate report on the digester field (particles advected
    between steps, inlet feed mask), printed as a markdown table."""
    import argparse

    import torch

    from . import adm1 as A
    ap = argparse.ArgumentParser(description=main.__doc__)
    ap.add_argument("--n", type=int, default=1 << 22)
    ap.add_argument("--steps", type=int, default=96)
    ap.add_argument("--rtol", type=float, default=1e-8)
    args = ap.parse_args()
    w = W.digester_field(args.n, seed=3, steps=args.steps)
    atol = W.atol_vector(args.rtol)
    ctx64 = A.Context(w.ld, rtol=args.rtol, atol=atol)
    ctx32 = A.Context(w.ld, rtol=args.rtol, atol=atol, rate_precision=1)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    X, T, S_in, pos = t(w.X), t(w.T), t(w.feed), t(w.extra["pos"])
    flow = A.make_flow(w.extra["flow"])
    D = torch.zeros(w.n, dtype=torch.float64, device="cuda")
    fidx = torch.zeros(w.n, dtype=torch.int32, device="cuda")
    dt_s = w.dt * 86400.0

    def mask():
        A.adm1_feed_mask(pos, w.ld, w.n, W.INLET_Z, W.INLET_R, 1.0, 1, 0, D, fidx)

    def D_at(s):
        if s > 0:
            A.adm1_advect(pos, w.ld, w.n, flow, dt_s, W.advect_substeps(dt_s))
        mask()
        print(f"# step {s}", file=sys.stderr, flush=True)
        return D

    mask()
    rep = fp32_rate_report(ctx64, ctx32, X, T, D, fidx, S_in, w.dt, w.n, steps=args.steps,
                           D_at=D_at)
    print(f"Digester field, {w.n} particles, {args.steps} coupling steps of 1/96 d, rtol "
          f"{args.rtol:g}; FP32 rates against the FP64 path; relative error "
          f"|x32 - x64| / max(|x64|, 1e-4 x_nom) (right-hand side: scale 1e-3 max|f|).\n")
    print("| entry | rhs max | rhs p99 | state max | state p99 | state median |")
    print("|---|---|---|---|---|---|")
    for line in format_report(rep).splitlines()[1:]:
        f = ["—" if v == "nan" else v for v in line.split()]  # algebraic: no rhs row
        print("| " + " | ".join(f) + " |")
    per_step = [float(np.nanmax(np.array(s)[:, 0])) for s in rep["state"]]
    print("\nWorst state entry after each step: " + ", ".join(f"{v:.2e}" for v in per_step))


if __name__ == "__main__":
    main()
