"""Coupling driver: the analytic flow field (CPU pins of the oracle) and the
advection / feed-mask kernels against it (GPU)."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import transport as OT
from paper_2311_08927_amd import workloads as W


def _field():
    f = W.flow_field(3)
    return f["omega"], f["R"], f["H"], np.array(f["a"])


def test_field_is_divergence_free_and_tangent():
    omega, R, H, a = _field()
    rng = np.random.default_rng(0)
    n = 500
    r = R * np.sqrt(rng.random(n)) * 0.95
    th = 2 * np.pi * rng.random(n)
    z = H * (0.02 + 0.96 * rng.random(n))
    x, y = r * np.cos(th), r * np.sin(th)
    div = OT.divergence(x, y, z, omega, R, H, a)
    ux, uy, uz = OT.velocity(x, y, z, omega, R, H, a)
    scale = np.max(np.abs(np.stack([ux, uy, uz]))) / R
    assert np.max(np.abs(div)) < 1e-6 * scale
    # radial velocity vanishes at the wall, axial velocity at bottom and top
    xw, yw = R * np.cos(th), R * np.sin(th)
    uxw, uyw, _ = OT.velocity(xw, yw, z, omega, R, H, a)
    ur = (uxw * xw + uyw * yw) / R
    assert np.max(np.abs(ur)) < 1e-12
    for zb in (0.0, H):
        assert np.max(np.abs(OT.velocity(x, y, np.full(n, zb), omega, R, H, a)[2])) < 1e-12
    # solid-body rotation at the mixer speed (12 rpm) gives 0.126 m/s at the wall
    ut = (-uyw * 0 + (uyw * xw - uxw * yw) / R)
    assert np.allclose(ut, omega * R, rtol=1e-12)
    assert abs(omega * R - 0.1257) < 1e-3


def test_feed_mask_fraction():
    """Uniform positions: the inlet cylinder holds (0.03/0.1)^2 (0.02/0.3) of
    the volume (0.6 %)."""
    pos = W.cylinder_positions(200_000, seed=3)
    m = OT.feed_mask(pos[:, :200_000].astype(np.float64), W.INLET_Z, W.INLET_R)
    frac = (W.INLET_R / W.TANK_R) ** 2 * (W.TANK_H - W.INLET_Z) / W.TANK_H
    assert abs(m.mean() - frac) < 5 * np.sqrt(frac / 200_000)


@pytest.mark.gpu
def test_advect_and_mask_against_oracle():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2311_08927_amd import adm1 as A
    n = 5000
    pos0 = W.cylinder_positions(n, seed=5)
    f = W.flow_field(3)
    dpos = torch.from_numpy(pos0.copy()).cuda()
    ld = pos0.shape[1]
    A.adm1_advect(dpos, ld, n, A.make_flow(f), 900.0, 900)
    torch.cuda.synchronize()
    got = dpos.cpu().numpy()[:, :n]
    ref = OT.advect(pos0[:, :n], f["omega"], f["R"], f["H"], f["a"], 900.0, 900)
    err = np.abs(got - ref)
    print("advection max abs err (m):", err.max())
    assert err.max() < 2e-4
    assert np.all(got[0] ** 2 + got[1] ** 2 <= (f["R"] * (1 + 1e-6)) ** 2)
    # feed mask on the GPU positions is exact
    D = torch.empty(n, dtype=torch.float64, device="cuda")
    fidx = torch.empty(n, dtype=torch.int32, device="cuda")
    flag = torch.empty(n, dtype=torch.uint8, device="cuda")
    A.adm1_feed_mask(dpos, ld, n, W.INLET_Z, W.INLET_R, 1.0, 1, 0, D, fidx, flag)
    torch.cuda.synchronize()
    m = OT.feed_mask(got.astype(np.float32).astype(np.float64), np.float32(W.INLET_Z),
                     np.float32(W.INLET_R))
    fl = flag.cpu().numpy().astype(bool)
    # membership decided in FP32 on both sides: compare away from the boundary
    x, y, z = got
    margin = (np.abs(z - W.INLET_Z) > 1e-6) & (np.abs(np.sqrt(x * x + y * y) - W.INLET_R) > 1e-6)
    assert np.array_equal(fl[margin], m[margin])
    assert np.array_equal(D.cpu().numpy() == 1.0, fl)
    assert np.array_equal(fidx.cpu().numpy() == 1, fl)
