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
    """Trajectories against the FP64 oracle over 60 s (the meridional loops
    turn over in tens of seconds; over a whole interval the two FP64
    trajectories drift apart along the closed streamlines from their
    different rounding, as any two nearby trajectories of this shear flow
    do); over a whole interval
    the particles stay in the tank and uniformly spread, and the feed mask on
    the GPU positions is exact."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2311_08927_amd import adm1 as A
    n = 5000
    pos0 = W.cylinder_positions(n, seed=5)
    f = W.flow_field(3)
    ld = pos0.shape[1]
    dpos = torch.from_numpy(pos0.copy()).cuda()
    A.adm1_advect(dpos, ld, n, A.make_flow(f), 60.0, 60)
    torch.cuda.synchronize()
    got = dpos.cpu().numpy()[:, :n]
    ref = OT.advect(pos0[:, :n], f["omega"], f["R"], f["H"], f["a"], 60.0, 60)
    err = np.abs(got - ref).max(axis=0)
    print(f"advection over 60 s, abs err (m): p99 {np.quantile(err, 0.99):.2e}, "
          f"max {err.max():.2e}")
    # both sides advance in FP64; the GPU rounds its result to FP32 once
    # (half an ulp of 0.3 m is 1.5e-8 m)
    assert np.quantile(err, 0.99) < 1e-7
    assert err.max() < 1e-6
    # a whole interval on a larger population
    n = 40_000
    pos0 = W.cylinder_positions(n, seed=6)
    ld = pos0.shape[1]
    dpos = torch.from_numpy(pos0.copy()).cuda()
    A.adm1_advect(dpos, ld, n, A.make_flow(f), 900.0, 900)
    torch.cuda.synchronize()
    got = dpos.cpu().numpy()[:, :n]
    x, y, z = got
    r2 = x * x + y * y
    assert np.all(r2 <= (f["R"] * (1 + 1e-6)) ** 2)
    assert np.all((z >= 0) & (z <= f["H"]))
    assert abs(r2.mean() / (f["R"] ** 2 / 2) - 1.0) < 0.02
    frac = (W.INLET_R / W.TANK_R) ** 2 * (W.TANK_H - W.INLET_Z) / W.TANK_H
    D = torch.empty(n, dtype=torch.float64, device="cuda")
    fidx = torch.empty(n, dtype=torch.int32, device="cuda")
    flag = torch.empty(n, dtype=torch.uint8, device="cuda")
    A.adm1_feed_mask(dpos, ld, n, W.INLET_Z, W.INLET_R, 1.0, 1, 0, D, fidx, flag)
    torch.cuda.synchronize()
    fl = flag.cpu().numpy().astype(bool)
    assert abs(fl.mean() - frac) < 5 * np.sqrt(frac / n)
    m = OT.feed_mask(got.astype(np.float32).astype(np.float64), np.float32(W.INLET_Z),
                     np.float32(W.INLET_R))
    # membership decided in FP32 on both sides: compare away from the boundary
    margin = (np.abs(z - W.INLET_Z) > 1e-6) & (np.abs(np.sqrt(r2) - W.INLET_R) > 1e-6)
    assert np.array_equal(fl[margin], m[margin])
    assert np.array_equal(D.cpu().numpy() == 1.0, fl)
    assert np.array_equal(fidx.cpu().numpy() == 1, fl)


def test_pure_rotation_is_exact():
    """No meridional modes: one interval of 900 substeps turns every particle
    by omega t about the axis and keeps its radius and height."""
    f = W.flow_field(3)
    pos = W.cylinder_positions(2000, seed=7)[:, :2000].astype(np.float64)
    t = 900.0
    out = OT.advect(pos, f["omega"], f["R"], f["H"], np.zeros(4), t, 900)
    c, s = np.cos(f["omega"] * t), np.sin(f["omega"] * t)
    ref = np.stack([c * pos[0] - s * pos[1], s * pos[0] + c * pos[1], pos[2]])
    assert np.max(np.abs(out - ref)) < 1e-12


def test_advection_keeps_particles_uniform():
    """The field is divergence free, so uniformly placed particles stay
    uniform: after one interval the mean of r^2 stays R^2/2 and the inlet
    region still holds its volume fraction of the particles."""
    omega, R, H, a = _field()
    n = 20_000
    pos = W.cylinder_positions(n, seed=9)[:, :n].astype(np.float64)
    out = OT.advect(pos, omega, R, H, a, 900.0, 900)
    r2 = out[0] ** 2 + out[1] ** 2
    assert abs(r2.mean() / (R * R / 2) - 1.0) < 0.02
    frac = (W.INLET_R / W.TANK_R) ** 2 * (W.TANK_H - W.INLET_Z) / W.TANK_H
    m = OT.feed_mask(out, W.INLET_Z, W.INLET_R)
    assert abs(m.mean() - frac) < 5 * np.sqrt(frac / n)


def test_meridional_rk4_converges():
    """Over 30 s the 1 s substep agrees with half-second substeps to well
    under the particle spacing of the 2^22-particle field (1.3 mm; here
    0.3 mm at most), and the gap shrinks at about fourth order.  Over a whole interval the loops repeat
    tens of times and trajectory phases drift apart; the particle
    distribution stays uniform (test above)."""
    omega, R, H, a = _field()
    pos = W.cylinder_positions(500, seed=2)[:, :500].astype(np.float64)
    p1, p2, p4 = (OT.advect(pos, omega, R, H, a, 30.0, m) for m in (30, 60, 120))
    inside = (np.sqrt(p4[0] ** 2 + p4[1] ** 2) < 0.99 * R) & (p4[2] > 0.01 * H) & \
        (p4[2] < 0.99 * H)
    e1 = np.max(np.abs(p1 - p2)[:, inside])
    e2 = np.max(np.abs(p2 - p4)[:, inside])
    assert e1 < 1e-3
    assert e1 / e2 > 8.0


@pytest.mark.gpu
def test_gpu_rotation_keeps_radii():
    """Pure rotation (no meridional modes) over ten intervals of 900 substeps:
    the three-shear turn keeps every particle's radius and height, where a
    matrix of rounded cos and sin scales every radius alike each substep
    (in FP32, ~3e-5 per interval, which piled particles onto the wall)."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2311_08927_amd import adm1 as A
    n = 20_000
    pos0 = W.cylinder_positions(n, seed=8)
    ld = pos0.shape[1]
    f = dict(W.flow_field(3))
    f["a"] = [0.0, 0.0, 0.0, 0.0]
    dpos = torch.from_numpy(pos0.copy()).cuda()
    for _ in range(10):
        A.adm1_advect(dpos, ld, n, A.make_flow(f), 900.0, 900)
    torch.cuda.synchronize()
    got = dpos.cpu().numpy()[:, :n].astype(np.float64)
    p0 = pos0[:, :n].astype(np.float64)
    r0, r1 = np.hypot(p0[0], p0[1]), np.hypot(got[0], got[1])
    drift = np.abs(r1 - r0) / W.TANK_R
    print(f"radius change after 10 intervals: max {drift.max():.2e}, mean signed "
          f"{np.mean((r1 - r0) / W.TANK_R):.2e}")
    assert drift.max() < 2e-5
    assert abs(np.mean((r1 - r0) / W.TANK_R)) < 2e-6
    assert np.array_equal(got[2], p0[2])


@pytest.mark.gpu
def test_gpu_no_collapse_onto_the_axis():
    """Four hour-long intervals at the field's substep: no particle reaches
    the axis.  With the positions advanced in FP32, increments near the
    axial stagnation points rounded away and a few particles per interval
    (of 4 M) froze in z while their radius shrank to denormals, then piled
    up at one point of the axis (dozens at one position), which the
    diffusion operator cannot take."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2311_08927_amd import adm1 as A
    n = 1 << 20
    pos0 = W.cylinder_positions(n, seed=3)
    ld = pos0.shape[1]
    f = W.flow_field(3)
    dpos = torch.from_numpy(pos0).cuda()
    for _ in range(4):
        A.adm1_advect(dpos, ld, n, A.make_flow(f), 900.0, W.advect_substeps(900.0))
    torch.cuda.synchronize()
    got = dpos.cpu().numpy()[:, :n].astype(np.float64)
    r = np.hypot(got[0], got[1])
    print(f"smallest radius after four intervals: {r.min():.3e} m")
    assert r.min() > 1e-9
    assert len(np.unique(got.T, axis=0)) == n
