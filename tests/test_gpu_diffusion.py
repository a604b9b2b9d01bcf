"""GPU parity of diffusion between particles (adm1_diffuse: uniform-grid
neighbour search + SPH diffusion operator) against the brute-force oracle,
through the C ABI: neighbour counts bit-exact, updates within rounding of
the pair sums, conservation, determinism, particles outside the grid box,
argument errors, and a sampled check on the full digester field."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import diffusion as OD
from paper_2311_08927_amd import workloads as W

pytestmark = pytest.mark.gpu

D_MOL = 1e-9 * 86400.0  # m2/d


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def box_case(n, seed, spacing_factor=1.3, outside=0):
    """n particles uniform in a 4 x 3 x 2 cm box (some placed outside it),
    perturbed nominal states; h = spacing_factor x mean spacing."""
    g = np.random.default_rng(seed)
    ld = W.pad_ld(n, 64)
    lo, hi = np.array([0.0, 0.0, 0.0]), np.array([0.04, 0.03, 0.02])
    pos = np.zeros((3, ld), dtype=np.float32)
    pos[:, :n] = (lo[:, None] + (hi - lo)[:, None] * g.random((3, n))).astype(np.float32)
    if outside:
        pos[:, :outside] += np.float32(0.004) * np.sign(g.standard_normal((3, outside)))
    spacing = (np.prod(hi - lo) / n) ** (1 / 3)
    X = W.perturbed_states(n, seed, ld=ld)
    return pos, X, spacing_factor * spacing, np.prod(hi - lo) / n, lo, hi


def run_gpu(torch, pos, X, n, h, V_p, lo, hi, dt, substeps, with_counts=True):
    from paper_2311_08927_amd import adm1 as A
    grid = A.Grid(A.make_diffusion(h, D_MOL, V_p, lo, hi), X.shape[1])
    dX = torch.from_numpy(X.copy()).cuda()
    dpos = torch.from_numpy(pos).cuda()
    cnt = torch.full((n,), -1, dtype=torch.int32, device="cuda") if with_counts else None
    grid.diffuse(dX, dpos, n, dt, substeps, cnt)
    torch.cuda.synchronize()
    out = dX.cpu().numpy(), None if cnt is None else cnt.cpu().numpy()
    grid.close()
    return out


@pytest.mark.parametrize("n,outside", [(3000, 0), (1000, 40)])
def test_neighbours_and_one_step(torch_cuda, n, outside):
    pos, X, h, V_p, lo, hi = box_case(n, 3 + n, outside=outside)
    dt = 0.02
    Xg, cnt = run_gpu(torch_cuda, pos, X, n, h, V_p, lo, hi, dt, 1)
    P = pos[:, :n].astype(np.float64)
    ref = OD.neighbour_counts(P, h)
    assert np.array_equal(cnt, ref), np.nonzero(cnt != ref)
    print(f"n={n}: {ref.mean():.1f} neighbours per particle")
    rate, absum = OD.diffusion_rate(P, X[OD.DIFFUSING, :n], h, V_p, D_MOL)
    dg = Xg[OD.DIFFUSING, :n] - X[OD.DIFFUSING, :n]
    do = dt * rate
    err = np.abs(dg - do) / (dt * absum + 1e-300)
    print(f"update error / absolute pair sum: max {err.max():.2e}")
    assert err.max() < 1e-12
    assert np.max(np.abs(do)) > 1e-6 * np.max(np.abs(X[OD.DIFFUSING, :n]))
    rest = [i for i in range(35) if i not in OD.DIFFUSING]
    assert np.array_equal(Xg[rest], X[rest])
    # conservation: the pair terms cancel over the particles
    tot = dg.sum(axis=1)
    assert np.all(np.abs(tot) < 1e-11 * (dt * absum).sum(axis=1))


def test_substeps_against_oracle_and_repeatable(torch_cuda):
    n = 2000
    pos, X, h, V_p, lo, hi = box_case(n, 11)
    dt, m = 0.05, 4
    Xg, _ = run_gpu(torch_cuda, pos, X, n, h, V_p, lo, hi, dt, m, with_counts=False)
    Xg2, _ = run_gpu(torch_cuda, pos, X, n, h, V_p, lo, hi, dt, m, with_counts=False)
    assert np.array_equal(Xg, Xg2)
    Xo = OD.diffuse(X, pos.astype(np.float64), n, h, V_p, D_MOL, dt, m)
    _, absum = OD.diffusion_rate(pos[:, :n].astype(np.float64), X[OD.DIFFUSING, :n], h, V_p,
                                 D_MOL)
    err = np.abs(Xg[OD.DIFFUSING, :n] - Xo[OD.DIFFUSING, :n]) / (dt * absum + 1e-300)
    print(f"{m} substeps: error / absolute pair sum max {err.max():.2e}")
    assert err.max() < 1e-11


def test_digester_field_sampled(torch_cuda):
    """The lab-digester field at 2^22 particles (h = 1.3 x the mean spacing,
    the first of eight steps of molecular diffusion over a 1/96-d interval):
    48 seeded particles recomputed by the oracle against all particles."""
    n = 1 << 22
    w = W.digester_field(n, seed=3, steps=1)
    pos = w.extra["pos"]
    V_p = w.extra["V_p"]
    h = 1.3 * V_p ** (1 / 3)
    lo = [-W.TANK_R, -W.TANK_R, 0.0]
    hi = [W.TANK_R, W.TANK_R, W.TANK_H]
    dt, m = 1.0 / 96.0, 8
    from paper_2311_08927_amd import adm1 as A
    grid = A.Grid(A.make_diffusion(h, D_MOL, V_p, lo, hi), w.ld)
    dX = torch_cuda.from_numpy(np.ascontiguousarray(w.X)).cuda()
    dpos = torch_cuda.from_numpy(np.ascontiguousarray(pos)).cuda()
    cnt = torch_cuda.zeros(n, dtype=torch_cuda.int32, device="cuda")
    grid.diffuse(dX, dpos, n, dt / m, 1, cnt)  # first substep alone
    torch_cuda.cuda.synchronize()
    Xg = dX.cpu().numpy()
    c = cnt.cpu().numpy()
    grid.close()
    idx = np.sort(np.random.default_rng(8).choice(n, 48, replace=False))
    P = pos[:, :n].astype(np.float64)
    rate, cref = OD.diffusion_rate_at(P, w.X[OD.DIFFUSING, :n], idx, h, V_p, D_MOL)
    assert np.array_equal(c[idx], cref)
    dg = Xg[OD.DIFFUSING][:, idx] - w.X[OD.DIFFUSING][:, idx]
    do = dt / m * rate
    scale = np.max(np.abs(do), axis=1, keepdims=True) + 1e-300
    err = np.abs(dg - do) / scale
    print(f"field 2^22: {c.mean():.1f} neighbours per particle; sampled update error "
          f"{err.max():.2e} of the largest sampled update")
    assert err.max() < 1e-9


def test_grid_and_diffuse_arguments(torch_cuda):
    from paper_2311_08927_amd import adm1 as A
    ok = A.make_diffusion(0.002, D_MOL, 1e-9, [0, 0, 0], [0.04, 0.03, 0.02])
    for bad in (A.make_diffusion(0.0, D_MOL, 1e-9, [0, 0, 0], [1, 1, 1]),
                A.make_diffusion(0.002, -1.0, 1e-9, [0, 0, 0], [1, 1, 1]),
                A.make_diffusion(0.002, D_MOL, 0.0, [0, 0, 0], [1, 1, 1]),
                A.make_diffusion(0.002, D_MOL, 1e-9, [0, 0, 0], [0, 1, 1]),
                A.make_diffusion(1e-6, D_MOL, 1e-9, [0, 0, 0], [1, 1, 1])):  # 2^36 cells
        assert A.adm1_grid_create(bad, 1024, check=False) == -5
    assert A.adm1_grid_create(ok, 0, check=False) == -2
    grid = A.Grid(ok, 256)
    X = torch_cuda.zeros((35, 256), dtype=torch_cuda.float64, device="cuda")
    pos = torch_cuda.zeros((3, 256), dtype=torch_cuda.float32, device="cuda")
    h = grid.handle
    assert A.adm1_diffuse(h, X, 256, pos, 300, 0.1, 1, check=False) == -2
    assert A.adm1_diffuse(h, X, 256, pos, 100, 0.0, 1, check=False) == -9
    assert A.adm1_diffuse(h, X, 256, pos, 100, 0.1, 0, check=False) == -5
    assert A.adm1_diffuse(h, X, 256, None, 100, 0.1, 1, check=False) == -1
    assert A.adm1_diffuse(h, X, 256, pos, 0, 0.1, 1, check=False) == 0
    grid.close()


def test_max_principle_on_the_advected_field(torch_cuda):
    """2^21 field particles advected for three hour-long intervals, then one
    call at twice the stable substep count: every diffused row stays within
    its range before the call and keeps its total.  Explicit Euler with
    substep x row rate <= 1 is a convex combination of neighbouring values;
    random placement reaches row rates of ~20 D/h^2, so these substeps keep
    every row at or below ~0.5.  When FP32 advection piled particles onto
    the tank axis, the pile's row rates reached ~117 D/h^2 and these rows
    went negative."""
    torch = torch_cuda
    from paper_2311_08927_amd import adm1 as A
    n = 1 << 21
    w = W.digester_field(n, seed=3, steps=1)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    X, pos = t(w.X), t(w.extra["pos"])
    flow = A.make_flow(w.extra["flow"])
    for _ in range(3):
        A.adm1_advect(pos, w.ld, n, flow, 900.0, W.advect_substeps(900.0))
    V_p = w.extra["V_p"]
    grid = A.Grid(A.make_diffusion(1.3 * V_p ** (1 / 3), D_MOL, V_p,
                                   [-W.TANK_R, -W.TANK_R, 0.0], [W.TANK_R, W.TANK_R, W.TANK_H]),
                  w.ld)
    try:
        rows = list(OD.DIFFUSING)
        before = X[rows, :n].clone()
        sub = 2 * grid.stable_substeps(w.dt)
        grid.diffuse(X, pos, n, w.dt, sub)
        torch.cuda.synchronize()
        after = X[rows, :n]
        lo, hi = before.min(dim=1).values, before.max(dim=1).values
        span = hi - lo
        print(f"{sub} substeps; lowest margin below the old minimum "
              f"{float(((after.min(dim=1).values - lo) / span).min()):.2e} of the range")
        assert bool(torch.all(after.min(dim=1).values >= lo - 1e-12 * span))
        assert bool(torch.all(after.max(dim=1).values <= hi + 1e-12 * span))
        s0, s1 = before.sum(dim=1), after.sum(dim=1)
        assert float(((s1 - s0).abs() / s0.abs()).max()) < 1e-12
    finally:
        grid.close()
