"""GPU tests of the runtime pieces: HIP-graph capture of a coupling step,
the autotuner and the launch-configuration setter (through the C ABI)."""
from __future__ import annotations

import numpy as np
import pytest

from oracle.adm1 import Oracle
from paper_2311_08927_amd import workloads as W
from tests.gpu_common import PARITY_TOL, DeviceWorkload, parity

pytestmark = pytest.mark.gpu
RTOL = 1e-8


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def make_ctx(n_max, **kw):
    from paper_2311_08927_amd.adm1 import Context
    return Context(n_max, rtol=RTOL, atol=W.atol_vector(RTOL), **kw)


def test_graph_replay_matches_eager(torch_cuda):
    """Replays of a captured coupling step equal the eager steps bit for bit,
    with unrelated GPU work and host synchronisations between replays; a
    feed change between replays is picked up."""
    torch = torch_cuda
    from paper_2311_08927_amd import adm1 as A
    w = W.batched_population(4096, seed=7)
    ctx = make_ctx(w.ld, variant=A.VARIANT_SPARSE2)
    eager = DeviceWorkload(w)
    graphd = DeviceWorkload(w)
    V = torch.full((w.n,), 1.0, dtype=torch.float64, device="cuda")
    outs = {}
    for tag, dw in (("e", eager), ("g", graphd)):
        outs[tag] = dict(q=torch.empty(w.n, dtype=torch.float64, device="cuda"),
                         qc=torch.empty(w.n, dtype=torch.float64, device="cuda"),
                         tot=torch.empty(4, dtype=torch.float64, device="cuda"))
    s = torch.cuda.Stream()
    feed_g = A.feed_struct(graphd.D, graphd.fidx, graphd.S_in)
    aux_g = A.adm1_aux(graphd.H.data_ptr(), graphd.hlast.data_ptr())
    og = outs["g"]
    g = A.adm1_graph_capture_step(ctx.handle, graphd.X, w.ld, graphd.T, feed_g, w.dt, w.n,
                                  aux_g, graphd.status, graphd.nsteps, V, og["q"], og["qc"],
                                  og["tot"], s)
    try:
        junk = torch.zeros(1 << 20, device="cuda")
        for k in range(4):
            D = torch.from_numpy(w.D_at(k)).cuda()
            eager.D.copy_(D)
            graphd.D.copy_(D)
            torch.cuda.synchronize()
            ctx.step(eager.X, eager.T, eager.D, eager.fidx, eager.S_in, w.dt, n=w.n,
                     H=eager.H, hlast=eager.hlast, status=eager.status, nsteps=eager.nsteps)
            oe = outs["e"]
            A.adm1_gas_flux(ctx.handle, eager.X, w.ld, eager.T, V, w.n, oe["q"], oe["qc"],
                            oe["tot"])
            torch.cuda.synchronize()
            junk.add_(1.0)  # unrelated eager work between replays
            A.adm1_graph_launch(g, s)
            s.synchronize()
            assert torch.equal(eager.X, graphd.X), k
            assert torch.equal(oe["tot"], og["tot"]), k
            assert torch.equal(eager.nsteps, graphd.nsteps), k
    finally:
        A.adm1_graph_destroy(g)


def test_autotune_and_launch_setting(torch_cuda, tmp_path, monkeypatch):
    torch = torch_cuda
    from paper_2311_08927_amd import adm1 as A
    from paper_2311_08927_amd import autotune as AT
    monkeypatch.setattr(AT, "CACHE", str(tmp_path / "tune.json"))
    monkeypatch.setattr(AT, "PACKAGED", str(tmp_path / "packaged.json"))
    w = W.batched_population(8192, seed=8)
    ctx = make_ctx(w.ld)
    dw = DeviceWorkload(w)
    res = AT.autotune(ctx, dw.X, dw.T, dw.D, dw.fidx, dw.S_in, w.dt, n=w.n, tag="test")
    assert tuple(res["choice"]) in [tuple(c) for c in AT.CANDIDATES]
    assert len(res["timings_ms"]) == len(AT.CANDIDATES)
    # the space: lanes per particle 1 and 2; the Newton matrix in private
    # memory, registers or LDS; waves per CU 1-4; service batches 1-8
    assert {c[0] for c in AT.CANDIDATES} == {A.VARIANT_DENSE1, A.VARIANT_SPARSE1,
                                             A.VARIANT_SPARSE1_LDS, A.VARIANT_SPARSE2}
    assert {c[1] for c in AT.CANDIDATES if c[0] == A.VARIANT_SPARSE2} == {1, 2, 3, 4}
    assert {c[2] for c in AT.CANDIDATES if c[0] == A.VARIANT_SPARSE2} == {1, 2, 4, 8}
    print("autotune:", res["layout"], {k: round(v, 2) for k, v in res["timings_ms"].items()})
    # cached second call
    res2 = AT.autotune(ctx, dw.X, dw.T, dw.D, dw.fidx, dw.S_in, w.dt, n=w.n, tag="test")
    assert res2["choice"] == res["choice"] and res2["source"] == "user cache"
    # a packaged choice is used when the user cache has none
    import json
    key = next(iter(json.load(open(tmp_path / "tune.json"))))
    (tmp_path / "packaged.json").write_text(json.dumps({key: dict(res, choice=[2, 2, 8])}))
    (tmp_path / "tune.json").unlink()
    res3 = AT.autotune(ctx, dw.X, dw.T, dw.D, dw.fidx, dw.S_in, w.dt, n=w.n, tag="test")
    assert res3["choice"] == [2, 2, 8] and res3["source"] == "packaged" and res3["cached"]
    # the tuned launch gives the oracle's answer on a slice
    sub = W.subset(w, np.arange(0, w.n, 97))
    dsub = DeviceWorkload(sub)
    ctx.step(dsub.X, dsub.T, dsub.D, dsub.fidx, dsub.S_in, sub.dt, n=sub.n)
    orc = Oracle(W.params_path(), rtol=RTOL, atol=W.atol_vector(RTOL))
    Xo = sub.X.copy()
    orc.step(Xo, sub.T, sub.D, sub.fidx, sub.feed, sub.dt, n=sub.n)
    assert parity(dsub.X.cpu().numpy(), Xo, sub.n) <= PARITY_TOL
    with pytest.raises(A.ADM1Error):
        A.adm1_set_launch(ctx.handle, 7, 0)
    with pytest.raises(A.ADM1Error):
        A.adm1_set_launch(ctx.handle, A.VARIANT_SPARSE2, 9)
    with pytest.raises(A.ADM1Error):
        A.adm1_set_service_batch(ctx.handle, 33)
    torch.cuda.synchronize()


@pytest.mark.parametrize("batch", [1, 8, 32])
def test_service_batch_does_not_change_results(torch_cuda, batch):
    """Restarting particles in batches of any size gives the same results
    (bit for bit) as the default batch, cold and warm intervals."""
    from paper_2311_08927_amd import adm1 as A
    w = W.batched_population(3000, seed=10)
    outs = []
    for sb in (0, batch):
        ctx = make_ctx(w.ld, variant=A.VARIANT_SPARSE2)
        A.adm1_set_service_batch(ctx.handle, sb)
        d = DeviceWorkload(w)
        for k in range(2):
            d.set_D(w.D_at(k))
            ctx.step(d.X, d.T, d.D, d.fidx, d.S_in, w.dt, n=w.n, H=d.H, hlast=d.hlast,
                     nsteps=d.nsteps)
        outs.append((d.X.cpu().numpy(), d.nsteps.cpu().numpy()))
    assert np.array_equal(outs[0][0], outs[1][0])
    assert np.array_equal(outs[0][1], outs[1][1])


@pytest.mark.parametrize("blocks", [1, 3])
def test_sparse2_grid_sizes(torch_cuda, blocks):
    """The persistent kernel gives the same particles the same results
    whatever the grid size (work-queue order does not matter)."""
    from paper_2311_08927_amd import adm1 as A
    w = W.cstr_population(256, seed=9)
    ref = make_ctx(w.ld, variant=A.VARIANT_SPARSE2)
    d0 = DeviceWorkload(w)
    ref.step(d0.X, d0.T, d0.D, d0.fidx, d0.S_in, w.dt, n=w.n)
    ctx = make_ctx(w.ld)
    A.adm1_set_launch(ctx.handle, A.VARIANT_SPARSE2, blocks)
    d1 = DeviceWorkload(w)
    ctx.step(d1.X, d1.T, d1.D, d1.fidx, d1.S_in, w.dt, n=w.n)
    assert np.array_equal(d0.X.cpu().numpy(), d1.X.cpu().numpy())


def _cost_bucket(h: np.ndarray, dt: float) -> np.ndarray:
    """Bucket of the cost order as its header comment defines it."""
    b = np.full(h.shape, 1023, dtype=np.int64)
    warm = h > 0.0
    with np.errstate(divide="ignore", over="ignore"):
        x = dt / h[warm] * 8.0
    b[warm] = np.where(x < 1023.0, np.floor(np.minimum(x, 1023.0)), 1023).astype(np.int64)
    return b


@pytest.mark.parametrize("n", [1, 1000, (1 << 20) + 7])
def test_cost_order_is_sorted_permutation(torch_cuda, n):
    """adm1_cost_order returns a permutation of 0..n-1 along which the cost
    bucket does not increase, for step sizes that span every bucket and the
    special values (cold, zero, NaN, inf, denormal-sized); a second call on
    the same context (smaller n) is right too (the histogram is left clear)."""
    torch = torch_cuda
    from paper_2311_08927_amd import adm1 as A
    dt = W.DT
    ctx = make_ctx(8)
    g = np.random.default_rng(n)
    for m in (n, max(1, n // 3)):
        h = dt / np.exp(g.uniform(-2.0, 7.5, m))
        special = g.integers(0, m, size=min(m, 64))
        h[special] = g.choice([-1.0, 0.0, np.nan, np.inf, 1e-300, dt / 8.0, dt / 1023.0 * 8.0,
                               dt / 2.0], size=special.size)
        hd = torch.from_numpy(h).cuda()
        order = torch.full((m,), -1, dtype=torch.int32, device="cuda")
        A.adm1_cost_order(ctx.handle, hd, dt, m, order)
        torch.cuda.synchronize()
        o = order.cpu().numpy().astype(np.int64)
        assert np.array_equal(np.sort(o), np.arange(m))
        k = _cost_bucket(h, dt)[o]
        assert np.all(np.diff(k) <= 0)
    with pytest.raises(A.ADM1Error):
        A.adm1_set_order(ctx.handle, 2)


def test_queue_order_does_not_change_results(torch_cuda):
    """Index order and cost order of the work queue give every particle the
    same result bit for bit over warm-started coupling steps (2^16 particles,
    so the queue cycles many times per wave)."""
    torch = torch_cuda
    from paper_2311_08927_amd import adm1 as A
    w = W.batched_population(1 << 16, seed=11)
    runs = {}
    for mode in (A.ORDER_INDEX, A.ORDER_COST):
        ctx = make_ctx(w.ld, variant=A.VARIANT_SPARSE2)
        A.adm1_set_order(ctx.handle, mode)
        dw = DeviceWorkload(w)
        snaps = []
        for k in range(3):
            dw.set_D(w.D_at(k))
            ctx.step(dw.X, dw.T, dw.D, dw.fidx, dw.S_in, w.dt, n=w.n, H=dw.H, hlast=dw.hlast,
                     status=dw.status, nsteps=dw.nsteps)
            torch.cuda.synchronize()
            snaps.append([t.cpu().numpy().copy() for t in (dw.X, dw.H, dw.hlast, dw.status,
                                                           dw.nsteps)])
        runs[mode] = snaps
    for a, b in zip(runs[A.ORDER_INDEX], runs[A.ORDER_COST]):
        for x, y in zip(a, b):
            assert np.array_equal(x, y, equal_nan=True)
    assert int((runs[A.ORDER_COST][-1][3] != 0).sum()) == 0


def test_fixed_step_and_diffusion_in_a_graph(torch_cuda):
    """adm1_step_fixed and adm1_diffuse (grid build, two substeps) captured
    together into one graph: every replay equals the same eager calls bit for
    bit, with unrelated GPU work and host synchronisations between replays
    (the calls launch kernels only: no allocation, no memset)."""
    torch = torch_cuda
    from paper_2311_08927_amd import adm1 as A
    n = 3000
    w = W.cstr_population(n, seed=5)
    ctx = make_ctx(w.ld)
    g = np.random.default_rng(9)
    pos_h = np.zeros((3, w.ld), dtype=np.float32)
    pos_h[:, :n] = (g.random((3, n)) * np.array([[0.04], [0.03], [0.02]])).astype(np.float32)
    pos = torch.from_numpy(pos_h).cuda()
    V_p = 0.04 * 0.03 * 0.02 / n
    grid = A.Grid(A.make_diffusion(1.3 * V_p ** (1 / 3), 1e-9 * 86400.0, V_p, [0, 0, 0],
                                   [0.04, 0.03, 0.02]), w.ld)
    eager, graphd = DeviceWorkload(w), DeviceWorkload(w)
    dt_fixed, dt_diff = 0.5 / 86400.0, 600.0 / 86400.0

    def calls(dw):
        ctx.step_fixed(dw.X, dw.T, dw.D, dw.fidx, dw.S_in, dt_fixed, 10, A.FIXED_EULER, n=n,
                       H=dw.H, status=dw.status)
        grid.diffuse(dw.X, pos, n, dt_diff, 2)

    cg = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    with torch.cuda.graph(cg, stream=s, capture_error_mode="relaxed"):
        calls(graphd)
    try:
        junk = torch.zeros(1 << 20, device="cuda")
        for k in range(4):
            calls(eager)
            torch.cuda.synchronize()
            junk.add_(1.0)
            cg.replay()
            torch.cuda.synchronize()
            assert torch.equal(eager.X, graphd.X), k
            assert torch.equal(eager.H, graphd.H), k
            assert (graphd.status == 0).all(), k
    finally:
        del cg
        grid.close()
