"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Sizes are chosen so the oracle finishes in seconds while spanning several
64-particle tiles and a ragged tail; the full-size checks compare sampled
particles that the oracle recomputes one by one.
"""
from __future__ import annotations

import numpy as np
import pytest

from oracle.adm1 import DIFF, ND, NX, Oracle
from paper_2311_08927_amd import workloads as W
from tests.gpu_common import PARITY_TOL, DeviceWorkload, parity, run_side_by_side

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


def make_ctx(n_max, variant=None, rate_precision=0):
    from paper_2311_08927_amd.adm1 import Context
    kw = {}
    if variant is not None:
        kw["variant"] = variant
    return Context(n_max, rtol=RTOL, atol=W.atol_vector(RTOL), rate_precision=rate_precision,
                   **kw)


VARIANTS = [0, 1, 2, 3]


# ---------------------------------------------------------------------------
# right-hand side and Jacobian
# ---------------------------------------------------------------------------
def test_rhs_parity(torch_cuda, orc):
    w = W.cstr_population(200, seed=11)
    ctx = make_ctx(w.ld)
    dw = DeviceWorkload(w)
    dxdt, H, st = ctx.rhs(dw.X, dw.T, dw.D, dw.fidx, dw.S_in, n=w.n)
    dxdt = dxdt.cpu().numpy()[:, :w.n]
    H = H.cpu().numpy()
    assert (st.cpu().numpy() == 0).all()
    fo = np.zeros((ND, w.n))
    Ho = np.zeros(w.n)
    for i in range(w.n):
        f, _, h = orc.rhs(w.X[:, i], w.T[i], w.D[i], w.feed[w.fidx[i]])
        fo[:, i] = f
        Ho[i] = h
    # scale of each entry's derivative over the population
    scale = np.abs(fo).max(axis=1, keepdims=True)
    err = np.abs(dxdt - fo) / (np.abs(fo) + 1e-3 * scale)
    print(f"rhs parity: max rel err {err.max():.3e}; S_H+ rel err "
          f"{np.max(np.abs(H - Ho) / Ho):.3e}")
    assert np.max(np.abs(H - Ho) / Ho) < 1e-13
    assert err.max() < 1e-11


def test_rhs_fp32_rates_report(torch_cuda, orc):
    """FP32 rate evaluation: errors are reported; they must stay at the
    single-precision level, far from the FP64 path's."""
    w = W.cstr_population(128, seed=12)
    ctx = make_ctx(w.ld)
    dw = DeviceWorkload(w)
    d64, _, _ = ctx.rhs(dw.X, dw.T, dw.D, dw.fidx, dw.S_in, n=w.n, rate_precision=0)
    d32, _, st = ctx.rhs(dw.X, dw.T, dw.D, dw.fidx, dw.S_in, n=w.n, rate_precision=1)
    d64 = d64.cpu().numpy()[:, :w.n]
    d32 = d32.cpu().numpy()[:, :w.n]
    scale = np.abs(d64).max(axis=1, keepdims=True)
    err = np.abs(d32 - d64) / (np.abs(d64) + 1e-3 * scale)
    print("fp32-rate rhs error per entry (max):", np.array2string(err.max(axis=1),
                                                                  precision=2))
    assert (st.cpu().numpy() == 0).all()
    assert err.max() < 1e-2
    assert err.max() > 1e-12  # really computed in FP32


def test_jacobian_parity(torch_cuda, orc):
    w = W.cstr_population(64, seed=13)
    ctx = make_ctx(w.ld)
    dw = DeviceWorkload(w)
    J, st = ctx.jacobian(dw.X, dw.T, dw.D, dw.fidx, dw.S_in, n=w.n)
    J = J.cpu().numpy()
    assert (st.cpu().numpy() == 0).all()
    worst = 0.0
    for i in range(w.n):
        Jo = orc.jacobian(w.X[:, i], w.T[i], w.D[i], w.feed[w.fidx[i]])
        scale = np.abs(Jo).max(axis=1, keepdims=True) + 1e-300
        worst = max(worst, float(np.max(np.abs(J[i] - Jo) / scale)))
    print(f"jacobian parity: max row-relative err {worst:.3e}")
    assert worst < 1e-10


# ---------------------------------------------------------------------------
# the step: small populations, several tiles and a ragged tail
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("variant", VARIANTS)
def test_step_parity_cstr(torch_cuda, orc, variant):
    """CSTR-per-particle population, 200 particles (ragged last tile), the
    first 6 coupling intervals including the cold-start transient."""
    w = W.cstr_population(200, seed=1)
    ctx = make_ctx(w.ld, variant=variant)
    worst, xg, xo, stg, sto, cg, co = run_side_by_side(ctx, orc, w, steps=6)
    print(f"variant {variant}: parity {worst:.3e}; accepted steps gpu/oracle "
          f"{cg[0, :w.n].sum()}/{co[0, :w.n].sum()}; equal step counts "
          f"{np.mean(cg[0, :w.n] == co[0, :w.n]):.3f}")
    assert (stg & 0x7F == 0).all() and (sto & 0x7F == 0).all()
    assert worst <= PARITY_TOL


@pytest.mark.parametrize("n", [1, 31, 33, 65])
def test_step_parity_tiny_and_ragged(torch_cuda, orc, n):
    """Counts that leave the persistent two-lanes-per-particle kernel with a
    single particle, a part-filled wave (32 particles per wave) or one
    particle past a full wave; two intervals (cold, then warm)."""
    w = W.cstr_population(n, seed=20 + n)
    ctx = make_ctx(w.ld)
    worst, xg, xo, stg, sto, cg, co = run_side_by_side(ctx, orc, w, steps=2)
    print(f"n={n}: parity {worst:.3e}")
    assert (stg & 0x7F == 0).all() and (sto & 0x7F == 0).all()
    assert worst <= PARITY_TOL
    # columns past n are untouched
    assert np.array_equal(xg[:, n:], w.X[:, n:])


def test_step_parity_cstr_full_day(torch_cuda, orc):
    """The whole CSTR population: 256 particles, 96 coupling intervals of
    1/96 d (one simulated day), parity checked at every interval end."""
    w = W.cstr_population(256, seed=1)
    ctx = make_ctx(w.ld)
    worst, xg, xo, stg, sto, cg, co = run_side_by_side(ctx, orc, w, steps=96,
                                                       nthreads=None)
    print(f"full day: parity {worst:.3e} over 96 intervals; accepted steps in the last "
          f"interval gpu/oracle {cg[0, :w.n].sum()}/{co[0, :w.n].sum()}")
    assert (stg & 0x7F == 0).all() and (sto & 0x7F == 0).all()
    assert worst <= PARITY_TOL


def test_steady_state(torch_cuda, orc):
    """At the oracle's CSTR steady state of the nominal reactor the GPU
    right-hand side vanishes to 1e-10 of the flux scale, and one simulated
    day of GPU integration stays within 1e-8 of it."""
    import torch
    nom = W.nominal()
    x = nom["state"]
    n, ld = 64, 64
    X = np.repeat(x[:, None], ld, axis=1)
    T = np.full(n, nom["T"])
    D = np.full(n, nom["D"])
    feed = np.ascontiguousarray(nom["feed"][None, :])
    fidx = np.zeros(n, dtype=np.int32)
    ctx = make_ctx(ld)
    dX = torch.from_numpy(X).cuda()
    dT, dD = torch.from_numpy(T).cuda(), torch.from_numpy(D).cuda()
    dS, dfi = torch.from_numpy(feed).cuda(), torch.from_numpy(fidx).cuda()
    f, _, st = ctx.rhs(dX, dT, dD, dfi, dS, n=n)
    f = f.cpu().numpy()[:, :n]
    # flux scale of each entry: its dilution exchange D |x|
    rel = np.max(np.abs(f) / (D[0] * np.abs(x[np.array(DIFF)])[:, None]))
    print(f"steady state: max |f| / (D |x|) = {rel:.3e}")
    assert (st.cpu().numpy() == 0).all()
    assert rel <= 1e-10
    H = torch.full((n,), -1.0, dtype=torch.float64, device="cuda")
    hl = H.clone()
    for _ in range(96):
        ctx.step(dX, dT, dD, dfi, dS, 1.0 / 96, n=n, H=H, hlast=hl)
    xe = dX.cpu().numpy()[:, :n]
    drift = np.max(np.abs(xe - x[:, None]) / np.maximum(np.abs(x[:, None]),
                                                       1e-4 * x[:, None]))
    print(f"steady state: drift over one day {drift:.3e}")
    assert drift <= 1e-8


@pytest.mark.parametrize("variant", VARIANTS)
def test_step_parity_batched_subset(torch_cuda, orc, variant):
    """Batched population (per-particle temperature, pulsed feed zone): a
    seeded subset of 320 particles holding the zone share, 10 intervals."""
    w = W.batched_population(1 << 14, seed=2)
    rng = np.random.default_rng(5)
    zone = np.flatnonzero(w.zone)
    other = np.flatnonzero(~w.zone)
    idx = np.sort(np.concatenate([rng.choice(zone, 64, replace=False),
                                  rng.choice(other, 256, replace=False)]))
    sub = W.subset(w, idx)
    ctx = make_ctx(sub.ld, variant=variant)
    worst, xg, xo, stg, sto, cg, co = run_side_by_side(ctx, orc, sub, steps=10)
    print(f"variant {variant}: batched subset parity {worst:.3e}")
    assert (stg & 0x7F == 0).all()
    assert worst <= PARITY_TOL


@pytest.mark.parametrize("variant", VARIANTS)
def test_step_full_size_sampled(torch_cuda, orc, variant):
    """The full 2^20-particle batched population for one coupling interval in
    the benchmark's launch configuration; 96 sampled particles (zone ones
    included) recomputed by the oracle."""
    import torch
    w = W.batched_population(1 << 20, seed=2)
    ctx = make_ctx(w.ld, variant=variant)
    dw = DeviceWorkload(w)
    ctx.step(dw.X, dw.T, dw.D, dw.fidx, dw.S_in, w.dt, n=w.n, H=dw.H, hlast=dw.hlast,
             status=dw.status, nsteps=dw.nsteps)
    torch.cuda.synchronize()
    rng = np.random.default_rng(9)
    idx = np.sort(np.concatenate([rng.choice(np.flatnonzero(w.zone), 16, replace=False),
                                  rng.choice(w.n, 78, replace=False), [0, w.n - 1]]))
    idx = np.unique(idx)
    sub = W.subset(w, idx)
    Xo = sub.X.copy()
    st_o, _ = orc.step(Xo, sub.T, sub.D, sub.fidx, sub.feed, sub.dt, n=sub.n)
    xg = dw.X[:, torch.from_numpy(idx).cuda()].cpu().numpy()
    worst = parity(xg, Xo, sub.n)
    stg = dw.status.cpu().numpy()
    print(f"variant {variant}: full-size sampled parity {worst:.3e}; status counts "
          f"{np.bincount(stg & 0x7F, minlength=5)}")
    assert (stg & 0x7F == 0).all()
    assert worst <= PARITY_TOL


def test_step_full_size_warm_sampled(torch_cuda, orc):
    """The benchmark's configuration over three coupling intervals: 2^20
    particles with warm starts carried between intervals (so the work queue
    runs in cost order) and the pulsed feed zone; 96 sampled particles
    recomputed by the oracle over the same three intervals with its own warm
    starts, compared after the last one, step counts included."""
    import torch
    w = W.batched_population(1 << 20, seed=2)
    ctx = make_ctx(w.ld)
    dw = DeviceWorkload(w)
    for k in range(3):
        dw.set_D(w.D_at(k))
        ctx.step(dw.X, dw.T, dw.D, dw.fidx, dw.S_in, w.dt, n=w.n, H=dw.H, hlast=dw.hlast,
                 status=dw.status, nsteps=dw.nsteps)
    torch.cuda.synchronize()
    rng = np.random.default_rng(19)
    idx = np.unique(np.concatenate([rng.choice(np.flatnonzero(w.zone), 16, replace=False),
                                    rng.choice(w.n, 78, replace=False), [0, w.n - 1]]))
    sub = W.subset(w, idx)
    Xo = sub.X.copy()
    Ho = np.full(sub.ld, -1.0)
    hlo = np.full(sub.ld, -1.0)
    for k in range(3):
        st_o, cnt_o = orc.step(Xo, sub.T, w.D_at(k)[idx], sub.fidx, sub.feed, sub.dt, H=Ho,
                               hlast=hlo, n=sub.n)
        assert (st_o & 0x7F == 0).all()
    it = torch.from_numpy(idx).cuda()
    xg = dw.X[:, it].cpu().numpy()
    worst = parity(xg, Xo, sub.n)
    acc_g = dw.nsteps[0, it].cpu().numpy()
    stg = dw.status.cpu().numpy()
    print(f"full-size warm sampled parity {worst:.3e}; accepted steps in the third interval "
          f"GPU {acc_g.sum()} oracle {cnt_o[0, :sub.n].sum()}")
    assert (stg & 0x7F == 0).all()
    assert worst <= PARITY_TOL
    assert np.array_equal(acc_g, cnt_o[0, :sub.n])


# ---------------------------------------------------------------------------
# gas flux, determinism, edge cases
# ---------------------------------------------------------------------------
def test_gas_flux_parity_and_determinism(torch_cuda, orc):
    import torch
    w = W.cstr_population(1000, seed=21)
    ctx = make_ctx(w.ld)
    dw = DeviceWorkload(w)
    V = torch.full((w.n,), 3400.0, dtype=torch.float64, device="cuda")
    q, qc, tot = ctx.gas_flux(dw.X, dw.T, V, n=w.n)
    q2, qc2, tot2 = ctx.gas_flux(dw.X, dw.T, V, n=w.n)
    q, qc, tot = q.cpu().numpy(), qc.cpu().numpy(), tot.cpu().numpy()
    assert np.array_equal(tot, tot2.cpu().numpy())
    ref = np.array([orc.gas_flux(w.X[:, i], w.T[i], 3400.0) for i in range(w.n)])
    assert np.max(np.abs(q - ref[:, 0]) / np.maximum(ref[:, 0], 1e-300)) < 1e-13
    assert np.max(np.abs(qc - ref[:, 2]) / np.maximum(ref[:, 2], 1e-300)) < 1e-13
    assert np.allclose(tot, ref.sum(axis=0), rtol=1e-12, atol=0)


def test_step_deterministic_and_permutation_invariant(torch_cuda):
    import torch
    w = W.cstr_population(192, seed=3)
    ctx = make_ctx(w.ld)
    outs = []
    for _ in range(2):
        dw = DeviceWorkload(w)
        ctx.step(dw.X, dw.T, dw.D, dw.fidx, dw.S_in, w.dt, n=w.n, H=dw.H, hlast=dw.hlast)
        outs.append(dw.X.cpu().numpy())
    assert np.array_equal(outs[0], outs[1])
    perm = np.random.default_rng(0).permutation(w.n)
    wp = W.subset(w, perm)
    dwp = DeviceWorkload(wp)
    ctx.step(dwp.X, dwp.T, dwp.D, dwp.fidx, dwp.S_in, w.dt, n=wp.n, H=dwp.H, hlast=dwp.hlast)
    xp = dwp.X.cpu().numpy()[:, :wp.n]
    assert np.array_equal(xp, outs[0][:, perm])
    torch.cuda.synchronize()


@pytest.mark.parametrize("order,batch", [(0, 1), (0, 4), (1, 1), (1, 4)])
def test_warm_steps_independent_of_particle_placement(torch_cuda, order, batch):
    """Batched population (per-particle temperatures, pulsed feed zone): three
    coupling intervals with warm starts in index or cost order and service
    batches of 1 or 4 give, particle by particle, bit-identical states, warm
    starts and step counts when the particles are permuted (regression test:
    an out-of-line call made under a partial exec mask once changed the
    warm-start guesses of waiting pairs, so a particle's rounding depended
    on its neighbours)."""
    import torch
    from paper_2311_08927_amd import adm1 as A
    full = W.batched_population(1 << 13, seed=2)
    w = W.subset(full, np.arange(0, full.n, 16))
    perm = np.random.default_rng(0).permutation(w.n)
    inv = np.argsort(perm)
    outs = []
    for wk in (w, W.subset(w, perm)):
        ctx = make_ctx(wk.ld)
        A.adm1_set_order(ctx.handle, order)
        A.adm1_set_service_batch(ctx.handle, batch)
        dw = DeviceWorkload(wk)
        for s in range(3):
            dw.set_D(wk.D_at(s))
            ctx.step(dw.X, dw.T, dw.D, dw.fidx, dw.S_in, wk.dt, n=wk.n, H=dw.H, hlast=dw.hlast,
                     status=dw.status, nsteps=dw.nsteps)
        torch.cuda.synchronize()
        outs.append((dw.X.cpu().numpy()[:, :wk.n], dw.H.cpu().numpy()[:wk.n],
                     dw.hlast.cpu().numpy()[:wk.n], dw.nsteps.cpu().numpy()[:, :wk.n]))
        ctx.close()
    a, b = outs
    assert np.array_equal(a[0], b[0][:, inv])
    assert np.array_equal(a[1], b[1][inv]) and np.array_equal(a[2], b[2][inv])
    assert np.array_equal(a[3], b[3][:, inv])


def test_failures_are_isolated(torch_cuda):
    """Non-finite input, a bad feed row and max_steps = 1 set their status
    codes and leave those particles' states untouched; others proceed."""
    import torch
    w = W.cstr_population(128, seed=4)
    X0 = w.X.copy()
    w.X[5, 3] = np.nan
    w.fidx[7] = 10_000
    ctx = make_ctx(w.ld)
    dw = DeviceWorkload(w)
    st = ctx.step(dw.X, dw.T, dw.D, dw.fidx, dw.S_in, w.dt, n=w.n)
    st = st.cpu().numpy()
    xg = dw.X.cpu().numpy()
    assert st[3] == 4 and st[7] == 4
    assert np.isnan(xg[5, 3]) and np.array_equal(xg[:, 7], X0[:, 7])
    ok = np.setdiff1d(np.arange(w.n), [3, 7])
    assert (st[ok] & 0x7F == 0).all()
    ctx.set_opts(max_steps=1)
    dw2 = DeviceWorkload(W.cstr_population(128, seed=4))
    st2 = ctx.step(dw2.X, dw2.T, dw2.D, dw2.fidx, dw2.S_in, w.dt, n=w.n).cpu().numpy()
    assert (st2 == 3).all()
    assert np.array_equal(dw2.X.cpu().numpy(), W.cstr_population(128, seed=4).X)
    torch.cuda.synchronize()


def test_empty_and_argument_errors(torch_cuda):
    import torch
    from paper_2311_08927_amd import adm1 as A
    w = W.cstr_population(64, seed=5)
    ctx = make_ctx(w.ld)
    dw = DeviceWorkload(w)
    feed = A.feed_struct(dw.D, dw.fidx, dw.S_in)
    st = torch.zeros(w.n, dtype=torch.uint8, device="cuda")
    h = ctx.handle
    # n = 0 is a no-op
    assert A.adm1_step_particles(h, dw.X, w.ld, dw.T, feed, w.dt, 0, None, st, None) == 0
    assert A.adm1_step_particles(h, dw.X, w.ld, dw.T, feed, w.dt, w.ld + 1, None, st, None,
                                 check=False) == -2
    assert A.adm1_step_particles(h, dw.X, 100, dw.T, feed, w.dt, w.n, None, st, None,
                                 check=False) == -2
    assert A.adm1_step_particles(h, 0, w.ld, dw.T, feed, w.dt, w.n, None, st, None,
                                 check=False) == -1
    host = np.zeros((NX, w.ld))
    assert A.adm1_step_particles(h, host.ctypes.data, w.ld, dw.T, feed, w.dt, w.n, None, st,
                                 None, check=False) == -3
    assert A.adm1_step_particles(h, dw.X, w.ld, dw.T, feed, -1.0, w.n, None, st, None,
                                 check=False) == -9
    assert np.array_equal(dw.X.cpu().numpy(), w.X)
