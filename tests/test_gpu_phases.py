"""GPU parity for particle phases (sec. 5, several particle kinds): a
mixed population of active, sediment and inert particles (kinetic factors
1, 0.25 and 0), advanced through the C ABI and by the oracle with the same
phase ids and factors."""
from __future__ import annotations

import numpy as np
import pytest

from oracle.adm1 import DIFF, ND, Oracle
from paper_2311_08927_amd import workloads as W
from tests.gpu_common import PARITY_TOL, DeviceWorkload, parity

pytestmark = pytest.mark.gpu

RTOL = 1e-8
KIN = W.PHASE_KIN
# entries that only dilution moves in an inert particle (no gas exchange)
DILUTION_ONLY = list(range(0, 7)) + [10, 11] + list(range(12, 24)) + [24, 25]


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def orc():
    return Oracle(W.params_path(), rtol=RTOL, atol=W.atol_vector(RTOL))


def _ctx(n_max, **kw):
    from paper_2311_08927_amd.adm1 import Context
    ctx = Context(n_max, rtol=RTOL, atol=W.atol_vector(RTOL), **kw)
    ctx.set_phase_kinetics(KIN)
    return ctx


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("variant", [0, 1, 2, 3])
def test_mixed_phase_step_parity(torch_cuda, orc, variant):
    """700 particles (10 full tiles and a ragged 60), three coupling
    intervals with warm starts and the pulsed dilution of the CSTR recipe;
    FP64 parity and equal accepted-step counts per particle."""
    torch = torch_cuda
    w = W.cstr_population(700, seed=51)
    ph = W.mixed_phases(w.n, seed=51, ld=w.ld)
    ctx = _ctx(w.ld, variant=variant)
    dw = DeviceWorkload(w)
    dph = _dev(torch, ph)
    Xo = w.X.copy()
    Ho, hlo = np.full(w.ld, -1.0), np.full(w.ld, -1.0)
    worst = 0.0
    for s in range(3):
        D = w.D_at(s)
        dw.set_D(D)
        ctx.step(dw.X, dw.T, dw.D, dw.fidx, dw.S_in, w.dt, n=w.n, H=dw.H, hlast=dw.hlast,
                 status=dw.status, nsteps=dw.nsteps, phase=dph)
        st_o, cnt_o = orc.step(Xo, w.T, D, w.fidx, w.feed, w.dt, H=Ho, hlast=hlo, n=w.n,
                               phase=ph, phase_kin=KIN)
        torch.cuda.synchronize()
        worst = max(worst, parity(dw.X.cpu().numpy(), Xo, w.n))
        assert (dw.status.cpu().numpy() & 0x7F == 0).all() and (st_o & 0x7F == 0).all()
        assert np.array_equal(dw.nsteps[0, :w.n].cpu().numpy(), cnt_o[0, :w.n])
    ctx.close()
    print(f"variant {variant}: mixed-phase parity {worst:.3e} "
          f"(phases {np.bincount(ph[:w.n]).tolist()})")
    assert worst <= PARITY_TOL


def test_phases_change_the_result_and_inert_closed_particles_hold(torch_cuda, orc):
    """The phases are in effect: the mixed result differs from the
    single-phase one exactly where the factor is not 1, and a closed inert
    particle keeps every entry that only dilution moves."""
    torch = torch_cuda
    w = W.cstr_population(256, seed=52)
    ph = W.mixed_phases(w.n, seed=52, ld=w.ld)
    D = w.D.copy()
    D[::3] = 0.0
    ctx = _ctx(w.ld)
    outs = []
    for phase in (None, _dev(torch, ph)):
        dw = DeviceWorkload(w)
        dw.set_D(D)
        ctx.step(dw.X, dw.T, dw.D, dw.fidx, dw.S_in, w.dt, n=w.n, status=dw.status,
                 phase=phase)
        torch.cuda.synchronize()
        assert (dw.status.cpu().numpy() & 0x7F == 0).all()
        outs.append(dw.X.cpu().numpy())
    plain, mixed = outs
    active = ph[:w.n] == 0
    assert np.array_equal(plain[:, :w.n][:, active], mixed[:, :w.n][:, active])
    assert (np.abs(plain[:, :w.n][:, ~active] - mixed[:, :w.n][:, ~active]).max(axis=0)
            > 0).all()
    inert_closed = np.flatnonzero((ph[:w.n] == 2) & (D[:w.n] == 0.0))
    assert inert_closed.size > 0
    for k in DILUTION_ONLY:
        assert np.array_equal(mixed[k, inert_closed], w.X[k, inert_closed])


def test_phase_rhs_jacobian_and_fixed_step(torch_cuda, orc):
    """adm1_rhs, adm1_jacobian and the fixed-step scheme with phases against
    the oracle's per-particle factor."""
    torch = torch_cuda
    w = W.cstr_population(130, seed=53)
    ph = W.mixed_phases(w.n, seed=53, ld=w.ld)
    ctx = _ctx(w.ld)
    dw = DeviceWorkload(w)
    dph = _dev(torch, ph)
    f, H, st = ctx.rhs(dw.X, dw.T, dw.D, dw.fidx, dw.S_in, n=w.n, phase=dph)
    J, stj = ctx.jacobian(dw.X, dw.T, dw.D, dw.fidx, dw.S_in, n=w.n, phase=dph)
    f = f.cpu().numpy()[:, :w.n]
    J = J.cpu().numpy()
    assert (st.cpu().numpy() == 0).all() and (stj.cpu().numpy() == 0).all()
    fo = np.zeros((ND, w.n))
    err_j = 0.0
    for i in range(w.n):
        kin = KIN[ph[i]]
        fo[:, i] = orc.rhs(w.X[:, i], w.T[i], w.D[i], w.feed[w.fidx[i]], kin=kin)[0]
        Jo = orc.jacobian(w.X[:, i], w.T[i], w.D[i], w.feed[w.fidx[i]], kin=kin)
        Jg = J[i].reshape(ND, ND)
        scale = np.abs(Jo).max(axis=1, keepdims=True) + 1e-300
        err_j = max(err_j, float(np.max(np.abs(Jg - Jo) / scale)))
    scale = np.abs(fo).max(axis=1, keepdims=True)
    err_f = float(np.max(np.abs(f - fo) / (np.abs(fo) + 1e-3 * scale)))
    print(f"phases: rhs parity {err_f:.3e}, jacobian row-relative {err_j:.3e}")
    assert err_f < 1e-11 and err_j < 1e-11
    # fixed-step classical RK4: one 1/96-d interval in 90 steps of 10 s
    from paper_2311_08927_amd.adm1 import FIXED_RK4
    dw2 = DeviceWorkload(w)
    stf = ctx.step_fixed(dw2.X, dw2.T, dw2.D, dw2.fidx, dw2.S_in, w.dt, 90, method=FIXED_RK4,
                         n=w.n, phase=dph)
    Xo = w.X.copy()
    sto = orc.run_fixed(Xo, w.T, w.D, w.fidx, w.feed, w.dt, 90, method="rk4", n=w.n,
                        phase=ph, phase_kin=KIN)
    torch.cuda.synchronize()
    assert (stf.cpu().numpy() == 0).all() and (sto == 0).all()
    err = parity(dw2.X.cpu().numpy(), Xo, w.n)
    print(f"phases: fixed-step RK4 parity {err:.3e}")
    assert err <= PARITY_TOL


def test_full_size_mixed_phases_sampled(torch_cuda, orc):
    """2^20 particles of the batched recipe with mixed phases for one
    interval in the default launch; 96 sampled particles recomputed by the
    oracle."""
    torch = torch_cuda
    w = W.batched_population(1 << 20, seed=2)
    ph = W.mixed_phases(w.n, seed=2, ld=w.ld)
    ctx = _ctx(w.ld)
    dw = DeviceWorkload(w)
    ctx.step(dw.X, dw.T, dw.D, dw.fidx, dw.S_in, w.dt, n=w.n, H=dw.H, hlast=dw.hlast,
             status=dw.status, nsteps=dw.nsteps, phase=_dev(torch, ph))
    torch.cuda.synchronize()
    rng = np.random.default_rng(29)
    idx = np.unique(np.concatenate([rng.choice(np.flatnonzero(ph[:w.n] == k), 24, replace=False)
                                    for k in range(3)] + [rng.choice(w.n, 22, replace=False),
                                                          [0, w.n - 1]]))
    sub = W.subset(w, idx)
    Xo = sub.X.copy()
    st_o, cnt_o = orc.step(Xo, sub.T, sub.D, sub.fidx, sub.feed, sub.dt, n=sub.n,
                           phase=ph[idx], phase_kin=KIN)
    it = torch.from_numpy(idx).cuda()
    worst = parity(dw.X[:, it].cpu().numpy(), Xo, sub.n)
    stg = dw.status.cpu().numpy()
    print(f"full-size mixed phases: sampled parity {worst:.3e}, status counts "
          f"{np.bincount(stg & 0x7F, minlength=5)}")
    assert (stg & 0x7F == 0).all() and (st_o & 0x7F == 0).all()
    assert worst <= PARITY_TOL
    assert np.array_equal(dw.nsteps[0, it].cpu().numpy(), cnt_o[0, :sub.n])


def test_phase_kinetics_validation(torch_cuda):
    from paper_2311_08927_amd.adm1 import ADM1Error
    ctx = _ctx(64)
    for bad in ([-0.5], [np.nan], [np.inf], np.ones(257)):
        with pytest.raises(ADM1Error):
            ctx.set_phase_kinetics(bad)
    ctx.set_phase_kinetics([])            # back to factor 1 everywhere
    ctx.close()


def test_default_factors_are_one(torch_cuda):
    """A phase array without a table set (every id factor 1) gives the
    single-phase result bit for bit; ids far beyond a short table too."""
    torch = torch_cuda
    from paper_2311_08927_amd.adm1 import Context
    w = W.cstr_population(100, seed=54)
    ctx = Context(w.ld, rtol=RTOL, atol=W.atol_vector(RTOL))
    outs = []
    for phase, table in ((None, None), (np.full(w.ld, 7, np.uint8), None),
                         (np.full(w.ld, 200, np.uint8), [0.0, 0.5])):
        if table is not None:
            ctx.set_phase_kinetics(table)
        dw = DeviceWorkload(w)
        ctx.step(dw.X, dw.T, dw.D, dw.fidx, dw.S_in, w.dt, n=w.n,
                 phase=None if phase is None else _dev(torch, phase))
        torch.cuda.synchronize()
        outs.append(dw.X.cpu().numpy())
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], outs[2])
    ctx.close()


def test_static_step_with_phases(torch_cuda):
    """The allocation-free entry point reads the same phase table."""
    torch = torch_cuda
    from paper_2311_08927_amd import adm1 as A
    w = W.cstr_population(300, seed=55)
    ph = _dev(torch, W.mixed_phases(w.n, seed=55, ld=w.ld))
    ctx = _ctx(w.ld)
    outs = []
    for static in (False, True):
        dw = DeviceWorkload(w)
        feed = A.feed_struct(dw.D, dw.fidx, dw.S_in, ph)
        aux = A.adm1_aux(A._ptr(dw.H), A._ptr(dw.hlast))
        fn = A.adm1_step_particles_static if static else A.adm1_step_particles
        fn(ctx.handle, dw.X, w.ld, dw.T, feed, w.dt, w.n, aux, dw.status, dw.nsteps)
        torch.cuda.synchronize()
        outs.append(dw.X.cpu().numpy())
    assert np.array_equal(outs[0], outs[1])
    ctx.close()


def test_surrogate_refuses_phases(torch_cuda):
    torch = torch_cuda
    from paper_2311_08927_amd import surrogate as S
    from paper_2311_08927_amd.adm1 import ADM1Error
    w = W.cstr_population(64, seed=56)
    ctx = _ctx(w.ld)
    sur = S.Surrogate(ctx, w.ld)
    dw = DeviceWorkload(w)
    with pytest.raises(ADM1Error, match="feed"):
        sur.step(dw.X, dw.T, dw.D, dw.fidx, dw.S_in, w.dt, S.adm1_gate(0.1, 1e-3, 1e-3), n=w.n,
                 phase=_dev(torch, W.mixed_phases(w.n, seed=56, ld=w.ld)))
    sur.close()
    ctx.close()


def test_integration_order_and_layout():
    assert len(DIFF) == ND
