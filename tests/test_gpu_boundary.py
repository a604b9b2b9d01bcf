"""GPU checks of the boundary helpers: eq. 7 alone (adm1_solve_ph) against
the oracle's eq. 7 solve, and the outcome counters (adm1_last_failures)
against the status array they summarise."""
from __future__ import annotations

import numpy as np
import pytest

from oracle.adm1 import Oracle
from paper_2311_08927_amd import workloads as W
from tests.gpu_common import DeviceWorkload

pytestmark = pytest.mark.gpu

RTOL = 1e-8
# ion totals of eq. 7: S_va, S_bu, S_pro, S_ac, S_IC, S_IN, S_cat, S_an
TOTALS = [3, 4, 5, 6, 9, 10, 24, 25]


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def orc():
    return Oracle(W.params_path(), rtol=RTOL, atol=W.atol_vector(RTOL))


def make_ctx(n_max, **kw):
    from paper_2311_08927_amd.adm1 import Context
    return Context(n_max, rtol=RTOL, atol=W.atol_vector(RTOL), **kw)


def wide_totals(n, seed):
    """Perturbed CSTR states whose eq. 7 totals are spread over a decade
    either way (lognormal sigma 1), at temperatures 30-40 C: pH from about
    5.5 to 9."""
    w = W.cstr_population(n, seed=seed)
    g = np.random.default_rng(seed + 1000)
    w.X[TOTALS, :n] *= np.exp(g.standard_normal((len(TOTALS), n)))
    w.T[:n] = g.uniform(303.15, 313.15, n)
    return w


@pytest.mark.parametrize("n", [1, 300])
def test_solve_ph_matches_oracle(torch_cuda, orc, n):
    """Element by element against the oracle's bracketed eq. 7 solve, cold
    and warm started; a ragged count (300: four 64-lane tiles and a tail)."""
    torch = torch_cuda
    w = wide_totals(n, seed=31)
    ctx = make_ctx(w.ld)
    dw = DeviceWorkload(w)
    H, pH, st = ctx.solve_ph(dw.X, dw.T, n=n)
    H = H.cpu().numpy()
    pH = pH.cpu().numpy()
    assert (st.cpu().numpy() == 0).all()
    Ho = np.array([orc.solve_ph(w.X[:, i], w.T[i]) for i in range(n)])
    rel = np.abs(H - Ho) / Ho
    print(f"solve_ph n={n}: pH {(-np.log10(Ho)).min():.2f}..{(-np.log10(Ho)).max():.2f}, "
          f"max rel err {rel.max():.2e}")
    assert rel.max() <= 1e-12
    assert np.max(np.abs(pH + np.log10(Ho))) <= 1e-12
    # warm start from a nearby value converges to the same root
    guess = torch.from_numpy(Ho * 1.3).to("cuda")
    H2, _, st2 = ctx.solve_ph(dw.X, dw.T, n=n, H_guess=guess)
    assert (st2.cpu().numpy() == 0).all()
    assert np.max(np.abs(H2.cpu().numpy() - Ho) / Ho) <= 1e-12
    # the ion totals fix S_H+: the rest of the state does not enter
    X2 = dw.X.clone()
    for k in [0, 1, 2, 12, 16, 32, 33, 34]:
        X2[k] *= 3.0
    H3, _, _ = ctx.solve_ph(X2, dw.T, n=n)
    assert torch.equal(H3, torch.from_numpy(H).to("cuda"))


def test_solve_ph_invalid_inputs(torch_cuda):
    """Non-finite totals or temperature: status 4 and NaN, others unaffected."""
    w = W.cstr_population(64, seed=32)
    w.X[9, 5] = np.nan
    w.T[9] = np.inf
    w.T[11] = -1.0
    ctx = make_ctx(w.ld)
    dw = DeviceWorkload(w)
    H, pH, st = ctx.solve_ph(dw.X, dw.T, n=w.n)
    st = st.cpu().numpy()
    H = H.cpu().numpy()
    bad = [5, 9, 11]
    assert (st[bad] == 4).all() and np.isnan(H[bad]).all()
    ok = np.setdiff1d(np.arange(w.n), bad)
    assert (st[ok] == 0).all() and np.isfinite(H[ok]).all()


def test_last_failures_counts_the_status(torch_cuda):
    """The counters equal the host's count of the step's status array, for
    the adaptive step and the fixed-step scheme, and a call with n = 0
    clears them."""
    torch = torch_cuda
    w = W.cstr_population(200, seed=33)
    w.X[5, 3] = np.nan       # non-finite input
    w.fidx[7] = 10_000       # feed row out of range
    w.T[11] = np.nan
    ctx = make_ctx(w.ld)
    dw = DeviceWorkload(w)
    st = ctx.step(dw.X, dw.T, dw.D, dw.fidx, dw.S_in, w.dt, n=w.n).cpu().numpy()
    c = ctx.last_failures()
    code = st & 0x7F
    assert c["counted"] == w.n
    assert c["failed"] == int((code != 0).sum()) == 3
    assert c["nonfinite"] == 3
    for k, name in [(1, "algebraic"), (2, "underflow"), (3, "max_steps")]:
        assert c[name] == int((code == k).sum()) == 0
    assert c["negative"] == int(((code == 0) & ((st & 0x80) != 0)).sum())
    # max_steps = 1: every valid particle stops with code 3
    ctx.set_opts(max_steps=1)
    dw2 = DeviceWorkload(W.cstr_population(200, seed=33))
    st2 = ctx.step(dw2.X, dw2.T, dw2.D, dw2.fidx, dw2.S_in, w.dt, n=w.n).cpu().numpy()
    c2 = ctx.last_failures()
    assert c2["max_steps"] == int(((st2 & 0x7F) == 3).sum()) == w.n
    assert c2["failed"] == w.n
    ctx.set_opts(max_steps=100000)
    # the fixed-step scheme reports through the same counters
    dw3 = DeviceWorkload(W.cstr_population(200, seed=34))
    st3 = ctx.step_fixed(dw3.X, dw3.T, dw3.D, dw3.fidx, dw3.S_in, 0.5 / 86400.0, 10,
                         n=w.n).cpu().numpy()
    c3 = ctx.last_failures()
    assert c3["counted"] == w.n and c3["failed"] == int(((st3 & 0x7F) != 0).sum()) == 0
    # an empty call resets
    ctx.step(dw3.X, dw3.T, dw3.D, dw3.fidx, dw3.S_in, w.dt, n=0,
             status=torch.zeros(1, dtype=torch.uint8, device="cuda"))
    c4 = ctx.last_failures()
    assert all(v == 0 for v in c4.values())



def test_last_failures_past_one_grid_pass(torch_cuda):
    """The count runs on a fixed grid of 256 blocks of 256 threads, each
    thread taking 16 consecutive status bytes per pass: one pass covers
    2^20 bytes.  With 2^20 + 53 particles the first threads take a second
    pass and the last 5 bytes are a ragged end read byte by byte.  Invalid
    inputs planted on both sides of a 16-byte group, of the pass boundary
    and in the ragged end are all counted, and the counts equal the host's
    count of the status array."""
    n = (1 << 20) + 53
    w = W.cstr_population(n, seed=35)
    ctx = make_ctx(w.ld)
    dw = DeviceWorkload(w)
    bad = [0, 15, 16, (1 << 20) - 1, 1 << 20, (1 << 20) + 1, n - 5, n - 1]
    for i in bad[::2]:
        dw.X[4, i] = float("nan")
    for i in bad[1::2]:
        dw.T[i] = -1.0
    st = ctx.step_fixed(dw.X, dw.T, dw.D, dw.fidx, dw.S_in, 0.5 / 86400.0, 10,
                        n=w.n).cpu().numpy()
    c = ctx.last_failures()
    code = st & 0x7F
    assert c["counted"] == w.n
    assert sorted(np.nonzero(code)[0].tolist()) == bad
    assert c["failed"] == c["nonfinite"] == int((code == 4).sum()) == len(bad)
    assert c["negative"] == int(((code == 0) & ((st & 0x80) != 0)).sum())


def test_init_refuses_non_integer_hill_exponents(torch_cuda):
    """The kernels take the pH inhibition's power by multiplication, so a
    parameter set whose Hill exponent 3 / (pH_UL - pH_LL) is not an integer
    from 1 to 4 is refused at initialisation; integer ones are accepted."""
    from paper_2311_08927_amd import adm1 as A
    base = A.load_params()
    for ul, ok in ((5.5, True), (5.0, True), (4.75, True), (7.0, True), (5.2, False),
                   (4.5, False), (10.0, False)):
        vals = dict(base, pH_UL_aa=ul)
        if ok:
            A.Context(64, rtol=1e-8, atol=W.atol_vector(1e-8), params=vals).close()
        else:
            with pytest.raises(A.ADM1Error, match="-4"):
                A.Context(64, rtol=1e-8, atol=W.atol_vector(1e-8), params=vals)
