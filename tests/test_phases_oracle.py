"""Pins of the oracle's particle phases (sec. 5, several particle kinds such
as sediments or inert matter): a phase scales every biochemical rate by its
kinetic factor, while dilution and the liquid-gas transfers act as in any
particle.  Checked against what that definition fixes: factor 1 is the
plain model, factor 0 leaves pure dilution (closed form) and a scaled factor
equals scaling every rate constant (each rate of eq. 2 is proportional to its
own constant).  CPU only."""
from __future__ import annotations

import numpy as np
import pytest

from oracle.adm1 import NX, Oracle
from paper_2311_08927_amd import workloads as W

RTOL = 1e-8
RATE_CONSTANTS = ["k_dis", "k_hyd_ch", "k_hyd_pr", "k_hyd_li", "k_m_su", "k_m_aa", "k_m_fa",
                  "k_m_c4", "k_m_pro", "k_m_ac", "k_m_h2", "k_dec_su", "k_dec_aa", "k_dec_fa",
                  "k_dec_c4", "k_dec_pro", "k_dec_ac", "k_dec_h2"]
# state entries that neither react in an inert phase nor exchange with the
# gas: only dilution moves them (S_su..S_ac, S_IN, S_I, X_*, S_cat, S_an)
DILUTION_ONLY = list(range(0, 7)) + [10, 11] + list(range(12, 24)) + [24, 25]


def _orc(values=None):
    return Oracle(values or W.params_path(), rtol=RTOL, atol=W.atol_vector(RTOL))


def _scaled(factor):
    base = dict(_orc().values)
    for k in RATE_CONSTANTS:
        base[k] = base[k] * factor
    return base


def test_factor_one_is_the_plain_model():
    w = W.cstr_population(40, seed=5)
    a, b = w.X.copy(), w.X.copy()
    orc = _orc()
    sa, ca = orc.step(a, w.T, w.D, w.fidx, w.feed, w.dt, n=w.n)
    ph = np.arange(w.n, dtype=np.uint8) % 3
    sb, cb = orc.step(b, w.T, w.D, w.fidx, w.feed, w.dt, n=w.n, phase=ph,
                      phase_kin=[1.0, 1.0, 1.0])
    assert np.array_equal(a, b) and np.array_equal(ca, cb) and np.array_equal(sa, sb)


def test_scaled_factor_equals_scaled_rate_constants():
    """rhs and a whole interval with factor 0.37 against the plain model with
    every biochemical rate constant times 0.37."""
    f = 0.37
    w = W.cstr_population(24, seed=6)
    plain, scaled = _orc(), _orc(_scaled(f))
    for i in range(w.n):
        x, T, D, s = w.X[:, i], w.T[i], w.D[i], w.feed[w.fidx[i]]
        fa, _, Ha = plain.rhs(x, T, D, s, kin=f)
        fb, _, Hb = scaled.rhs(x, T, D, s)
        assert np.allclose(fa, fb, rtol=1e-13, atol=1e-13 * np.abs(fb).max())
        assert Ha == pytest.approx(Hb, rel=1e-14)
        Ja = plain.jacobian(x, T, D, s, kin=f)
        Jb = scaled.jacobian(x, T, D, s)
        assert np.allclose(Ja, Jb, rtol=1e-12, atol=1e-12 * np.abs(Jb).max())
    a, b = w.X.copy(), w.X.copy()
    plain.step(a, w.T, w.D, w.fidx, w.feed, w.dt, n=w.n,
               phase=np.zeros(w.n, np.uint8), phase_kin=[f])
    scaled.step(b, w.T, w.D, w.fidx, w.feed, w.dt, n=w.n)
    rel = np.abs(a[:, :w.n] - b[:, :w.n]) / np.maximum(np.abs(b[:, :w.n]), 1e-12)
    assert rel.max() < 1e-9


def test_inert_phase_is_pure_dilution():
    """Factor 0 with inflow: the entries that do not meet the gas follow the
    closed form S_in + (x0 - S_in) exp(-D t); a closed inert particle keeps
    them exactly."""
    w = W.cstr_population(32, seed=7)
    orc = _orc()
    X = w.X.copy()
    D = w.D.copy()
    D[::4] = 0.0                                     # some closed particles
    st, _ = orc.step(X, w.T, D, w.fidx, w.feed, w.dt, n=w.n,
                     phase=np.ones(w.n, np.uint8), phase_kin=[1.0, 0.0])
    assert (st & 0x7F == 0).all()
    for i in range(w.n):
        s_in = w.feed[w.fidx[i]]
        for k in DILUTION_ONLY:
            want = s_in[k] + (w.X[k, i] - s_in[k]) * np.exp(-D[i] * w.dt)
            if D[i] == 0.0:
                assert X[k, i] == w.X[k, i], (i, k)
            else:
                assert X[k, i] == pytest.approx(want, rel=50 * RTOL, abs=1e-12), (i, k)


def test_phase_ids_beyond_the_table_have_factor_one():
    w = W.cstr_population(8, seed=8)
    orc = _orc()
    a, b = w.X.copy(), w.X.copy()
    orc.step(a, w.T, w.D, w.fidx, w.feed, w.dt, n=w.n)
    orc.step(b, w.T, w.D, w.fidx, w.feed, w.dt, n=w.n, phase=np.full(w.n, 200, np.uint8),
             phase_kin=[0.0, 0.0])
    assert np.array_equal(a, b)


def test_inert_fixed_step_and_rhs():
    """The fixed-step scheme and the right-hand side see the factor too: an
    inert particle's rates vanish, so its derivative of the dilution-only
    entries is D (S_in - x)."""
    w = W.cstr_population(4, seed=9)
    orc = _orc()
    x, T, D, s = w.X[:, 0], w.T[0], w.D[0], w.feed[w.fidx[0]]
    f, _, _ = orc.rhs(x, T, D, s, kin=0.0)
    # f is in integration order: entries 0..6 are state 0..6, then 8.. (S_h2
    # is algebraic); map the dilution-only state rows to it
    from oracle.adm1 import DIFF
    pos = {st: k for k, st in enumerate(DIFF)}
    for k in DILUTION_ONLY:
        assert f[pos[k]] == pytest.approx(D * (s[k] - x[k]), rel=1e-14, abs=1e-300)
    X = w.X.copy()
    orc.run_fixed(X, w.T, w.D, w.fidx, w.feed, w.dt, 64, method="rk4", n=w.n,
                  phase=np.zeros(w.n, np.uint8), phase_kin=[0.0])
    for i in range(w.n):
        s_in = w.feed[w.fidx[i]]
        for k in DILUTION_ONLY:
            want = s_in[k] + (w.X[k, i] - s_in[k]) * np.exp(-w.D[i] * w.dt)
            assert X[k, i] == pytest.approx(want, rel=1e-9, abs=1e-12)
    assert NX == 35


def test_phase_factors_independent_of_thread_count():
    """The per-particle factors live until the threaded run returns: the
    result is the same on one thread and on many (regression test: a
    temporary factor array was once freed before the threads read it)."""
    w = W.cstr_population(300, seed=51)
    ph = W.mixed_phases(w.n, seed=51, ld=w.ld)
    orc = _orc()
    outs = []
    for nt in (1, 64):
        X = w.X.copy()
        st, _ = orc.step(X, w.T, w.D, w.fidx, w.feed, w.dt, n=w.n, phase=ph,
                         phase_kin=W.PHASE_KIN, nthreads=nt)
        assert (st & 0x7F == 0).all()
        outs.append(X)
    assert np.array_equal(outs[0], outs[1])
