"""Pins of the surrogate oracle (oracle/mlp.py) against what arithmetic and
the model fix: BF16 bit patterns, the normal CDF, finite differences, the
closed form of a first Adam step, Petersen-matrix continuity of the gate
weights, and the gate's verdict on an exact integrator transition."""
from __future__ import annotations

import math

import numpy as np
import pytest

from oracle import mlp as M
from oracle.adm1 import Oracle
from paper_2311_08927_amd import workloads as W


def test_bf16_rounding_bit_patterns():
    f = np.float32
    cases = {
        1.0: 0x3F80,
        -2.5: 0xC020,
        # exactly half an ulp above 1: tie to even (down)
        float(f(1.0) + f(2.0 ** -8)): 0x3F80,
        # 1 + 3 half-ulps: tie, odd lower neighbour -> up
        float(f(1.0) + f(3 * 2.0 ** -8)): 0x3F82,
        # just above a tie rounds up
        float(np.frombuffer(np.uint32(0x3F808001).tobytes(), np.float32)[0]): 0x3F81,
        float("inf"): 0x7F80,
        # the largest FP32 rounds to infinity
        float(np.finfo(np.float32).max): 0x7F80,
        0.0: 0x0000,
    }
    for x, bits in cases.items():
        assert int(M.bf16_bits(np.float32(x))) == bits, (x, hex(int(M.bf16_bits(x))), hex(bits))
    nan = M.bf16_bits(np.float32("nan"))
    assert (int(nan) & 0x7F80) == 0x7F80 and (int(nan) & 0x7F) != 0


def test_gelu_values():
    # GELU(x) = x Phi(x); Phi(1) = 0.8413447460685429 (standard normal CDF)
    assert abs(M.gelu(np.array(1.0)) - 0.8413447460685429) < 1e-15
    assert M.gelu(np.array(0.0)) == 0.0
    assert abs(M.gelu(np.array(10.0)) - 10.0) < 1e-15
    assert abs(M.gelu(np.array(-10.0))) < 1e-20
    # Phi(-1) = 1 - Phi(1)
    assert abs(M.gelu(np.array(-1.0)) + (1 - 0.8413447460685429)) < 1e-15
    z = np.linspace(-6, 6, 101)
    h = 1e-6
    fd = (M.gelu(z + h) - M.gelu(z - h)) / (2 * h)
    assert np.max(np.abs(fd - M.gelu_grad(z))) < 1e-8


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(0)
    p = M.init_params(1).astype(np.float64)
    p += 0.01 * rng.standard_normal(p.size)
    X = rng.standard_normal((4, M.IN))
    T = rng.standard_normal((4, M.OUT))
    _, g = M.loss_and_grad(p, X, T, round_bf16=False)
    assert g.size == M.NPARAMS == 216355
    # parameters of every layer, weights and biases
    offs, o = [], 0
    for i, n in M.DIMS:
        offs.append((o, i * n))
        offs.append((o + i * n, n))
        o += i * n + n
    idx = np.concatenate([rng.integers(a, a + c, 6) for a, c in offs])
    h = 1e-6
    for k in idx:
        pp, pm = p.copy(), p.copy()
        pp[k] += h
        pm[k] -= h
        fd = (M.loss_and_grad(pp, X, T, False)[0] - M.loss_and_grad(pm, X, T, False)[0]) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1e-3, abs(g[k])), (k, fd, g[k])


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(2)
    p = rng.standard_normal(100)
    g = rng.standard_normal(100)
    lr, eps = 1e-3, 1e-8
    p1, m1, v1 = M.adam_step(p, g, np.zeros(100), np.zeros(100), lr, 1, eps=eps)
    assert np.allclose(p1, p - lr * g / (np.abs(g) + eps), rtol=0, atol=1e-15)
    assert np.allclose(m1, 0.1 * g) and np.allclose(v1, 0.001 * g * g)


@pytest.fixture(scope="module")
def orc():
    return Oracle(W.params_path(), rtol=1e-8, atol=W.atol_vector(1e-8))


def test_gate_weights_close_the_petersen_matrix(orc):
    """Every process conserves the COD and nitrogen the gate weighs."""
    import json
    values = json.load(open(W.params_path()))["values"]
    cod, nw = M.gate_weights(orc, values)
    nu = orc.petersen()                      # [26][19]
    assert np.max(np.abs(cod[:26] @ nu)) < 1e-14
    assert np.max(np.abs(nw[:26] @ nu)) < 1e-14
    # nitrogen-free and COD-free entries
    assert cod[9] == cod[10] == cod[24] == cod[25] == 0.0
    assert nw[0] == nw[9] == 0.0


def test_gate_accepts_exact_transition_and_rejects_a_wrong_one(orc):
    import json
    values = json.load(open(W.params_path()))["values"]
    w = W.cstr_population(4, seed=1)
    dt = w.dt
    H = np.full(w.ld, -1.0)
    hl = np.full(w.ld, -1.0)
    X0 = w.X.copy()
    # past the initial transient of the perturbed states
    for _ in range(8):
        orc.step(X0, w.T, w.D, w.fidx, w.feed, dt, H=H, hlast=hl, n=w.n)
    X1 = X0.copy()
    orc.step(X1, w.T, w.D, w.fidx, w.feed, dt, H=H, hlast=hl, n=w.n)
    floor = 1e-6 * W.nominal()["state"]
    for i in range(w.n):
        x0, x1 = X0[:, i], X1[:, i]
        s_in = w.feed[w.fidx[i]]
        delta = np.log(np.maximum(x1, floor)) - np.log(np.maximum(x0, floor))
        ok, xs, Hs, res = M.gate(orc, values, x0, w.T[i], w.D[i], s_in, dt, delta, floor,
                                 -1.0, 5.0, 1e-6, 1e-5)
        assert ok, res
        # the projection reproduces the integrator's algebraic entries
        assert np.max(np.abs(xs - x1) / np.maximum(np.abs(x1), 1e-4 * W.nominal()["state"])) < 1e-9
        assert abs(Hs - H[i]) <= 1e-9 * H[i]
        # a 1 % error in the inorganic carbon breaks the bicarbonate equilibrium
        bad = delta.copy()
        bad[9] += 0.01
        ok2, _, _, res2 = M.gate(orc, values, x0, w.T[i], w.D[i], s_in, dt, bad, floor, -1.0,
                                 5.0, 1e-3, 1e-5)
        assert not ok2 and res2[1] > 1e-3
        # a 1 % error in X_xc breaks COD closure but not the ions
        bad = delta.copy()
        bad[12] += 0.01
        ok3, _, _, res3 = M.gate(orc, values, x0, w.T[i], w.D[i], s_in, dt, bad, floor, -1.0,
                                 5.0, 1e-3, 1e-5)
        assert not ok3 and res3[2] > 1e-5 and res3[1] < 1e-3
        # all-zero thresholds reject even the exact transition
        assert not M.gate(orc, values, x0, w.T[i], w.D[i], s_in, dt, delta, floor, -1.0,
                          0.0, 0.0, 0.0)[0]


def test_features_and_targets_invert_their_definition():
    """A state at exp(mean) standardises to zero features; a transition
    x1 = max(x0, floor) exp(mean + sd z) has targets z."""
    rng = np.random.default_rng(8)
    floor = 1e-6 * W.nominal()["state"]
    norm = {"in_mean": np.concatenate([np.log(W.nominal()["state"]) + 0.1 * rng.standard_normal(35),
                                       [308.0, math.log(1 / 96), 1.0]]),
            "in_sd": 0.5 + rng.random(38),
            "out_mean": 0.01 * rng.standard_normal(35),
            "out_sd": 0.05 + 0.1 * rng.random(35),
            "floor": floor}
    x = np.exp(norm["in_mean"][:35])[:, None]
    f = M.features(x, np.array([308.0]), np.array([1.0]), 1 / 96, norm)
    assert np.max(np.abs(f)) < 1e-5
    z = rng.standard_normal((35, 5))
    x0 = np.exp(norm["in_mean"][:35])[:, None] * np.exp(0.3 * rng.standard_normal((35, 5)))
    x1 = np.maximum(x0, floor[:, None]) * np.exp(norm["out_mean"][:, None] +
                                                norm["out_sd"][:, None] * z)
    t = M.targets(x0, x1, norm)
    assert np.max(np.abs(t - z.T)) < 1e-4
