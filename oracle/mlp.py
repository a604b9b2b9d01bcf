"""Oracle of the learned surrogate: plain FP64 NumPy reference of the MLP
(forward, backward, Adam), of its input features and targets, and of the
acceptance gate, used only as test infrastructure.

Storage precision follows the method's statement: BF16 weights, inputs and
hidden activations, FP32 outputs; everything else here is FP64.  BF16
rounding is round-to-nearest-even of the FP32 value (NaN kept quiet).

Pins (tests/test_mlp_oracle.py): BF16 rounding on hand-picked bit patterns;
GELU against x Phi(x) from the error function and its limits; the backward
pass against central finite differences on a small network in FP64 with
rounding off; one Adam step from zero moments against its closed form; the
gate's eq. 7 / eq. 8 projection against the integrator oracle's own solves
and the COD / nitrogen weights against the Petersen-matrix continuity.
"""
from __future__ import annotations

import math

import numpy as np

IN, HID, OUT = 38, 256, 35
IN_PAD, OUT_PAD = 64, 48
DIMS = [(IN, HID), (HID, HID), (HID, HID), (HID, HID), (HID, OUT)]
NPARAMS = sum(i * o + o for i, o in DIMS)


# ---------------------------------------------------------------------------
# BF16 rounding
# ---------------------------------------------------------------------------
def bf16_bits(x) -> np.ndarray:
    """uint16 BF16 bit patterns of x rounded through FP32, nearest-even."""
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    nan = (u & 0x7F800000) == 0x7F800000
    frac = (u & 0xFFFF) != 0
    r = (u + np.uint64(0x7FFF) + ((u >> np.uint64(16)) & np.uint64(1))) >> np.uint64(16)
    quiet = np.where(frac, np.uint64(0x40), np.uint64(0))
    r = np.where(nan, (u >> np.uint64(16)) | quiet, r)
    return (r & np.uint64(0xFFFF)).astype(np.uint16)


def bf16_value(bits) -> np.ndarray:
    """FP64 values of BF16 bit patterns."""
    b = np.asarray(bits, dtype=np.uint16).astype(np.uint32) << 16
    return b.view(np.float32).astype(np.float64)


def bf16(x) -> np.ndarray:
    return bf16_value(bf16_bits(x))


# ---------------------------------------------------------------------------
# GELU (erf form)
# ---------------------------------------------------------------------------
from scipy.special import erf as _erf  # noqa: E402


def gelu(z):
    return 0.5 * z * (1.0 + _erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + _erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(
        2.0 * math.pi)


# ---------------------------------------------------------------------------
# Parameters: flat vector, layer by layer W ([in][out]) then b ([out])
# ---------------------------------------------------------------------------
def unflatten(p: np.ndarray):
    out, o = [], 0
    for i, n in DIMS:
        W = p[o:o + i * n].reshape(i, n)
        o += i * n
        b = p[o:o + n]
        o += n
        out.append((W, b))
    assert o == p.size
    return out


def flatten(layers) -> np.ndarray:
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in layers])


def init_params(seed: int) -> np.ndarray:
    """W ~ N(0, 1/fan_in), b = 0 (seeded)."""
    rng = np.random.default_rng(seed)
    layers = [(rng.standard_normal((i, n)) / math.sqrt(i), np.zeros(n)) for i, n in DIMS]
    return flatten(layers).astype(np.float32)


# ---------------------------------------------------------------------------
# Forward / backward
# ---------------------------------------------------------------------------
def forward(p, X, round_bf16=True):
    """X: [B][38] inputs (already BF16 values when round_bf16).  Returns
    (Y [B][35], cache).  Weights enter as BF16 values and hidden activations
    are rounded to BF16 when round_bf16; biases stay FP32 values."""
    layers = unflatten(np.asarray(p, dtype=np.float64))
    q = bf16 if round_bf16 else (lambda a: a)
    a = np.asarray(X, dtype=np.float64)
    cache = []
    for li, (W, b) in enumerate(layers):
        Wq = q(W)
        z = a @ Wq + b
        cache.append((a, z, Wq))
        if li < len(layers) - 1:
            a = q(gelu(z))
    return z, cache


def loss_and_grad(p, X, T, round_bf16=True):
    """Mean squared error over the B x 35 outputs and its gradient with
    respect to the flat parameter vector (weights taken at their BF16
    values when round_bf16)."""
    Y, cache = forward(p, X, round_bf16)
    B = Y.shape[0]
    d = Y - T
    loss = float(np.sum(d * d) / (B * OUT))
    dz = 2.0 * d / (B * OUT)
    grads = []
    for li in range(len(cache) - 1, -1, -1):
        a, z, Wq = cache[li]
        grads.append((a.T @ dz, dz.sum(axis=0)))
        if li > 0:
            dh = dz @ Wq.T
            dz = dh * gelu_grad(cache[li - 1][1])
    return loss, flatten(grads[::-1])


def adam_step(p, g, m, v, lr, step, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (bias-corrected); returns (p, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


# ---------------------------------------------------------------------------
# Features and targets (FP64 arithmetic rounded to FP32 where the method
# stores FP32, then BF16 for the network input)
# ---------------------------------------------------------------------------
def features(X35, T, D, dt, norm):
    """X35: [35][n] states.  Returns BF16 values [n][38]."""
    fl = np.asarray(norm["floor"], dtype=np.float64)[:, None]
    lg = np.log(np.maximum(X35, fl)).astype(np.float32)
    raw = np.concatenate([lg, np.asarray(T, dtype=np.float32)[None, :],
                          np.full((1, X35.shape[1]), math.log(dt), dtype=np.float32),
                          (np.asarray(D) > 0).astype(np.float32)[None, :]]).T
    mean = np.asarray(norm["in_mean"], dtype=np.float32)
    sd = np.asarray(norm["in_sd"], dtype=np.float32)
    return bf16((raw - mean) / sd)


def targets(X0, X1, norm):
    """Standardised log increments [n][35] (FP32 values)."""
    fl = np.asarray(norm["floor"], dtype=np.float64)[:, None]
    d = (np.log(np.maximum(X1, fl)) - np.log(np.maximum(X0, fl))).astype(np.float32).T
    return ((d - np.asarray(norm["out_mean"], np.float32)) /
            np.asarray(norm["out_sd"], np.float32)).astype(np.float64)


# ---------------------------------------------------------------------------
# Gate
# ---------------------------------------------------------------------------
COD_ROWS = [0, 1, 2, 3, 4, 5, 6, 7, 8, 11, 12, 13, 14, 15, 16, 17, 18, 19, 20, 21, 22, 23]


def gate_weights(orc, values: dict):
    """COD and nitrogen weight of each of the 35 state rows (per unit liquid
    volume; the headspace rows weigh V_gas/V_liq).  Nitrogen contents are the
    integrator oracle's (those that close the Petersen matrix), plus 1 for
    S_IN."""
    cod = np.zeros(35)
    cod[COD_ROWS] = 1.0
    cod[32] = cod[33] = values["V_gas_per_V_liq"]
    nw = np.zeros(35)
    nw[:26] = orc.contents()[1]
    nw[10] = 1.0
    return cod, nw


def gate(orc, values, x0, T, D, s_in, dt, delta, floor, H_guess, max_dlog, tol_ion,
         tol_closure):
    """Gate of one particle.  x0: [35] pre-step state; delta: [35] log
    increments (the de-standardised network output).  Returns
    (accepted, x_hat [35] with projected algebraic entries, H, residuals
    (dlog, ion, cod, n))."""
    delta = np.asarray(delta, dtype=np.float64)
    floor = np.asarray(floor, dtype=np.float64)
    xh = np.maximum(x0, floor) * np.exp(delta)
    dl = float(np.max(np.abs(delta)))
    H = orc.solve_ph(xh, T, H_guess)
    Sh2 = orc.solve_h2(xh, T, H, D, s_in[7])
    xs = xh.copy()
    xs[7] = Sh2
    ka = [values["K_a_va"], values["K_a_bu"], values["K_a_pro"], values["K_a_ac"]]
    tc = orc.tconst(T)
    for k, (K, row) in enumerate(zip(ka, [3, 4, 5, 6])):
        xs[26 + k] = K * xh[row] / (K + H)
    xs[30] = tc["K_a_co2"] * xh[9] / (tc["K_a_co2"] + H)
    xs[31] = tc["K_a_IN"] * xh[10] / (tc["K_a_IN"] + H)
    rows = [7, 26, 27, 28, 29, 30, 31]
    ion = max(abs(xh[r] - xs[r]) / max(abs(xs[r]), 100.0 * floor[r]) for r in rows)
    cod, nw = gate_weights(orc, values)
    cin = float(np.dot(cod[:26], s_in))
    nin = float(np.dot(nw[:26], s_in))

    def outside(change, lo, hi, total):
        # distance of the change from the interval dt [lo, hi], relative
        return max(0.0, dt * lo - change, change - dt * hi) / abs(total)

    # bounds of the boundary fluxes over the interval, each factor taken
    # monotone between its end-point values
    L0, L1 = np.dot(cod[:26], x0[:26]), np.dot(cod[:26], xs[:26])
    q0, q1 = orc.gas_flux(x0, T, 1.0)[0], orc.gas_flux(xs, T, 1.0)[0]
    g0, g1 = x0[32] + x0[33], xs[32] + xs[33]
    Fc_lo = D * (cin - max(L0, L1)) - max(q0, q1) * max(g0, g1)
    Fc_hi = D * (cin - min(L0, L1)) - min(q0, q1) * min(g0, g1)
    C0, C1 = np.dot(cod, x0), np.dot(cod, xs)
    N0, N1 = np.dot(nw, x0), np.dot(nw, xs)
    rc = outside(C1 - C0, Fc_lo, Fc_hi, C0)
    rn = outside(N1 - N0, D * (nin - max(N0, N1)), D * (nin - min(N0, N1)), N0)
    ok = dl < max_dlog and ion < tol_ion and rc < tol_closure and rn < tol_closure
    return ok, xs, H, (dl, ion, rc, rn)
