"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: closed
forms, conservation laws of eq. 2, the order conditions of the published
Rosenbrock tableau, brute-force references, the half-points of the
inhibition forms of eqs. 3-6, and finite differences.
"""
from __future__ import annotations

import json
import math
import os

import numpy as np
import pytest

from oracle.adm1 import DIFF, ND, NLIQ, NX, Oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PARAMS = os.path.join(ROOT, "paper_2311_08927_amd", "data", "adm1_params.json")
NOMINAL = os.path.join(ROOT, "paper_2311_08927_amd", "data", "nominal.json")

NAMES = ["S_su", "S_aa", "S_fa", "S_va", "S_bu", "S_pro", "S_ac", "S_h2", "S_ch4", "S_IC",
         "S_IN", "S_I", "X_xc", "X_ch", "X_pr", "X_li", "X_su", "X_aa", "X_fa", "X_c4",
         "X_pro", "X_ac", "X_h2", "X_I", "S_cat", "S_an", "S_va_ion", "S_bu_ion",
         "S_pro_ion", "S_ac_ion", "S_hco3_ion", "S_nh3", "G_h2", "G_ch4", "G_co2"]
IX = {n: i for i, n in enumerate(NAMES)}
COD_LIQ = ["S_su", "S_aa", "S_fa", "S_va", "S_bu", "S_pro", "S_ac", "S_h2", "S_ch4", "S_I",
           "X_xc", "X_ch", "X_pr", "X_li", "X_su", "X_aa", "X_fa", "X_c4", "X_pro", "X_ac",
           "X_h2", "X_I"]
T0 = 308.15
DT = 1.0 / 96.0


def values():
    with open(PARAMS) as fh:
        return json.load(fh)["values"]


def nominal():
    with open(NOMINAL) as fh:
        d = json.load(fh)
    return np.array(d["state"]), np.array(d["feed"]), d["D"], d["T"]


def perturbed(seed, sigma=0.2):
    x, feed, D, T = nominal()
    g = np.random.default_rng(seed)
    x = x.copy()
    x[DIFF] *= np.exp(sigma * g.standard_normal(ND))
    return x, feed, D, T


def perturbed_smooth(seed):
    """Perturbed state for the smooth-solution pins (used with a closed
    headspace valve, whose clipped outflow law would put a kink in f)."""
    return perturbed(seed)


def closed_valve(rtol, atol=None):
    v = values()
    v["k_p_per_V_liq"] = 0.0
    return Oracle(v, rtol=rtol, atol=atol)


@pytest.fixture(scope="module")
def orc():
    return Oracle(PARAMS, rtol=1e-8)


# ---------------------------------------------------------------------------
# Rosenbrock tableau: order conditions (Hairer & Wanner, sec. IV.7)
# ---------------------------------------------------------------------------
def test_rodas4_order_conditions(orc):
    """The transformed (a, c) coefficients map back to (alpha, gamma, b); the
    method must satisfy the 8 order conditions of order 4 and the embedded
    method those of order 3."""
    g, A, C = orc.rodas4_tableau()
    s = 6
    # Gamma^{-1} = diag(1/gamma) - C (strictly lower C)
    Ginv = np.diag(np.full(s, 1.0 / g))
    for i in range(s):
        for j in range(i):
            Ginv[i, j] = -C[i, j]
    G = np.linalg.inv(Ginv)
    Afull = np.zeros((s, s))
    Afull[:, :5] = A
    alpha = Afull @ G
    alpha = np.tril(alpha, -1)
    m = np.array([A[5, 0], A[5, 1], A[5, 2], A[5, 3], 1.0, 1.0])
    mhat = np.array([A[5, 0], A[5, 1], A[5, 2], A[5, 3], 1.0, 0.0])
    b = m @ G
    bh = mhat @ G
    gam = G - np.diag(np.diag(G))  # gamma_ij, i > j
    beta = alpha + gam
    ai = alpha.sum(1)
    bp = beta.sum(1)

    def conds(w, order):
        c = [w.sum() - 1, w @ bp - (0.5 - g), w @ ai**2 - 1 / 3,
             w @ beta @ bp - (1 / 6 - g + g * g)]
        if order >= 4:
            c += [w @ ai**3 - 0.25, (w * ai) @ alpha @ bp - (1 / 8 - g / 3),
                  w @ beta @ ai**2 - (1 / 12 - g / 3),
                  w @ beta @ beta @ bp - (1 / 24 - g / 2 + 1.5 * g * g - g**3)]
        return np.abs(np.array(c))

    assert conds(b, 4).max() < 1e-12
    assert conds(bh, 3).max() < 1e-12
    # the embedded solution is NOT of order 4, so y1 - yhat1 is a genuine
    # O(h^4) error estimate (an embedded order-4 solution would make it vanish)
    assert conds(bh, 4).max() > 1e-3


# ---------------------------------------------------------------------------
# Stoichiometry: COD, N, C continuity per process (eq. 2 with the Petersen
# matrix of the standard ADM1)
# ---------------------------------------------------------------------------
def test_petersen_continuity(orc):
    nu = orc.petersen()
    C, N = orc.contents()
    cod = np.array([IX[n] for n in COD_LIQ])
    for j in range(19):
        assert abs(nu[cod, j].sum()) < 1e-15 * 10, j
        # carbon: organic C + S_IC; nitrogen: organic N + S_IN
        assert abs(C @ nu[:, j] + nu[IX["S_IC"], j]) < 1e-15, j
        assert abs(N @ nu[:, j] + nu[IX["S_IN"], j]) < 1e-15, j
    # every process consumes exactly one unit of its substrate or biomass
    subs = ["X_xc", "X_ch", "X_pr", "X_li", "S_su", "S_aa", "S_fa", "S_va", "S_bu",
            "S_pro", "S_ac", "S_h2", "X_su", "X_aa", "X_fa", "X_c4", "X_pro", "X_ac", "X_h2"]
    for j, s in enumerate(subs):
        assert nu[IX[s], j] == -1.0


def _rhs_full(orc, x, T, D, feed):
    f, xa, H = orc.rhs(x, T, D, feed)
    dx = np.zeros(NX)
    dx[DIFF] = f
    return dx, xa


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_global_balances(orc, seed):
    """d/dt [V_l COD_l + V_g COD_g] = q (COD_in - COD_l) - q_gas COD_g, and the
    same for N and C, to round-off (eq. 2 plus the headspace balance)."""
    x, feed, D, T = perturbed(seed)
    v = values()
    vg = v["V_gas_per_V_liq"]
    dx, xa = _rhs_full(orc, x, T, D, feed)
    r = orc.rates(xa, T, orc.rhs(x, T, D, feed)[2])
    q = r[22]
    C, N = orc.contents()
    cod = np.array([IX[n] for n in COD_LIQ])
    cod_l = xa[cod].sum()
    cod_in = feed[cod].sum()
    lhs = sum(dx[i] for i in cod if i != IX["S_h2"]) + vg * (dx[IX["G_h2"]] + dx[IX["G_ch4"]])
    rhs = D * (cod_in - cod_l) - q * (xa[IX["G_h2"]] + xa[IX["G_ch4"]])
    scale = D * (cod_in + cod_l) + abs(lhs) + 1.0
    assert abs(lhs - rhs) < 1e-13 * scale
    # nitrogen
    lhs = N @ dx[:NLIQ] + dx[IX["S_IN"]]
    rhs = D * (N @ feed + feed[IX["S_IN"]] - N @ xa[:NLIQ] - xa[IX["S_IN"]])
    assert abs(lhs - rhs) < 1e-13 * (abs(D) + 1.0)
    # carbon (methane carries C_ch4 per kg COD into the gas)
    cc = C.copy()
    lhs = cc @ dx[:NLIQ] + dx[IX["S_IC"]] + vg * (C[IX["S_ch4"]] * dx[IX["G_ch4"]]
                                                   + dx[IX["G_co2"]])
    rhs = (D * (cc @ feed + feed[IX["S_IC"]] - cc @ xa[:NLIQ] - xa[IX["S_IC"]])
           - q * (C[IX["S_ch4"]] * xa[IX["G_ch4"]] + xa[IX["G_co2"]]))
    assert abs(lhs - rhs) < 1e-12 * (abs(D) + 1.0)


def test_closed_reactor_conserves(orc):
    """No transport and no gas transfer: the reaction terms alone conserve
    COD, N and C exactly."""
    v = values()
    v.update(k_L_a=0.0, k_p_per_V_liq=0.0)
    o = Oracle(v, rtol=1e-8)
    x, feed, _, T = perturbed(5)
    dx, xa = _rhs_full(o, x, T, 0.0, feed)
    C, N = o.contents()
    cod = [IX[n] for n in COD_LIQ if n != "S_h2"]
    assert abs(sum(dx[i] for i in cod)) < 1e-14 * 50
    assert abs(N @ dx[:NLIQ] + dx[IX["S_IN"]]) < 1e-15 * 10
    assert abs(C @ dx[:NLIQ] + dx[IX["S_IC"]]) < 1e-15 * 10


# ---------------------------------------------------------------------------
# Eq. 7 (charge balance) and eq. 8 (S_h2 balance)
# ---------------------------------------------------------------------------
def test_pure_water(orc):
    x = np.zeros(NX)
    H = orc.solve_ph(x, T0)
    Kw = orc.tconst(T0)["K_w"]
    assert abs(H - math.sqrt(Kw)) <= 1e-14 * math.sqrt(Kw)


@pytest.mark.parametrize("a", [1e-6, 1e-4, 1e-2])
def test_strong_acid(orc, a):
    x = np.zeros(NX)
    x[IX["S_an"]] = a
    Kw = orc.tconst(T0)["K_w"]
    H = orc.solve_ph(x, T0)
    ref = 0.5 * (a + math.sqrt(a * a + 4 * Kw))
    assert abs(H - ref) <= 1e-13 * ref


@pytest.mark.parametrize("c,a", [(0.0, 0.5), (0.002, 0.5), (0.01, 1.0), (0.05, 0.2)])
def test_acetate_cation_cubic(orc, c, a):
    """Acetate (a kg COD/m3 = a/64 kmol) plus cation c: eq. 7 reduces to a
    cubic in S_H+; its positive root (numpy.roots) must match."""
    v = values()
    x = np.zeros(NX)
    x[IX["S_ac"]] = a
    x[IX["S_cat"]] = c
    Kw = orc.tconst(T0)["K_w"]
    Ka = v["K_a_ac"]
    A = a / 64.0
    # (c + H) H (Ka + H) - A Ka H - Kw (Ka + H) = 0
    coef = [1.0, c + Ka, c * Ka - A * Ka - Kw, -Kw * Ka]
    roots = np.roots(coef)
    pos = [r.real for r in roots if abs(r.imag) < 1e-20 and r.real > 0]
    assert len(pos) == 1
    H = orc.solve_ph(x, T0)
    assert abs(H - pos[0]) <= 1e-10 * pos[0]


def test_charge_balance_residual_random(orc):
    rng = np.random.default_rng(11)
    for _ in range(200):
        x = np.zeros(NX)
        for n in ["S_va", "S_bu", "S_pro", "S_ac"]:
            x[IX[n]] = 10 ** rng.uniform(-4, 1)
        for n in ["S_IC", "S_IN", "S_cat", "S_an"]:
            x[IX[n]] = 10 ** rng.uniform(-4, -0.5)
        T = rng.uniform(300, 320)
        H = orc.solve_ph(x, T)
        r = orc.charge_residual(x, T, H)
        scale = sum(abs(x[IX[n]]) for n in ["S_IC", "S_IN", "S_cat", "S_an"]) + \
            sum(x[IX[n]] for n in ["S_va", "S_bu", "S_pro", "S_ac"]) / 64 + H
        assert abs(r) <= 1e-13 * scale
        # unique root: residual changes sign across it
        assert orc.charge_residual(x, T, H * (1 - 1e-9)) < 0 < orc.charge_residual(
            x, T, H * (1 + 1e-9))


def test_h2_transfer_only_closed_form(orc):
    """No substrates and no biomass: eq. 8 reduces to
    D (S_in - S) - kLa (S - K_H RT G_h2) = 0."""
    v = values()
    x = np.zeros(NX)
    x[IX["G_h2"]] = 3e-5
    x[IX["S_IN"]] = 0.05
    D, s_in = 0.3, 4e-7
    c = orc.tconst(T0)
    S = orc.solve_h2(x, T0, 1e-7, D, s_in)
    ref = (D * s_in + v["k_L_a"] * c["K_H_h2"] * c["RT"] * x[IX["G_h2"]]) / (D + v["k_L_a"])
    assert abs(S - ref) <= 1e-13 * ref


def test_h2_root_monotone(orc):
    x, feed, D, T = perturbed(3)
    H = orc.solve_ph(x, T)
    S = orc.solve_h2(x, T, H, D, feed[IX["S_h2"]])
    assert S > 0
    y = x.copy()
    y[IX["S_h2"]] = S * (1 - 1e-8)
    hi = orc.h2_residual(y, T, H, D, feed[IX["S_h2"]])
    y[IX["S_h2"]] = S * (1 + 1e-8)
    lo = orc.h2_residual(y, T, H, D, feed[IX["S_h2"]])
    assert hi > 0 > lo


# ---------------------------------------------------------------------------
# Rate laws: inhibition half points (eqs. 3-6) and the Monod structure
# ---------------------------------------------------------------------------
def test_inhibition_half_points(orc):
    from oracle.adm1 import lib
    L = lib()
    assert L.orc_inhib(0, 0.0, 2e-6, 0) == 1.0            # eq. 5 at S_I = 0
    assert abs(L.orc_inhib(0, 2e-6, 2e-6, 0) - 0.5) < 1e-15   # eq. 5 at S_I = K_I
    assert abs(L.orc_inhib(1, 3e-4, 3e-4, 0) - 0.5) < 1e-15   # eq. 6 at S_I = K_I
    for LL, UL in [(4.0, 5.5), (6.0, 7.0), (5.0, 6.0)]:
        Hmid = 10 ** (-(LL + UL) / 2)                           # eq. 4 half point
        assert abs(L.orc_inhib(2, Hmid, LL, UL) - 0.5) < 1e-13
        # fully active at high pH, inhibited at low pH
        assert L.orc_inhib(2, 10 ** -(UL + 1), LL, UL) > 0.99
        assert L.orc_inhib(2, 10 ** -(LL - 1), LL, UL) < 0.01
        # the exponent: with n = 3/(UL - LL) the Hill form is a logistic in pH
        # that rises by 3 decades of (S_H+/K)^n between the limits, so at
        # pH = UL it reads 1/(1 + 10^-1.5) = 0.969346 and at pH = LL
        # 1/(1 + 10^1.5) = 0.030654 (n = 2/(UL - LL) would give 0.909, 0.091)
        assert abs(L.orc_inhib(2, 10 ** -UL, LL, UL) - 0.9693465699682844) < 1e-12
        assert abs(L.orc_inhib(2, 10 ** -LL, LL, UL) - 0.030653430031715604) < 1e-12


UPTAKE = [  # process index, substrate, K_S, biomass, k_m
    (4, "S_su", "K_S_su", "X_su", "k_m_su"), (5, "S_aa", "K_S_aa", "X_aa", "k_m_aa"),
    (6, "S_fa", "K_S_fa", "X_fa", "k_m_fa"), (9, "S_pro", "K_S_pro", "X_pro", "k_m_pro"),
    (10, "S_ac", "K_S_ac", "X_ac", "k_m_ac"), (11, "S_h2", "K_S_h2", "X_h2", "k_m_h2")]


@pytest.mark.parametrize("j,sub,KS,bio,km", UPTAKE)
def test_monod_structure(orc, j, sub, KS, bio, km):
    """Uptake rates are linear in their biomass, reach half their maximum at
    S = K_S of their own substrate, and the maximum is k_m X times the
    inhibition factors (pH fully active, N in excess, no h2/nh3)."""
    v = values()
    x = np.zeros(NX)
    x[IX["S_IN"]] = 1e3          # I_IN -> 1
    x[IX[bio]] = 0.7
    H = 1e-10                    # pH 10: every Hill factor -> 1
    x[IX[sub]] = v[KS]
    half = orc.rates(x, T0, H)[j]
    x[IX[sub]] = 1e12 * v[KS]
    full = orc.rates(x, T0, H)[j]
    if sub != "S_ac":  # acetate uptake is also inhibited by free ammonia (eq. 5)
        assert abs(full - v[km] * 0.7) <= 1e-6 * full
    assert abs(half / full - 0.5) < 1e-6
    x[IX[bio]] = 1.4
    assert abs(orc.rates(x, T0, H)[j] / full - 2.0) < 1e-12


def test_c4_competition(orc):
    v = values()
    x = np.zeros(NX)
    x[IX["S_IN"]] = 1e3
    x[IX["X_c4"]] = 1.0
    x[IX["S_va"]] = 1e9
    x[IX["S_bu"]] = 1e9
    r = orc.rates(x, T0, 1e-10)
    # equal excess of valerate and butyrate share the c4 capacity equally
    assert abs(r[7] - 0.5 * v["k_m_c4"]) < 1e-6 * v["k_m_c4"]
    assert abs(r[8] - 0.5 * v["k_m_c4"]) < 1e-6 * v["k_m_c4"]


def test_h2_inhibition_of_uptake(orc):
    """The LCFA, c4 and propionate uptakes are halved at S_h2 = K_I (eq. 5)."""
    v = values()
    x = np.zeros(NX)
    x[IX["S_IN"]] = 1e3
    for n in ["X_fa", "X_c4", "X_pro"]:
        x[IX[n]] = 1.0
    for n in ["S_fa", "S_va", "S_pro"]:
        x[IX[n]] = 1.0
    base = orc.rates(x, T0, 1e-10)
    for j, K in [(6, "K_I_h2_fa"), (7, "K_I_h2_c4"), (9, "K_I_h2_pro")]:
        y = x.copy()
        y[IX["S_h2"]] = v[K]
        assert abs(orc.rates(y, T0, 1e-10)[j] / base[j] - 0.5) < 1e-12


def test_arrhenius_and_vant_hoff(orc):
    v = values()
    c0 = orc.tconst(v["T_ref_kin"])
    assert abs(c0["arr"] - 1.0) < 1e-15
    cb = orc.tconst(v["T_base"])
    assert abs(cb["K_w"] - v["K_w_base"]) < 1e-28
    c1 = orc.tconst(318.15)
    # 55 kJ/mol roughly doubles the rates per 10 K near 35 C
    assert 1.8 < c1["arr"] < 2.1


def test_vant_hoff_against_physical_tables(orc):
    """Temperature dependence away from T_base, against measured values of
    the constants at 35 C (308.15 K) from standard tables.  A flipped sign of
    (1/T_base - 1/T), or a wrong enthalpy scale, moves every one of them far
    outside these bands (e.g. pK_w 14.32 instead of 13.68).

    Table values (independent of the parameter file):
      * pK_w(35 C) = 13.680 (ion product of water, CRC Handbook);
      * p_h2o(35 C) = 5.628 kPa (saturated water vapour, CRC Handbook); the
        parameter set's exponential form is an approximation, within 2 %;
      * pK_a1 of carbonic acid 6.309 at 35 C (Harned & Davis 1943);
      * pK_a of NH4+ 0.09018 + 2729.92/T (Emerson et al. 1975): 8.949;
      * Henry's law solubility ratios k_H(35 C)/k_H(25 C) from the
        d ln k_H / d(1/T) of Sander's compilation (2015): CO2 2400 K -> 0.770,
        CH4 1600 K -> 0.840, H2 500 K -> 0.947.
    """
    c = orc.tconst(308.15)
    cb = orc.tconst(298.15)
    assert abs(-math.log10(c["K_w"]) - 13.680) < 0.01
    assert abs(c["p_h2o"] / 0.05628 - 1.0) < 0.02
    assert abs(-math.log10(c["K_a_co2"]) - 6.309) < 0.01
    assert abs(-math.log10(c["K_a_IN"]) - (0.09018 + 2729.92 / 308.15)) < 0.02
    assert abs(c["K_H_co2"] / cb["K_H_co2"] / 0.770 - 1.0) < 0.02
    assert abs(c["K_H_ch4"] / cb["K_H_ch4"] / 0.840 - 1.0) < 0.02
    assert abs(c["K_H_h2"] / cb["K_H_h2"] / 0.947 - 1.0) < 0.01
    # R T in bar m3/kmol at 35 C (ideal gas): 0.0831446 * 308.15
    assert abs(c["RT"] - 25.6211) < 1e-3


def _headspace_state(T, p_h2, p_ch4, p_co2):
    """Nominal liquid with the headspace set to given partial pressures
    (bar); COD per kmol is 16 for H2 and 64 for CH4."""
    x, _, _, _ = nominal()
    x = x.copy()
    RT = 0.083145 * T
    x[IX["G_h2"]] = 16.0 * p_h2 / RT
    x[IX["G_ch4"]] = 64.0 * p_ch4 / RT
    x[IX["G_co2"]] = p_co2 / RT
    return x


def test_valve_law_worked_example(orc):
    """Gas outflow through the headspace valve (sec. 2.2 gas release; Table 1
    P_atm = 1.013 bar, tank V_liq = 3400 m3 with k_p = 5e4 m3/(d bar)).

    Worked by hand at T_base = 298.15 K, where p_h2o is its base value
    0.0313 bar: p_ch4 = 1.2, p_co2 = 0.7947, p_h2 = 0 bar give
    P_gas = 1.2 + 0.7947 + 0.0313 = 2.026 bar = 2 P_atm.  The outflow,
    k_p (P_gas - P_atm) P_gas / P_atm = 5e4 * 1.013 * 2 = 101,300 m3/d for
    the tank, i.e. 101300/3400 = 29.7941176... per m3 of liquid; its methane
    share is q p_ch4 / P_gas = 50,000 * 1.2 = 60,000 m3/d and its CO2 share
    50,000 * 0.7947 = 39,735 m3/d.  Dropping the P_gas/P_atm factor gives
    50,650; using P_gas instead of the overpressure gives 202,600."""
    T = 298.15
    x = _headspace_state(T, 0.0, 1.2, 0.7947)
    q = orc.gas_flux(x, T, 3400.0)
    assert abs(q[0] - 101300.0) < 1e-8 * 101300.0
    assert q[1] == 0.0
    assert abs(q[2] - 60000.0) < 1e-8 * 60000.0
    assert abs(q[3] - 39735.0) < 1e-8 * 39735.0
    r = orc.rates(x, T, 1e-7)
    assert abs(r[22] - 101300.0 / 3400.0) < 1e-12 * 30.0
    assert abs(r[26] - 2.026) < 1e-12
    # the rates and the headspace balance use the same outflow: with the
    # liquid-gas transfer switched off, dG_i/dt = -(q/V_liq) G_i / (V_gas/V_liq)
    v = values()
    v["k_L_a"] = 0.0
    o2 = Oracle(v, rtol=1e-8)
    f, _, _ = o2.rhs(x, T, 0.0, np.zeros(NLIQ))
    dx = np.zeros(NX)
    dx[DIFF] = f
    vg = v["V_gas_per_V_liq"]
    for g in ["G_ch4", "G_co2"]:
        want = -(101300.0 / 3400.0) * x[IX[g]] / vg
        assert abs(dx[IX[g]] - want) < 1e-12 * abs(want), g


def test_valve_closed_at_or_below_atmosphere(orc):
    """No flow while the headspace is at or below P_atm (the valve does not
    draw air in): P_gas = 0.9 bar and P_gas = P_atm exactly both give zero,
    and the methane share is zero with it."""
    T = 298.15
    for p_ch4, p_co2 in [(0.5, 0.3687), (0.6, 1.013 - 0.6 - 0.0313)]:
        x = _headspace_state(T, 0.0, p_ch4, p_co2)
        P = p_ch4 + p_co2 + 0.0313
        assert P <= 1.013 + 1e-15
        q = orc.gas_flux(x, T, 3400.0)
        assert (q == 0.0).all(), (P, q)
        assert orc.rates(x, T, 1e-7)[22] == 0.0
    # just above P_atm the flow starts at zero and grows linearly:
    # q ~ k_p dP for a small overpressure dP
    dP = 1e-6
    x = _headspace_state(T, 0.0, 0.6, 1.013 - 0.6 - 0.0313 + dP)
    q = orc.gas_flux(x, T, 3400.0)[0]
    assert abs(q / (5e4 * dP) - 1.0) < 1e-5


# ---------------------------------------------------------------------------
# Jacobian: complex step against central finite differences
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("seed", [1, 7])
def test_jacobian_vs_finite_differences(orc, seed):
    x, feed, D, T = perturbed(seed)
    J = orc.jacobian(x, T, D, feed)
    Jfd = np.zeros_like(J)
    for k, row in enumerate(DIFF):
        h = 1e-6 * max(abs(x[row]), 1e-8)
        xp = x.copy(); xp[row] += h
        xm = x.copy(); xm[row] -= h
        Jfd[:, k] = (orc.rhs(xp, T, D, feed)[0] - orc.rhs(xm, T, D, feed)[0]) / (2 * h)
    scale = np.abs(J).max(axis=1, keepdims=True) + 1e-12
    assert np.max(np.abs(J - Jfd) / scale) < 2e-5


# ---------------------------------------------------------------------------
# Integrator: closed forms, small-step reference, order, steady state
# ---------------------------------------------------------------------------
def _run(o, x, T, D, feed, dt, steps=1):
    X = x.reshape(NX, 1).copy()
    H = np.array([-1.0]); hl = np.array([-1.0])
    for _ in range(steps):
        st, _ = o.step(X, [T], [D], [0], feed[None, :], dt, H=H, hlast=hl, nthreads=1)
        assert (st[0] & 0x7F) == 0, st
    return X[:, 0]


def test_washout_closed_form():
    """All kinetic constants and the gas exchange zero: every liquid entry
    relaxes as x_in + (x0 - x_in) exp(-D t)."""
    v = values()
    for k in list(v):
        if k.startswith(("k_m_", "k_dec_", "k_hyd_")) or k in ("k_dis",):
            v[k] = 0.0
    v.update(k_L_a=0.0, k_p_per_V_liq=0.0)
    o = Oracle(v, rtol=1e-10, atol=np.full(ND, 1e-14))
    x, feed, D, T = perturbed(2)
    D = 3.0
    t = 0.5
    xe = _run(o, x, T, D, feed, t)
    liq = [i for i in range(NLIQ) if i != IX["S_h2"]]
    ref = feed[liq] + (x[liq] - feed[liq]) * math.exp(-D * t)
    assert np.max(np.abs(xe[liq] - ref) / np.abs(ref)) < 1e-8
    # gas untouched
    assert np.array_equal(xe[32:35], x[32:35])


def test_bateman_chain():
    """No biomass, closed reactor: disintegration and hydrolysis are a linear
    chain X_xc -> X_ch/X_pr/X_li/S_I/X_I with closed-form (Bateman) solutions."""
    v = values()
    o = Oracle(v, rtol=1e-10, atol=np.full(ND, 1e-14))
    x, feed, _, T = nominal()
    x = x.copy()
    for n in ["X_su", "X_aa", "X_fa", "X_c4", "X_pro", "X_ac", "X_h2"]:
        x[IX[n]] = 0.0
    x[IX["X_xc"]], x[IX["X_ch"]], x[IX["X_li"]] = 5.0, 0.7, 0.3
    t = 2.0
    xe = _run(o, x, T, 0.0, feed, t)
    arr = o.tconst(T)["arr"]
    k1 = arr * v["k_dis"]
    X0 = 5.0
    assert abs(xe[IX["X_xc"]] - X0 * math.exp(-k1 * t)) < 1e-8 * X0
    for name, f, kname, c0 in [("X_ch", "f_ch_xc", "k_hyd_ch", 0.7),
                               ("X_li", "f_li_xc", "k_hyd_li", 0.3)]:
        k2 = arr * v[kname]
        ref = c0 * math.exp(-k2 * t) + v[f] * k1 * X0 * (math.exp(-k1 * t) - math.exp(-k2 * t)) \
            / (k2 - k1)
        assert abs(xe[IX[name]] - ref) < 1e-8 * max(ref, 1e-3), name
    ref = x[IX["S_I"]] + v["f_sI_xc"] * X0 * (1 - math.exp(-k1 * t))
    assert abs(xe[IX["S_I"]] - ref) < 1e-8 * ref


def test_closed_headspace_henry():
    """No reactions, D = 0, closed valve: methane relaxes between liquid and
    headspace as a two-compartment linear system."""
    v = values()
    for k in list(v):
        if k.startswith(("k_m_", "k_dec_", "k_hyd_")) or k in ("k_dis",):
            v[k] = 0.0
    v["k_p_per_V_liq"] = 0.0
    o = Oracle(v, rtol=1e-10, atol=np.full(ND, 1e-14))
    x, feed, _, T = nominal()
    x = x.copy()
    S0, G0 = 0.2, 0.05
    x[IX["S_ch4"]], x[IX["G_ch4"]] = S0, G0
    t = 0.05
    xe = _run(o, x, T, 0.0, feed, t)
    c = o.tconst(T)
    a, b, vg = v["k_L_a"], c["K_H_ch4"] * c["RT"], v["V_gas_per_V_liq"]
    M = S0 + vg * G0
    u = (S0 - b * G0) * math.exp(-a * (1 + b / vg) * t)
    G = (M - u) / (vg + b)
    S = M - vg * G
    assert abs(xe[IX["S_ch4"]] - S) < 1e-8 * S
    assert abs(xe[IX["G_ch4"]] - G) < 1e-8 * G


def _rk4_richardson(o, x, T, D, feed, dt):
    prev = None
    n = 16
    while True:
        y1 = o.fixed(x, T, D, feed, dt, n, "rk4")
        y2 = o.fixed(x, T, D, feed, dt, 2 * n, "rk4")
        ext = y2 + (y2 - y1) / 15.0
        nom = nominal()[0]
        if prev is not None and np.max(np.abs(ext - prev) / np.maximum(np.abs(ext), 1e-4 * nom)) < 1e-11:
            return ext
        prev = ext
        n *= 2
        assert n < 1 << 16


@pytest.mark.parametrize("seed", [1, 4])
def test_small_step_reference(seed):
    """Adaptive Rodas4 at rtol 1e-10 against classical RK4 with halved steps
    and Richardson extrapolation over one coupling interval."""
    x, feed, D, T = perturbed_smooth(seed)
    nom = nominal()[0]
    o = closed_valve(1e-10, 1e-4 * 1e-10 * nom[DIFF])
    ref = _rk4_richardson(o, x, T, D, feed, DT)
    xe = _run(o, x, T, D, feed, DT)
    err = np.abs(xe - ref) / np.maximum(np.abs(ref), 1e-4 * nom)
    assert err.max() < 1e-8
    # and the production tolerance meets the parity bound against the truth
    o8 = closed_valve(1e-8, 1e-4 * 1e-8 * nom[DIFF])
    xe8 = _run(o8, x, T, D, feed, DT)
    err8 = np.abs(xe8 - ref) / np.maximum(np.abs(ref), 1e-4 * nom)
    assert err8.max() < 1e-6


def test_rodas4_convergence_order():
    x, feed, D, T = perturbed_smooth(6)
    o = closed_valve(1e-8)
    ref = _rk4_richardson(o, x, T, D, feed, DT)
    errs = []
    for n in [4, 8, 16]:
        y = o.fixed(x, T, D, feed, DT, n, "rodas4")
        errs.append(np.max(np.abs(y[DIFF] - ref[DIFF]) / np.maximum(np.abs(ref[DIFF]), 1e-3)))
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert all(3.3 < p < 5.0 for p in orders), (errs, orders)


def test_nominal_is_steady_state(orc):
    x, feed, D, T = nominal()
    f, xa, H = orc.rhs(x, T, D, feed)
    flux = D * (np.abs(feed[[i for i in DIFF if i < NLIQ]]).sum() + 1.0)
    assert np.max(np.abs(f)) <= 1e-10 * flux
    assert 7.0 <= -math.log10(H) <= 7.6
    nom = x
    o = Oracle(PARAMS, rtol=1e-8, atol=1e-4 * 1e-8 * nom[DIFF])
    xe = _run(o, x, T, D, feed, 1.0)
    assert np.max(np.abs(xe - x) / np.abs(x)) < 1e-8


def test_failed_particle_keeps_input():
    o = Oracle(PARAMS, rtol=1e-8)
    x, feed, D, T = perturbed(1)
    X = np.stack([x, x], axis=1).copy()
    X[3, 1] = np.nan
    st, _ = o.step(X, [T, T], [D, D], [0, 0], feed[None, :], DT, nthreads=1)
    assert st[1] == 4 and st[0] & 0x7F == 0
    assert np.isnan(X[3, 1]) and np.array_equal(X[[0, 1, 2], 1], x[[0, 1, 2]])


# ---------------------------------------------------------------------------
# Fixed-step explicit scheme of the paper (sec. 2.3, sec. 4.3)
# ---------------------------------------------------------------------------
SEC = 1.0 / 86400.0  # one second in days


def test_euler_washout_recursion():
    """No kinetics, no gas exchange: explicit Euler on x' = D (x_in - x) is
    the recursion x_n = x_in + (1 - D h)^n (x_0 - x_in) in every liquid
    entry (S_h2 is algebraic)."""
    v = values()
    for k in list(v):
        if k.startswith(("k_m_", "k_dec_", "k_hyd_")) or k in ("k_dis",):
            v[k] = 0.0
    v.update(k_L_a=0.0, k_p_per_V_liq=0.0)
    o = Oracle(v, rtol=1e-8)
    x, feed, _, T = perturbed(3)
    D, dt, n = 40.0, 0.01, 7
    xe = o.fixed(x, T, D, feed, dt, n, "euler")
    h = dt / n
    liq = [i for i in range(NLIQ) if i != IX["S_h2"]]
    ref = feed[liq] + (1.0 - D * h) ** n * (x[liq] - feed[liq])
    assert np.max(np.abs(xe[liq] - ref) / np.abs(ref)) < 1e-13
    assert np.array_equal(xe[32:35], x[32:35])


def test_euler_first_order():
    """Global error of explicit Euler against the RK4 reference halves with
    the step (order 1), over a quarter of a coupling interval."""
    x, feed, D, T = perturbed_smooth(5)
    o = closed_valve(1e-8)
    dt = DT / 4
    ref = _rk4_richardson(o, x, T, D, feed, dt)
    errs = []
    for n in [256, 512, 1024]:
        y = o.fixed(x, T, D, feed, dt, n, "euler")
        errs.append(np.max(np.abs(y[DIFF] - ref[DIFF]) / np.maximum(np.abs(ref[DIFF]), 1e-3)))
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert all(0.85 < p < 1.15 for p in orders), (errs, orders)


@pytest.mark.parametrize("seed", [2, 9])
def test_euler_paper_interval_against_adaptive(seed):
    """The paper's coupling interval Dt = 0.5 s in ten explicit steps of
    0.05 s against the adaptive Rodas4 solution at rtol 1e-10: the
    difference is the explicit scheme's own truncation error (largest in the
    headspace CO2, which relaxes at ~1,600 1/d from a perturbed state), a
    few 1e-6, and it falls tenfold with ten times the steps."""
    x, feed, D, T = perturbed(seed)
    nom = nominal()[0]
    o = Oracle(PARAMS, rtol=1e-10, atol=1e-4 * 1e-10 * nom[DIFF])
    Dt = 0.5 * SEC
    ya = _run(o, x, T, D, feed, Dt)
    err = []
    for n in (10, 100):
        ye = o.fixed(x, T, D, feed, Dt, n, "euler")
        err.append((np.abs(ye - ya) / np.maximum(np.abs(ya), 1e-4 * nom)).max())
    assert err[0] < 2e-5
    assert 8.0 < err[0] / err[1] < 12.0, err



def test_tolerance_proportionality():
    """The adaptive integration's error against its own rtol-1e-12 solution
    falls with the tolerance: near rtol at 1e-8 and about 100 times that at
    1e-6, over two coupling intervals from perturbed states (an error
    controller that did not steer would not show it)."""
    nom = nominal()[0]
    e = {}
    for seed in range(1, 9):
        x, feed, D, T = perturbed(seed)
        res = {}
        for rt in (1e-6, 1e-8, 1e-12):
            res[rt] = _run(Oracle(PARAMS, rtol=rt, atol=1e-4 * rt * nom[DIFF]), x, T, D, feed,
                           DT, steps=2)
        den = np.maximum(np.abs(res[1e-12]), 1e-4 * nom)
        for rt in (1e-6, 1e-8):
            e[rt] = max(e.get(rt, 0.0), float(np.max(np.abs(res[rt] - res[1e-12]) / den)))
    assert e[1e-8] < 1e-7
    assert 20.0 < e[1e-6] / e[1e-8] < 500.0
