"""Seeded synthetic workloads for the per-particle ADM1 step.

This module only draws inputs: initial states, feeds, temperatures, particle
positions and flow-field coefficients.  It holds none of the model's
arithmetic, so both the HIP path and the oracle can be fed from it.

Recipe (shapes follow the paper's two cases, sec. 3):
  * nominal state / feed: the Case-1 CSTR steady state (Table 1 reactor,
    35 C) under a fixed synthetic feed, stored in data/nominal.json;
  * initial states: the 28 differential entries are the nominal values times
    exp(0.2 z), z ~ N(0, 1) (median preserving); the 7 algebraic entries are
    left at their nominal values, since the step recomputes them;
  * RNG: numpy Generator(PCG64) seeded per workload; large populations are
    drawn in fixed chunks of 2^18 particles from SeedSequence(seed).spawn, so
    the values do not depend on how the caller slices the work.
"""
from __future__ import annotations

import json
import os
from dataclasses import dataclass, field

import numpy as np

DATA = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data")
NX, ND, NLIQ = 35, 28, 26
DIFF = np.array([0, 1, 2, 3, 4, 5, 6, 8, 9, 10, 11, 12, 13, 14, 15, 16, 17, 18, 19, 20,
                 21, 22, 23, 24, 25, 32, 33, 34])
# biodegradable inflow COD: S_su, S_aa, S_fa, S_va, S_bu, S_pro, S_ac, X_xc, X_ch,
# X_pr, X_li
BIODEGRADABLE = np.array([0, 1, 2, 3, 4, 5, 6, 12, 13, 14, 15])
CHUNK = 1 << 18
DT = 1.0 / 96.0


def nominal() -> dict:
    with open(os.path.join(DATA, "nominal.json")) as fh:
        d = json.load(fh)
    d["state"] = np.array(d["state"], dtype=np.float64)
    d["feed"] = np.array(d["feed"], dtype=np.float64)
    return d


def params_path() -> str:
    return os.path.join(DATA, "adm1_params.json")


def atol_vector(rtol: float) -> np.ndarray:
    """Absolute tolerances of the 28 differential entries: 1e-4 rtol x_nom."""
    return 1e-4 * rtol * nominal()["state"][DIFF]


def pad_ld(n: int, mult: int = 256) -> int:
    return max(mult, (n + mult - 1) // mult * mult)


def _chunks(n: int, seed: int):
    ss = np.random.SeedSequence(seed)
    nch = (n + CHUNK - 1) // CHUNK
    for c, child in enumerate(ss.spawn(nch)):
        yield c * CHUNK, min(n, (c + 1) * CHUNK), np.random.Generator(np.random.PCG64(child))


def perturbed_states(n: int, seed: int, sigma: float = 0.2, ld: int | None = None):
    """x[35][ld] float64: nominal x exp(sigma z) on the differential entries."""
    nom = nominal()["state"]
    ld = pad_ld(n) if ld is None else ld
    X = np.empty((NX, ld), dtype=np.float64)
    X[:] = nom[:, None]
    for a, b, g in _chunks(n, seed):
        z = g.standard_normal((ND, b - a))
        X[DIFF, a:b] = nom[DIFF, None] * np.exp(sigma * z)
    return X


@dataclass
class Workload:
    name: str
    n: int
    ld: int
    X: np.ndarray            # [35][ld] initial state
    T: np.ndarray            # [n] temperature, K
    D: np.ndarray            # [n] dilution rate of the current coupling step, 1/d
    fidx: np.ndarray         # [n] int32 feed row
    feed: np.ndarray         # [n_feed][26]
    dt: float = DT
    steps: int = 1
    rtol: float = 1e-8
    zone: np.ndarray | None = None  # bool [n] feed-zone membership
    extra: dict = field(default_factory=dict)

    def D_at(self, step: int) -> np.ndarray:
        """Dilution rates for coupling step `step` (pulsed zones)."""
        if self.zone is None:
            return self.D
        D = np.zeros(self.n)
        if step % 2 == 0:
            D[self.zone] = 1.0
        return D


def cstr_population(n: int = 256, seed: int = 1, steps: int = 96) -> Workload:
    """Plain CSTR-per-particle population: every particle is a full Case-1
    reactor (D = 178.45/3400 1/d, 35 C) with its own perturbed state and its
    own perturbed feed (sigma 0.2, own RNG stream)."""
    nom = nominal()
    X = perturbed_states(n, seed)
    g = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 7])))
    feed = nom["feed"][None, :] * np.exp(0.2 * g.standard_normal((n, NLIQ)))
    return Workload("cstr", n, X.shape[1], X, np.full(n, nom["T"]), np.full(n, nom["D"]),
                    np.arange(n, dtype=np.int32), np.ascontiguousarray(feed), steps=steps)


def pulse_feed() -> np.ndarray:
    """Feed-zone inflow: the nominal feed with biodegradable COD x10."""
    f = nominal()["feed"].copy()
    f[BIODEGRADABLE] *= 10.0
    return f


def batched_population(n: int = 1 << 20, seed: int = 2, steps: int = 10,
                       zone_frac: float = 0.05) -> Workload:
    """Batched population: T ~ U(303.15, 313.15) K, a Bernoulli(zone_frac)
    feed zone scattered in index that receives the pulse feed at D = 1 1/d
    on even coupling steps; all other particles are closed (D = 0)."""
    X = perturbed_states(n, seed)
    T = np.empty(n)
    zone = np.empty(n, dtype=bool)
    for a, b, g in _chunks(n, seed + 1000):
        T[a:b] = g.uniform(303.15, 313.15, b - a)
        zone[a:b] = g.random(b - a) < zone_frac
    feed = np.stack([nominal()["feed"], pulse_feed()])
    fidx = zone.astype(np.int32)
    w = Workload("batched", n, X.shape[1], X, T, np.zeros(n), fidx, feed, steps=steps,
                 zone=zone)
    w.D = w.D_at(0)
    return w


TANK_R, TANK_H = 0.1, 0.3          # m, lab-scale cylinder (sec. 3.2 scale)
MIXER_RPM = 12.0                    # paper Table 2
INLET_Z, INLET_R = 0.28, 0.03       # top inlet region, m
# Advection substep of the field (s).  RK4 shrinks a closed orbit of angular
# frequency w by about (w h)^6 / 72 per step; the fastest meridional cells
# turn at a few tenths per second, and 1 s steps let particles spiral into
# their cores over a few intervals (neighbour counts at the 99.99th
# percentile grew from 107 to 194 in five intervals); 0.25 s keeps the
# particle density even (108 after five intervals).
ADVECT_SUBSTEP_S = 0.25


def advect_substeps(dt_seconds: float) -> int:
    """Advection substeps for a coupling interval of dt_seconds."""
    return max(1, int(round(dt_seconds / ADVECT_SUBSTEP_S)))


FLOW_MODES = 4


def flow_field(seed: int = 3) -> dict:
    """Seeded smooth flow: solid-body rotation at the mixer speed plus four
    axisymmetric stream-function modes with N(0, 0.5^2) amplitudes."""
    g = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 11])))
    a = 0.5 * g.standard_normal(FLOW_MODES)
    return {"omega": MIXER_RPM * 2 * np.pi / 60.0, "R": TANK_R, "H": TANK_H,
            "a": [float(v) for v in a]}


def cylinder_positions(n: int, seed: int, ld: int | None = None) -> np.ndarray:
    """float32 [3][ld] positions uniform in the tank volume."""
    ld = pad_ld(n) if ld is None else ld
    P = np.zeros((3, ld), dtype=np.float32)
    for a_, b_, g in _chunks(n, seed + 2000):
        u = g.random((3, b_ - a_))
        r = TANK_R * np.sqrt(u[0])
        th = 2 * np.pi * u[1]
        P[0, a_:b_] = r * np.cos(th)
        P[1, a_:b_] = r * np.sin(th)
        P[2, a_:b_] = TANK_H * u[2]
    return P


def digester_field(n: int = 1 << 22, seed: int = 3, steps: int = 96,
                   T_K: float = 308.5) -> Workload:
    """Lab-digester field: particles uniform in the cylinder (r 0.1 m,
    h 0.3 m) advected by the seeded flow between coupling steps; particles
    in the top inlet (z >= 0.28 m, r <= 0.03 m) at the start of an interval
    receive the pulse feed at D = 1 1/d, the others are closed; T = 308.5 K
    (paper Table 2).  Liquid volume per particle = tank volume / n."""
    X = perturbed_states(n, seed)
    pos = cylinder_positions(n, seed, X.shape[1])
    feed = np.stack([nominal()["feed"], pulse_feed()])
    w = Workload("digester", n, X.shape[1], X, np.full(n, T_K), np.zeros(n),
                 np.zeros(n, dtype=np.int32), feed, steps=steps)
    w.extra = {"pos": pos, "flow": flow_field(seed),
               "V_p": np.pi * TANK_R ** 2 * TANK_H / n}
    return w


def subset(w: Workload, idx: np.ndarray) -> Workload:
    """The particles idx of w as their own workload (for oracle samples)."""
    idx = np.asarray(idx)
    m = len(idx)
    ld = pad_ld(m, 64)
    X = np.zeros((NX, ld))
    X[:, :m] = w.X[:, idx]
    X[:, m:] = w.X[:, idx[:1]]
    return Workload(w.name + "_subset", m, ld, X, w.T[idx].copy(), w.D[idx].copy(),
                    w.fidx[idx].copy(), w.feed, w.dt, w.steps, w.rtol,
                    None if w.zone is None else w.zone[idx].copy(), dict(w.extra))


# Particle phases (sec. 5, several particle kinds): an active liquid phase,
# a settled sediment phase with reduced biological activity and an inert
# phase with none.  The factors scale every biochemical rate of a particle.
PHASE_KIN = np.array([1.0, 0.25, 0.0])
PHASE_SHARES = (0.7, 0.2, 0.1)


def mixed_phases(n: int, seed: int, ld: int | None = None) -> np.ndarray:
    """uint8 phase ids [ld] (0 beyond n): each particle draws phase k with
    probability PHASE_SHARES[k]."""
    ld = n if ld is None else ld
    rng = np.random.default_rng(seed + 9001)
    ph = np.zeros(ld, dtype=np.uint8)
    ph[:n] = rng.choice(len(PHASE_SHARES), size=n, p=PHASE_SHARES).astype(np.uint8)
    return ph
