"""Plain FP64 oracle of diffusion between the AD particles.

TEST INFRASTRUCTURE ONLY: the test suite and the benchmark's CPU-baseline
leg use it; the HIP product path never does.

The paper names diffusion between particles as missing (sec. 2.3: only
advective transport is modelled so far) and as its first next step (sec. 5)
without giving an operator.  The reading taken here is the standard SPH
diffusion operator: with every particle carrying the same volume V_p (sec.
2.3: tank volume over particle count),

    dC_i/dt = D * 2 * sum_{j != i, r_ij < 2h} V_p (C_i - C_j) W'(r_ij) / r_ij,

the Brookshaw / Cleary-Monaghan form of the Laplacian, with the 3-D
Wendland C2 kernel of support radius 2h,

    W(r) = a (1 - q/2)^4 (2q + 1),  q = r/h,  a = 21 / (16 pi h^3),
    W'(r) / r = -5 a / h^2 (1 - q/2)^3.

It acts on the soluble entries of the state (DIFFUSING rows); particulates,
the algebraic entries and the headspace do not diffuse.  Pairs are found by
brute force over all particles, in index order.  Explicit Euler advances
the state over dt in equal substeps.
"""
from __future__ import annotations

import math

import numpy as np

# soluble differential entries: S_su .. S_ac, S_ch4, S_IC, S_IN, S_I, S_cat, S_an
DIFFUSING = [0, 1, 2, 3, 4, 5, 6, 8, 9, 10, 11, 24, 25]


def kernel_w(r, h):
    """Wendland C2 kernel in 3-D, support radius 2h (1/m^3)."""
    q = np.asarray(r, dtype=np.float64) / h
    a = 21.0 / (16.0 * math.pi * h ** 3)
    return np.where(q < 2.0, a * (1.0 - q / 2.0) ** 4 * (2.0 * q + 1.0), 0.0)


def kernel_f(r, h):
    """W'(r) / r of the same kernel (1/m^5)."""
    q = np.asarray(r, dtype=np.float64) / h
    a = 21.0 / (16.0 * math.pi * h ** 3)
    return np.where(q < 2.0, -5.0 * a / h ** 2 * (1.0 - q / 2.0) ** 3, 0.0)


def _pairs(pos, i0, i1, h):
    """Distances from particles i0..i1-1 to all particles and the mask of
    neighbours (r < 2h, j != i)."""
    d = pos[:, None, :] - pos[:, i0:i1, None]          # [3][rows][n]
    r = np.sqrt((d * d).sum(axis=0))
    mask = r < 2.0 * h
    rows = np.arange(i0, i1)
    mask[rows - i0, rows] = False
    return r, mask


def diffusion_rate(pos, C, h, V_p, D, chunk=256):
    """dC/dt of every particle.  pos: [3][n] (m, taken as float64), C: [k][n].
    Returns (rate [k][n], absolute-term sum [k][n]); the second is
    2 D V_p sum_j |C_i - C_j| |W'/r|, a scale for rounding comparisons."""
    pos = np.asarray(pos, dtype=np.float64)
    C = np.asarray(C, dtype=np.float64)
    n = pos.shape[1]
    rate = np.zeros_like(C)
    absum = np.zeros_like(C)
    for i0 in range(0, n, chunk):
        i1 = min(n, i0 + chunk)
        r, mask = _pairs(pos, i0, i1, h)
        F = np.where(mask, kernel_f(r, h), 0.0)           # [rows][n]
        diff = C[:, i0:i1, None] - C[:, None, :]          # [k][rows][n]
        rate[:, i0:i1] = 2.0 * D * V_p * (diff * F[None]).sum(axis=2)
        absum[:, i0:i1] = 2.0 * D * V_p * (np.abs(diff) * np.abs(F)[None]).sum(axis=2)
    return rate, absum


def diffusion_rate_at(pos, C, idx, h, V_p, D):
    """dC/dt of the particles idx only, each against all particles (for
    sampled checks of large populations).  Returns (rate [k][len(idx)],
    neighbour counts [len(idx)])."""
    pos = np.asarray(pos, dtype=np.float64)
    C = np.asarray(C, dtype=np.float64)
    out = np.zeros((C.shape[0], len(idx)))
    cnt = np.zeros(len(idx), dtype=np.int64)
    for m, i in enumerate(idx):
        d = pos - pos[:, i:i + 1]
        r = np.sqrt((d * d).sum(axis=0))
        mask = r < 2.0 * h
        mask[i] = False
        j = np.nonzero(mask)[0]
        F = kernel_f(r[j], h)
        out[:, m] = 2.0 * D * V_p * ((C[:, i:i + 1] - C[:, j]) * F[None]).sum(axis=1)
        cnt[m] = len(j)
    return out, cnt


def neighbour_counts(pos, h, chunk=256):
    """Number of particles j != i within r < 2h of each particle i."""
    pos = np.asarray(pos, dtype=np.float64)
    n = pos.shape[1]
    out = np.zeros(n, dtype=np.int64)
    for i0 in range(0, n, chunk):
        i1 = min(n, i0 + chunk)
        _, mask = _pairs(pos, i0, i1, h)
        out[i0:i1] = mask.sum(axis=1)
    return out


def diffuse(state, pos, n, h, V_p, D, dt, substeps):
    """Explicit Euler over dt (days) in `substeps` equal steps on the
    DIFFUSING rows of state [35][ld] (columns 0..n-1); returns a new array."""
    X = np.array(state, dtype=np.float64)
    ht = dt / substeps
    for _ in range(substeps):
        rate, _ = diffusion_rate(pos[:, :n], X[DIFFUSING, :n], h, V_p, D)
        X[DIFFUSING, :n] += ht * rate
    return X
