"""Pins of the particle-diffusion oracle against the mathematics of the SPH
diffusion operator it follows (normalised kernel, its derivative, exact
Laplacian of quadratic fields on a lattice, conservation, the steady
uniform field) and a closed form of the explicit update."""
from __future__ import annotations

import math

import numpy as np
import pytest

from oracle import diffusion as OD


def test_kernel_is_normalised():
    h = 0.37
    r = np.linspace(0.0, 2.0 * h, 400_001)
    assert abs(np.trapezoid(4.0 * math.pi * r ** 2 * OD.kernel_w(r, h), r) - 1.0) < 1e-10


@pytest.mark.parametrize("q", [0.1, 0.7, 1.3, 1.9])
def test_gradient_over_r_is_the_kernel_derivative(q):
    h = 0.5
    r, e = q * h, 1e-7
    fd = (OD.kernel_w(r + e, h) - OD.kernel_w(r - e, h)) / (2 * e)
    assert abs(float(OD.kernel_f(r, h)) * r - float(fd)) < 1e-7 * abs(float(fd))
    assert OD.kernel_f(2.0 * h, h) == 0.0 and OD.kernel_w(2.0 * h, h) == 0.0


def lattice(m, d):
    g = np.arange(-m, m + 1) * d
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    return np.stack([X.ravel(), Y.ravel(), Z.ravel()])


@pytest.mark.parametrize("ratio", [1.5, 2.0])
def test_laplacian_of_quadratic_on_a_lattice(ratio):
    """C = x^2 + 2y^2 + 3z^2 has Laplacian 12; the operator at an interior
    lattice particle (volume d^3, h = ratio d) reproduces it to 0.1 %."""
    d = 0.01
    P = lattice(6, d)
    C = P[0] ** 2 + 2 * P[1] ** 2 + 3 * P[2] ** 2
    centre = int(np.argmin((P ** 2).sum(axis=0)))
    rate, _ = OD.diffusion_rate(P, C[None], ratio * d, d ** 3, 1.0)
    assert abs(rate[0, centre] - 12.0) < 0.012


def test_conservation_and_uniform_field():
    g = np.random.default_rng(4)
    P = g.random((3, 700)) * 0.05
    C = g.random((3, 700))
    rate, absum = OD.diffusion_rate(P, C, 0.004, 1e-7, 2.0)
    assert np.all(np.abs(rate.sum(axis=1)) < 1e-12 * absum.sum(axis=1))
    assert (absum > 0).any()
    flat, _ = OD.diffusion_rate(P, np.full((2, 700), 3.5), 0.004, 1e-7, 2.0)
    assert np.all(flat == 0.0)


def test_two_particles_closed_form():
    """Two particles at distance r: C_1 - C_2 decays by the factor
    (1 - 4 D V_p |W'/r| dt/m)^m over m explicit steps; their mean is kept."""
    h, Vp, D, r = 0.01, 2e-6, 3.0, 0.012
    pos = np.array([[0.0, r], [0.0, 0.0], [0.0, 0.0]])
    state = np.zeros((35, 2))
    state[OD.DIFFUSING, 0] = 2.0
    state[OD.DIFFUSING, 1] = 0.5
    dt, m = 1e-4, 7
    out = OD.diffuse(state, pos, 2, h, Vp, D, dt, m)
    k = 4.0 * D * Vp * abs(float(OD.kernel_f(r, h)))
    assert 0.1 < k * dt / m < 1.0      # a stable step that still moves the gap
    gap = 1.5 * (1.0 - k * dt / m) ** m
    for row in OD.DIFFUSING:
        assert abs((out[row, 0] - out[row, 1]) - gap) < 1e-14 * 1.5
        assert abs(out[row, 0] + out[row, 1] - 2.5) < 1e-14
    rest = [i for i in range(35) if i not in OD.DIFFUSING]
    assert np.array_equal(out[rest], state[rest])


def test_neighbour_counts_on_a_lattice():
    """Lattice spacing d, h = 0.75 d: the support 1.5 d holds the 6 face, 12
    edge neighbours (sqrt(2) d) and no corner ones (sqrt(3) d)."""
    d = 1.0
    P = lattice(3, d)
    cnt = OD.neighbour_counts(P, 0.75 * d)
    centre = int(np.argmin((P ** 2).sum(axis=0)))
    assert cnt[centre] == 18


def test_stability_bound_of_the_explicit_step():
    """The documented bound: sum_j V_p |W'/r| integrates to 3.5 / h^2, so on
    evenly spread particles the operator's rates stay below 14 D / h^2 and
    explicit Euler is stable for dt <= h^2 / (7 D).  On a lattice, a
    checkerboard perturbation (the fastest mode) decays with substeps of
    0.1 h^2 / D and grows with substeps of h^2 / D."""
    h = 0.5
    r = np.linspace(0.0, 2.0 * h, 200_001)
    integral = np.trapezoid(4.0 * math.pi * r ** 2 * -OD.kernel_f(r, h), r)
    assert abs(integral * h * h - 3.5) < 1e-8
    d = 1.0
    P = lattice(5, d)
    hl, D, Vp = 1.5 * d, 1.0, d ** 3
    chk = np.where((np.round(P / d).sum(axis=0) % 2) == 0, 1.0, -1.0)
    inner = np.all(np.abs(P) <= 2 * d, axis=0)
    state = np.zeros((35, P.shape[1]))
    state[OD.DIFFUSING[0]] = 1.0 + 0.01 * chk
    amp0 = np.abs(state[OD.DIFFUSING[0], inner] - 1.0).max()
    ok = OD.diffuse(state, P, P.shape[1], hl, Vp, D, 0.1 * hl * hl / D, 1)
    bad = OD.diffuse(state, P, P.shape[1], hl, Vp, D, 1.0 * hl * hl / D, 1)
    assert np.abs(ok[OD.DIFFUSING[0], inner] - 1.0).max() < amp0
    assert np.abs(bad[OD.DIFFUSING[0], inner] - 1.0).max() > amp0
    # randomly placed particles: interior row sums average the even-spread
    # 3.5 / h^2 but reach about twice it, hence the 0.05 h^2 / D substep
    g = np.random.default_rng(1)
    n, L = 4000, np.array([0.04, 0.03, 0.02])
    Q = g.random((3, n)) * L[:, None]
    Vq = np.prod(L) / n
    hq = 1.3 * Vq ** (1 / 3)
    rows = np.zeros(n)
    for i0 in range(0, n, 500):
        rr, mask = OD._pairs(Q, i0, min(n, i0 + 500), hq)
        rows[i0:i0 + 500] = np.where(mask, -OD.kernel_f(rr, hq), 0.0).sum(axis=1)
    rows *= Vq * hq * hq
    interior = np.all((Q > 2 * hq) & (Q < L[:, None] - 2 * hq), axis=0)
    assert abs(rows[interior].mean() / 3.5 - 1.0) < 0.05
    assert 1.4 < rows[interior].max() / 3.5 < 2.2
