"""Oracle of the coupling driver: particle displacement and feed mask.

TEST INFRASTRUCTURE ONLY.  Plain numpy, float64, written from the field's
definition: the tank of radius R and height H carries solid-body rotation
omega plus axisymmetric Stokes stream-function modes
    psi(r, z) = sum_k a_k r^2 (R^2 - r^2) sin(k pi z / H),
    u_r = -(1/r) dpsi/dz,  u_z = (1/r) dpsi/dr,  u_theta = omega r.
The meridional part (u_r, u_z) is axisymmetric, so it commutes with the
rotation: the flow over a substep h is the meridional flow (classical RK4)
followed by the exact turn of the (x, y) plane by omega h.  (RK4 on the whole
field damps the rotation by |R(i omega h)| < 1 per step, about 2 % at 12 rpm
and h = 1 s, so particles would spiral onto the axis within one interval.)
A particle that crosses the wall, the bottom or the lid by rounding is
reflected back inside (the boundary is an invariant set of the flow, so a
particle placed on it would stay there); the feed mask marks particles in the
inlet region z >= z_min, r <= r_max (sec. 2.3: the AD particles follow the
fluid particles).
"""
from __future__ import annotations

import numpy as np


def velocity(x, y, z, omega, R, H, a):
    r2 = x * x + y * y
    radial = np.zeros_like(x)
    axial = np.zeros_like(x)
    for k, ak in enumerate(a, start=1):
        kk = k * np.pi / H
        # u_r / r = -(1/r^2) dpsi/dz = -a_k (R^2 - r^2) kk cos(kk z)
        radial -= ak * (R * R - r2) * kk * np.cos(kk * z)
        # u_z = (1/r) dpsi/dr = a_k (2 R^2 - 4 r^2) sin(kk z)
        axial += ak * (2 * R * R - 4 * r2) * np.sin(kk * z)
    ux = radial * x - omega * y
    uy = radial * y + omega * x
    return ux, uy, axial


def divergence(x, y, z, omega, R, H, a, eps=1e-6):
    """Central-difference divergence of the field (pin: zero)."""
    d = 0.0
    for comp, (dx, dy, dz) in enumerate([(eps, 0, 0), (0, eps, 0), (0, 0, eps)]):
        up = velocity(x + dx, y + dy, z + dz, omega, R, H, a)[comp]
        um = velocity(x - dx, y - dy, z - dz, omega, R, H, a)[comp]
        d = d + (up - um) / (2 * eps)
    return d


def advect(pos, omega, R, H, a, dt_seconds, substeps):
    x, y, z = (np.array(pos[i], dtype=np.float64) for i in range(3))
    h = dt_seconds / substeps
    c, s_ = np.cos(omega * h), np.sin(omega * h)
    for _ in range(substeps):
        # meridional flow (omega = 0), classical RK4
        k1 = velocity(x, y, z, 0.0, R, H, a)
        k2 = velocity(x + 0.5 * h * k1[0], y + 0.5 * h * k1[1], z + 0.5 * h * k1[2],
                      0.0, R, H, a)
        k3 = velocity(x + 0.5 * h * k2[0], y + 0.5 * h * k2[1], z + 0.5 * h * k2[2],
                      0.0, R, H, a)
        k4 = velocity(x + h * k3[0], y + h * k3[1], z + h * k3[2], 0.0, R, H, a)
        x = x + h / 6 * (k1[0] + 2 * k2[0] + 2 * k3[0] + k4[0])
        y = y + h / 6 * (k1[1] + 2 * k2[1] + 2 * k3[1] + k4[1])
        z = z + h / 6 * (k1[2] + 2 * k2[2] + 2 * k3[2] + k4[2])
        # solid-body rotation, exact
        x, y = c * x - s_ * y, s_ * x + c * y
        r = np.sqrt(x * x + y * y)
        s = np.where(r > R, np.maximum(2.0 * R - r, 0.0) / np.maximum(r, 1e-300), 1.0)
        x, y = x * s, y * s
        z = np.where(z < 0.0, -z, z)
        z = np.where(z > H, 2.0 * H - z, z)
        z = np.clip(z, 0.0, H)
    return np.stack([x, y, z])


def feed_mask(pos, z_min, r_max):
    x, y, z = pos[0], pos[1], pos[2]
    return (z >= z_min) & (x * x + y * y <= r_max * r_max)
