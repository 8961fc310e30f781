"""Rigid planar bodies (the patchy colloids of Sec. 3.2) in FP64.

TEST INFRASTRUCTURE ONLY.  A body is a disk (its centre particle, of its
type's mass M) carrying massless member particles at fixed body-frame offsets
d0, turned by the body's angle theta: member position x_c + R(theta) d0.  The
paper simulates such bodies in 2d without naming a scheme; the reading used
here applies the BAOAB splitting of ``dynamics_ref`` to the body's planar
coordinates (x, y) with its mass and to theta with its moment of inertia I,
the force F being the sum over the centre and its members and the torque
tau = sum_m (d_m x f_m)_z about the centre (minimum image):

  B: v += dt/2 F/M,   w += dt/2 tau/I
  A: x += dt/2 v,     theta += dt/2 w
  O: v = c1 v + sqrt((1-c1^2) kT/M) (xi_x, xi_y),  w = c1 w + sqrt((1-c1^2) kT/I) xi_z
  A: x += dt/2 v,     theta += dt/2 w;   fold x into the box, theta into [-pi, pi)
     place the members;  forces at the new positions
  B: v += dt/2 F/M,   w += dt/2 tau/I

xi are the thermostat normals of the centre's tag (``philox_ref``).  Arrays are
indexed by tag.

Pins: a free body moves and turns uniformly; energy (translational, rotational
and potential) and the total angular momentum of colliding bodies are kept by
the gamma = 0 step (tests/test_oracle_pins.py); the Langevin branch brings a
free-body gas to equipartition, M <v_x^2> = M <v_y^2> = I <w^2> = kT
(tests/test_oracle_scales.py).
"""
from __future__ import annotations

import math

import numpy as np

from . import dynamics_ref, philox_ref, swap_ref


def _members(bodies):
    first = np.asarray(bodies["first"], dtype=np.int64)
    owner = np.repeat(np.arange(len(first) - 1), np.diff(first))
    return owner, np.asarray(bodies["member"], dtype=np.int64), np.asarray(bodies["offset"], dtype=np.float64)


def force_torque(pos, force, bodies, L):
    """(F [B,2], tau [B]) of every body."""
    Lv = np.broadcast_to(np.asarray(L, dtype=np.float64), (3,))
    c = np.asarray(bodies["centre"], dtype=np.int64)
    owner, mem, _ = _members(bodies)
    F = np.asarray(force, dtype=np.float64)[c, :2].copy()
    fm = np.asarray(force, dtype=np.float64)[mem, :2]
    np.add.at(F, owner, fm)
    d = swap_ref.min_image(np.asarray(pos, np.float64)[c[owner]], np.asarray(pos, np.float64)[mem], Lv)
    tau = np.zeros(len(c))
    np.add.at(tau, owner, d[:, 0] * fm[:, 1] - d[:, 1] * fm[:, 0])
    return F, tau


def place(pos, bodies, theta, L):
    """Member positions at the bodies' poses (folded into the box)."""
    x = np.asarray(pos, dtype=np.float64).copy()
    c = np.asarray(bodies["centre"], dtype=np.int64)
    owner, mem, off = _members(bodies)
    th = np.asarray(theta, dtype=np.float64)[owner]
    d = np.stack([np.cos(th) * off[:, 0] - np.sin(th) * off[:, 1],
                  np.sin(th) * off[:, 0] + np.cos(th) * off[:, 1]], axis=1)
    x[mem, :2] = x[c[owner], :2] + d
    x[mem], _ = dynamics_ref.wrap(x[mem], L)
    return x


def half_step(pos, vel, force, theta, omega, types, bodies, L, mass_by_type, dt, kT, gamma, seed, step, first):
    """One half of the body step (first: B A O A and the placement; else the last B)."""
    x = np.asarray(pos, dtype=np.float64).copy()
    v = np.asarray(vel, dtype=np.float64).copy()
    th = np.asarray(theta, dtype=np.float64).copy()
    w = np.asarray(omega, dtype=np.float64).copy()
    c = np.asarray(bodies["centre"], dtype=np.int64)
    M = np.asarray(mass_by_type, dtype=np.float64)[np.asarray(types)[c]]
    I = np.asarray(bodies["inertia"], dtype=np.float64)
    F, tau = force_torque(x, force, bodies, L)
    vc = v[c, :2] + 0.5 * dt * F / M[:, None]
    w = w + 0.5 * dt * tau / I
    if first:
        xc = x[c, :2] + 0.5 * dt * vc
        th = th + 0.5 * dt * w
        if gamma > 0.0:
            c1 = math.exp(-gamma * dt)
            xi = np.asarray(philox_ref.thermostat_normals(seed, c, step), dtype=np.float64)
            vc = c1 * vc + np.sqrt((1.0 - c1 * c1) * kT / M)[:, None] * xi[:, :2]
            w = c1 * w + np.sqrt((1.0 - c1 * c1) * kT / I) * xi[:, 2]
        xc = xc + 0.5 * dt * vc
        th = th + 0.5 * dt * w
        th = np.where(th >= math.pi, th - 2.0 * math.pi, np.where(th < -math.pi, th + 2.0 * math.pi, th))
        full = x[c].copy()
        full[:, :2] = xc
        x[c], _ = dynamics_ref.wrap(full, L)
        x = place(x, bodies, th, L)
    v[c, :2] = vc
    v[c, 2] = 0.0
    owner, mem, off = _members(bodies)
    tho = th[owner]
    d = np.stack([np.cos(tho) * off[:, 0] - np.sin(tho) * off[:, 1],
                  np.sin(tho) * off[:, 0] + np.cos(tho) * off[:, 1]], axis=1)
    v[mem, 0] = vc[owner, 0] - w[owner] * d[:, 1]
    v[mem, 1] = vc[owner, 1] + w[owner] * d[:, 0]
    v[mem, 2] = 0.0
    return x, v, th, w


def step(pos, vel, theta, omega, types, bodies, L, table, mass_by_type, dt, kT, gamma, seed, step_no,
         force=None):
    """One full body step; returns dict(pos, vel, theta, omega, F)."""
    f0 = swap_ref.evaluate(pos, types, L, table, scales=False)["F"] if force is None else force
    x, v, th, w = half_step(pos, vel, f0, theta, omega, types, bodies, L, mass_by_type, dt, kT, gamma, seed,
                            step_no, True)
    f1 = swap_ref.evaluate(x, types, L, table, scales=False)["F"]
    x, v, th, w = half_step(x, v, f1, th, w, types, bodies, L, mass_by_type, dt, kT, gamma, seed, step_no, False)
    return dict(pos=x, vel=v, theta=th, omega=w, F=f1)


def kinetic(vel, omega, types, bodies, mass_by_type):
    """(translational, rotational) kinetic energy of the bodies."""
    c = np.asarray(bodies["centre"], dtype=np.int64)
    M = np.asarray(mass_by_type, dtype=np.float64)[np.asarray(types)[c]]
    v = np.asarray(vel, dtype=np.float64)[c, :2]
    return 0.5 * float(np.sum(M * np.sum(v * v, axis=1))), \
        0.5 * float(np.sum(np.asarray(bodies["inertia"]) * np.asarray(omega, dtype=np.float64) ** 2))


def angular_momentum(pos, vel, omega, types, bodies, mass_by_type):
    """Total angular momentum about the origin (unwrapped positions assumed)."""
    c = np.asarray(bodies["centre"], dtype=np.int64)
    M = np.asarray(mass_by_type, dtype=np.float64)[np.asarray(types)[c]]
    x = np.asarray(pos, dtype=np.float64)[c]
    v = np.asarray(vel, dtype=np.float64)[c]
    return float(np.sum(M * (x[:, 0] * v[:, 1] - x[:, 1] * v[:, 0]))
                 + np.sum(np.asarray(bodies["inertia"]) * np.asarray(omega, dtype=np.float64)))
