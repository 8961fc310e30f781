"""One Langevin (BAOAB) or NVE (velocity Verlet) step in FP64.

TEST INFRASTRUCTURE ONLY.  The paper runs "canonical Langevin dynamics"
(Sec. 3.2) without naming a scheme; the reading used here is the BAOAB
splitting of Leimkuhler & Matthews (2013):

  B: v += (dt/2) F(x)/m
  A: x += (dt/2) v
  O: v  = c1 v + sqrt((1 - c1^2) kT/m) xi,   c1 = exp(-gamma dt)
  A: x += (dt/2) v
     wrap x into [-L/2, L/2) and count the image crossings
  B: v += (dt/2) F(x_new)/m

gamma = 0 gives velocity Verlet (NVE).  xi are the Philox/Box-Muller normals
of ``philox_ref`` keyed by (seed, tag, step).  dim = 2 (the paper's 2d boxes,
Sec. 3.2) keeps motion in the xy plane: the z component of xi is dropped, so
particles that share one z and have vz = 0 keep them.

Parity status: pinned by equipartition, NVE energy conservation and time
reversibility tests.
"""
from __future__ import annotations

import math

import numpy as np

from . import philox_ref, swap_ref


def wrap(x, L):
    """Fold into [-L/2, L/2); returns (x, image increments)."""
    Lv = np.broadcast_to(np.asarray(L, dtype=np.float64), (3,))
    img = np.zeros(x.shape, dtype=np.int64)
    hi = x >= 0.5 * Lv
    x = np.where(hi, x - Lv, x)
    img += hi
    lo = x < -0.5 * Lv
    x = np.where(lo, x + Lv, x)
    img -= lo
    return x, img


def baoab_step(pos, vel, types, tags, L, table, mass_by_type, dt, kT, gamma, seed, step,
               force=None, extra=None, dim=3, force_fn=None):
    """Advance (pos, vel) by one step; returns dict(pos, vel, image, F, F_old).

    extra(x) -> [N,3], if given, adds a further force (e.g. bond springs; x in
    the same order as pos).  force_fn(x) -> [N,3], if given, evaluates the
    potential's forces instead of ``swap_ref`` (e.g. the C brute force)."""
    x = np.asarray(pos, dtype=np.float64).copy()
    v = np.asarray(vel, dtype=np.float64).copy()
    m = np.asarray(mass_by_type, dtype=np.float64)[np.asarray(types)][:, None]

    def forces(y):
        f = force_fn(y) if force_fn is not None else swap_ref.evaluate(y, types, L, table, scales=False)["F"]
        return f if extra is None else f + extra(y)

    F = forces(x) if force is None else force
    v = v + 0.5 * dt * F / m
    x = x + 0.5 * dt * v
    if gamma > 0.0:
        c1 = math.exp(-gamma * dt)
        c2 = np.sqrt((1.0 - c1 * c1) * kT / m)
        xi = philox_ref.thermostat_normals(seed, tags, step)
        if dim == 2:
            xi = np.asarray(xi, dtype=np.float64).copy()
            xi[:, 2] = 0.0
        v = c1 * v + c2 * xi
    x = x + 0.5 * dt * v
    x, img = wrap(x, L)
    Fn = forces(x)
    v = v + 0.5 * dt * Fn / m
    return dict(pos=x, vel=v, image=img, F=Fn, F_old=F)


def kinetic_tensor(vel, types, mass_by_type):
    """sum_m m v_a v_b, ordered (xx, yy, zz, xy, xz, yz)."""
    v = np.asarray(vel, dtype=np.float64)
    m = np.asarray(mass_by_type, dtype=np.float64)[np.asarray(types)]
    K = np.einsum("p,pa,pb->ab", m, v, v)
    return np.array([K[0, 0], K[1, 1], K[2, 2], K[0, 1], K[0, 2], K[1, 2]])
