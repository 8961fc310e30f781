"""Rigid planar bodies on a System (the patchy colloids of Sec. 3.2).

A body is a disk (its centre particle) with massless member particles at fixed
body-frame offsets; both are particles of the System.  Each step launches the
stand-alone force kernel on every particle and the body kernel of
``rc_rigid_step`` for the two BAOAB halves; the list is rebuilt when a path
length passes the soft skin threshold.  Every step runs in the library's HIP
kernels; this module only holds the body arrays and sequences the calls.
"""
from __future__ import annotations

import math
import time

import numpy as np
import torch

from . import _lib as rcl
from . import api


class RigidBodies:
    def __init__(self, system, bodies: dict, theta, omega):
        """bodies: centre [B], first [B+1], member [M], offset [M, 2], inertia [B] (tags; host arrays)."""
        dev = system.device
        self.S = system
        self.b = {k: torch.as_tensor(np.ascontiguousarray(bodies[k]), device=dev)
                  for k in ("centre", "first", "member", "offset", "inertia")}
        for k in ("centre", "first", "member"):
            self.b[k] = self.b[k].to(torch.int32)
        self.b["offset"] = self.b["offset"].to(torch.float32).contiguous()
        self.b["inertia"] = self.b["inertia"].to(torch.float32)
        self.theta = torch.as_tensor(np.asarray(theta, np.float32), device=dev).clone()
        self.omega = torch.as_tensor(np.asarray(omega, np.float32), device=dev).clone()

    def _half(self, cfg, step, half):
        S = self.S
        api.rc_rigid_step(S.ctx, S.pos, S.vel, S.force, S.image, S.rtag, self.b, self.theta, self.omega, S.box,
                          cfg, step, half, S.status)

    def run(self, n_steps: int, cfg, step0: int = 0, soft_frac: float = 0.8) -> dict:
        """n_steps body steps (cfg: an integrator of dim 2); returns rebuild count and wall time."""
        S = self.S
        if not S.built:
            S.build()
        soft = 0.5 * S.r_buff * soft_frac
        S.compute_forces(gather=True, ev=False)
        rebuilds = 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(n_steps):
            self._half(cfg, step0 + k, rcl.RC_HALF_FIRST)
            mp = float(S.vel[:, 3].max())
            if not math.isfinite(mp):
                raise RuntimeError(f"rigid bodies: non-finite state at step {step0 + k}")
            if mp > soft:
                S.build()
                rebuilds += 1
            S.compute_forces(gather=True, ev=False)
            self._half(cfg, step0 + k, rcl.RC_HALF_SECOND)
        torch.cuda.synchronize()
        return {"rebuilds": rebuilds, "seconds": time.perf_counter() - t0}
