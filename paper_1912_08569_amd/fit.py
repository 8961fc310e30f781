"""Gradient fit of lambda through a Langevin trajectory.

The trajectory is BAOAB with the engine's own thermostat noise (the normals
``rc_md_run`` draws for the same seed, tags and steps, pre-drawn with
``rc_thermostat_normals``), so it is a deterministic, differentiable function
of lambda and follows the integrator of the engine; the forces come from
``swap_forces`` and the observable is the soft bond count per swap particle
(the sum of vhat over swap pairs, eq. pot) averaged over the steps.  Backpropagation through the trajectory uses
checkpointed recomputation: only every ``segment``-th state is kept in the
forward pass and each segment is recomputed in the backward pass, so memory
grows with steps/segment instead of steps.
"""
from __future__ import annotations

import math
from typing import Dict, List

import torch
from torch.utils.checkpoint import checkpoint

from . import api
from .autograd import SwapModel, soft_bonds, swap_forces


class TrajectoryFit:
    """Loss (mean soft bonds per swap particle - target)^2 over ``steps`` BAOAB steps."""

    def __init__(self, model: SwapModel, x0, v0, masses, dt: float, kT: float, gamma: float, steps: int,
                 segment: int, n_swap: int, seed: int = 0, step0: int = 0):
        self.model = model
        self.x0 = x0.detach().to(torch.float32)
        self.v0 = v0.detach().to(torch.float32)
        self.minv = (1.0 / masses.to(torch.float32)).reshape(-1, 1)
        self.dt, self.steps, self.segment = float(dt), int(steps), int(segment)
        c1 = math.exp(-gamma * dt)
        self.c1 = c1
        self.c2 = torch.sqrt((1.0 - c1 * c1) * kT * self.minv)
        # x0 is in tag order: row t of step k is the noise of tag t at step step0 + k
        xi = api.rc_thermostat_normals(seed, step0, self.steps, self.x0.shape[0], device=self.x0.device)
        self.noise = xi[..., :3].contiguous()
        self.n_swap = int(n_swap)

    def _segment(self, k0: int, k1: int, theta, x, v, F):
        h = 0.5 * self.dt
        acc = torch.zeros((), dtype=torch.float64, device=x.device)
        for k in range(k0, k1):
            v = v + h * F * self.minv
            x = x + h * v
            v = self.c1 * v + self.c2 * self.noise[k]
            x = x + h * v
            F = swap_forces(self.model, x, theta)
            v = v + h * F * self.minv
            acc = acc + soft_bonds(self.model, x)
        return x, v, F, acc

    def observable(self, theta, checkpointed: bool = True):
        """Mean soft bonds per swap particle over the trajectory (differentiable in theta)."""
        x, v = self.x0, self.v0
        F = swap_forces(self.model, x, theta)
        total = torch.zeros((), dtype=torch.float64, device=x.device)
        for k0 in range(0, self.steps, self.segment):
            k1 = min(k0 + self.segment, self.steps)
            if checkpointed:
                x, v, F, acc = checkpoint(self._segment, k0, k1, theta, x, v, F, use_reentrant=False)
            else:
                x, v, F, acc = self._segment(k0, k1, theta, x, v, F)
            total = total + acc
        return total / (self.steps * self.n_swap)

    def loss(self, theta, target: float, checkpointed: bool = True):
        return (self.observable(theta, checkpointed) - target) ** 2


def fit_lambda(fit: TrajectoryFit, entry, lam0: float, target: float, iters: int = 10, step: float = 0.1,
               lam_min: float = 0.0) -> List[Dict]:
    """Gradient descent on lambda of table entry ``entry`` = (a, b); returns the history.

    The first move has length ``step``; a move that raises the loss is undone
    and the step halved, a move that lowers it lets the step grow by half.
    """
    a, b = min(entry), max(entry)
    theta0 = fit.model.theta()
    mask = torch.zeros_like(theta0)
    mask[a, b, 2] = 1.0
    lam = float(lam0)
    hist: List[Dict] = []
    prev = None
    for it in range(iters):
        t = torch.tensor(lam, dtype=torch.float64, requires_grad=True)
        L = fit.loss(theta0 * (1 - mask) + mask * t, target)
        (g,) = torch.autograd.grad(L, t)
        rec = {"iter": it, "lambda": lam, "loss": float(L.detach()), "grad": float(g), "step": step}
        hist.append(rec)
        if prev is not None and rec["loss"] > prev["loss"]:
            lam, step = prev["lambda"], 0.5 * step       # undo, shorter move along the old gradient
            g_use = prev["grad"]
        else:
            prev, g_use = rec, float(g)
            if it > 0:
                step *= 1.5
        if g_use == 0.0:
            break
        lam = max(lam_min, lam - step * (1.0 if g_use > 0 else -1.0))
    return hist
