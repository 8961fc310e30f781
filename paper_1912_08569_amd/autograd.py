"""torch.autograd bindings: energy, forces and the soft bond count as
differentiable functions of the positions and of the per-entry parameters.

Positions are (N, 3) float32 device tensors in tag order (the engine's own
order changes at every list build; ``SwapModel`` maps between the two).  The
parameters are an (nt, nt, 3) float64 CPU tensor theta = (eps, sigma, lambda)
per entry; entry {a, b} is read from theta[min(a,b), max(a,b)] and its
gradient is reported there (the lower triangle gets zeros).  Every value and
derivative comes from the HIP library:

  energy   E(x, theta):  dE/dx = -F,  dE/dtheta = rc_param_grad
  forces   F(x, theta):  a . dF/dx = -H a (rc_force_hvp),  a . dF/dtheta = rc_param_vjp
  soft bonds B(x):        dB/dx = rc_soft_bonds' gradient
"""
from __future__ import annotations

import numpy as np
import torch

from . import _lib as rcl
from . import api


class SwapModel:
    """A ``System`` seen through tag-ordered positions and a parameter tensor.

    Keeps the neighbour list valid: a call whose positions moved more than
    half the skin (minimum image) from those of the last build rebuilds it.
    """

    def __init__(self, system):
        self.S = system
        self.L = torch.tensor(system.edges, dtype=torch.float32, device=system.device)
        self.half_skin = 0.5 * system.ctx.r_buff
        self.base = system.table.copy()
        self._theta = None
        system.build()
        self._perm = (system.pos[:, 3].view(torch.int32) >> rcl.RC_TYPE_BITS).long()
        self._ref = self._to_tag(system.pos).to(torch.float32)
        self.rebuilds = 0

    def positions(self) -> torch.Tensor:
        """Current positions of the system in tag order (N, 3)."""
        return self._to_tag(self.S.pos).clone()

    # ---- parameters ---------------------------------------------------------------------------
    def theta(self) -> torch.Tensor:
        t = self.base
        return torch.tensor(np.stack([t.epsilon, t.sigma, t.lam], axis=-1), dtype=torch.float64)

    def _load_theta(self, theta: torch.Tensor):
        th = theta.detach().cpu().numpy().astype(np.float64)
        if self._theta is not None and np.array_equal(th, self._theta):
            return
        nt = th.shape[0]
        tab = self.base.copy()
        for a in range(nt):
            for b in range(nt):
                lo, hi = min(a, b), max(a, b)
                if tab.kind[a, b] == 0:
                    continue
                tab.epsilon[a, b], tab.sigma[a, b] = th[lo, hi, 0], th[lo, hi, 1]
                tab.lam[a, b] = th[lo, hi, 2] if tab.kind[a, b] == rcl.RC_KIND_SWAP else tab.lam[a, b]
        self.S.set_table(tab)
        self._theta = th

    @staticmethod
    def _upper(g: np.ndarray) -> torch.Tensor:
        nt = g.shape[0]
        out = np.zeros_like(g)
        iu = np.triu_indices(nt)
        out[iu] = g[iu]
        return torch.from_numpy(out)

    # ---- positions ----------------------------------------------------------------------------------
    def _wrap(self, xyz):
        L = self.L
        w = xyz - L * torch.floor((xyz + 0.5 * L) / L)
        return torch.where(w >= 0.5 * L, w - L, w)

    def _load_x(self, xyz: torch.Tensor):
        x = self._wrap(xyz.detach().to(torch.float32))
        S = self.S
        d = x - self._ref
        d = d - self.L * torch.round(d / self.L)
        need = bool((d * d).sum(dim=1).max() > self.half_skin ** 2)
        S.invalidate()   # positions written here, outside the driver
        S.pos[:, :3] = x[self._perm]
        if need:
            S.build()
            self._perm = (S.pos[:, 3].view(torch.int32) >> rcl.RC_TYPE_BITS).long()
            self._ref = x.clone()
            self.rebuilds += 1
        return self._perm

    def _to_tag(self, arr):
        out = torch.empty((self.S.N, 3), dtype=arr.dtype, device=arr.device)
        out[self._perm] = arr[:, :3]
        return out

    def _to_engine(self, a_tag):
        a = torch.zeros((self.S.N, 4), dtype=torch.float32, device=self.S.device)
        a[:, :3] = a_tag.detach().to(torch.float32)[self._perm]
        return a

    # ---- evaluations (tag order) ---------------------------------------------------------------
    def load(self, xyz, theta):
        self._load_theta(theta)
        self._load_x(xyz)

    def forces_energy(self, xyz, theta):
        self.load(xyz, theta)
        F, ev = self.S.compute_forces(gather=True)
        return self._to_tag(F), ev[0].clone()

    def hvp(self, v_tag):
        return self._to_tag(self.S.hvp(self._to_engine(v_tag)))

    def param_grad(self):
        return self._upper(self.S.param_grad())

    def param_vjp(self, a_tag):
        return self._upper(self.S.param_vjp(self._to_engine(a_tag)))

    def soft_bonds(self, xyz):
        self._load_x(xyz)
        val, g = self.S.soft_bonds(grad=True)
        return val[0].clone(), self._to_tag(g)


class _Energy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, xyz, theta, model):
        F, E = model.forces_energy(xyz, theta)
        ctx.model = model
        ctx.save_for_backward(xyz, theta, F)
        return E

    @staticmethod
    def backward(ctx, gE):
        xyz, theta, F = ctx.saved_tensors
        gx = gt = None
        if ctx.needs_input_grad[0]:
            gx = -F * gE.to(F.dtype)
        if ctx.needs_input_grad[1]:
            ctx.model.load(xyz, theta)
            gt = ctx.model.param_grad() * gE.detach().cpu()
        return gx, gt, None


class _Forces(torch.autograd.Function):
    @staticmethod
    def forward(ctx, xyz, theta, model):
        F, _ = model.forces_energy(xyz, theta)
        ctx.model = model
        ctx.save_for_backward(xyz, theta)
        return F

    @staticmethod
    def backward(ctx, gF):
        xyz, theta = ctx.saved_tensors
        model = ctx.model
        model.load(xyz, theta)
        gx = -model.hvp(gF) if ctx.needs_input_grad[0] else None
        gt = model.param_vjp(gF) if ctx.needs_input_grad[1] else None
        return gx, gt, None


class _SoftBonds(torch.autograd.Function):
    @staticmethod
    def forward(ctx, xyz, model):
        B, g = model.soft_bonds(xyz)
        ctx.save_for_backward(g)
        return B

    @staticmethod
    def backward(ctx, gB):
        (g,) = ctx.saved_tensors
        return g * gB.to(g.dtype), None


def swap_energy(model: SwapModel, xyz: torch.Tensor, theta: torch.Tensor) -> torch.Tensor:
    """Total energy (float64 scalar), differentiable in xyz and theta."""
    return _Energy.apply(xyz, theta, model)


def swap_forces(model: SwapModel, xyz: torch.Tensor, theta: torch.Tensor) -> torch.Tensor:
    """Forces (N, 3) float32 in tag order, differentiable in xyz and theta."""
    return _Forces.apply(xyz, theta, model)


def soft_bonds(model: SwapModel, xyz: torch.Tensor) -> torch.Tensor:
    """Soft bond count (float64 scalar), differentiable in xyz."""
    return _SoftBonds.apply(xyz, model)
