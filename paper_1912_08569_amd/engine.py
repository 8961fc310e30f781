"""``System``: device buffers of one periodic system and calls into the engine.

Owns the torch tensors the C ABI works on (positions in two buffers,
velocities, image counters, tag map, neighbour list, cell workspace, status
word, rollback snapshots) and forwards to the ``rc_*`` entry points.  No
arithmetic of the method happens here.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np
import torch

from . import _lib as rcl
from . import api
from ._lib import RcError


@dataclasses.dataclass
class RunResult:
    stats: rcl.MdStats
    ev: Optional[np.ndarray]        # [rows, 13]: E, W(6), K(6)
    bonds: Optional[np.ndarray]     # [rows]


class System:
    """One periodic system on the current GPU.

    ``pos`` (N,3) FP32 in [-L/2, L/2), ``types`` (N,), ``L`` (FP32 edge or 3 edges),
    ``table`` (kind, epsilon, sigma, n, rcut, lam arrays), optional ``vel`` (N,3).
    """

    # Mean swap-range length from which the two-pass (sums) form of the step beats the one-pass walk
    # form.  The walk form pays a walk of the partner's swap range for every active swap entry; the
    # sums form pays one more pass over all particles.  Measured at 8k-1M particles: walk is faster
    # at 0.14 (site/colloid mixture), the two tie near 0.53, sums is faster from 0.8 on.
    AUTO_SUMS_KSWAP = 0.5

    def __init__(self, pos, types, L, table, vel=None, mass=None, r_buff: float = 0.3, k_max: int = 32,
                 rollback: bool = True, device: str = "cuda", bonds=None, fene=None, step_form: str = "auto"):
        self.device = torch.device(device)
        self.step_form = step_form
        self.ctx = api.Context(table, r_buff)
        self.r_buff = float(r_buff)
        self.table = table
        self.N = int(np.asarray(pos).shape[0])
        self.edges = [float(L)] * 3 if np.isscalar(L) else [float(x) for x in L]
        self.box = api.box(self.edges)
        nt = self.ctx.ntypes
        ty = np.asarray(types)
        if ty.size and (ty.min() < 0 or ty.max() >= nt):
            raise ValueError(f"particle types must lie in [0, {nt})")
        self.mass = np.ones(nt) if mass is None else np.asarray(mass, dtype=np.float64)
        N = self.N
        dev = self.device
        self.pos = api.pack_positions(pos, types, device=dev)
        self.pos_alt = torch.empty_like(self.pos)
        v = np.zeros((N, 4), np.float32)
        if vel is not None:
            v[:, :3] = np.asarray(vel, dtype=np.float32)
        self.vel = torch.from_numpy(v).to(dev)
        self.image = torch.zeros((N, 4), dtype=torch.int32, device=dev)
        self.rtag = torch.zeros(N, dtype=torch.int32, device=dev)
        self.k_max = int(k_max)
        self.nlist = torch.zeros(self.k_max * N, dtype=torch.int32, device=dev)
        self.nn = torch.zeros(N, dtype=torch.int32, device=dev)
        ws = api.rc_cells_workspace_bytes(self.ctx, N, self.box)
        self.ws = torch.empty(ws, dtype=torch.uint8, device=dev)
        self.status = torch.zeros(rcl.RC_STATUS_WORDS, dtype=torch.int32, device=dev)
        self.force = torch.zeros((N, 4), dtype=torch.float32, device=dev)
        self.ev = torch.zeros(13, dtype=torch.float64, device=dev)
        self.count = torch.zeros(1, dtype=torch.int64, device=dev)
        self.rollback = rollback
        if rollback:
            self.snap_pos = torch.empty_like(self.pos)
            self.snap_vel = torch.empty_like(self.vel)
            self.snap_image = torch.empty_like(self.image)
        # FENE springs: partner tags per tag, read through rtag (kept by every cell build)
        self.bonds = None
        if bonds is not None:
            if fene is None:
                raise ValueError("bonds need fene=(K, R0)")
            self.bonds = torch.from_numpy(np.ascontiguousarray(np.asarray(bonds, dtype=np.int32))).to(dev)
            self.fene = (float(fene[0]), float(fene[1]))
            api.rc_set_bonds(self.ctx, self.bonds, self.rtag, *self.fene)
            self.ev_fene = torch.zeros(7, dtype=torch.float64, device=dev)
        self.built = False
        self._continues = False     # the state is what the last run left (its list may be kept)
        self._log = None            # log rows of the last run (ev rows, then bond counts)
        self._log_np = None         # numpy view of _log
        self._bufs_cache = None     # (tensors, MdBuffers, log address) of the last run
        # the context's large scratch (packed list, switching sums, HVP sums) in a torch-owned buffer
        self._attach_workspace(nvec=1)

    def _attach_workspace(self, nvec: int):
        self._ws_nvec = int(nvec)
        nb = self.ctx.workspace_bytes(self.N, self.k_max, self._ws_nvec)
        self.work = None
        self.ctx.set_workspace(None)
        self.work = torch.empty(nb, dtype=torch.uint8, device=self.device)
        self.ctx.set_workspace(self.work, self.N, self.k_max, self._ws_nvec)

    @classmethod
    def from_workload(cls, sysw, **kw):
        extra = {}
        if getattr(sysw, "bonds", None) is not None:
            extra = {"bonds": sysw.bonds, "fene": sysw.fene}
        return cls(sysw.pos, sysw.types, sysw.L, sysw.table, vel=sysw.vel, mass=sysw.mass, **extra, **kw)

    # ---- neighbour list -----------------------------------------------------------
    def _grow(self, k_needed: int):
        self.k_max = int(max(k_needed + 4, int(self.k_max * 1.5)))
        self.nlist = torch.zeros(self.k_max * self.N, dtype=torch.int32, device=self.device)
        self._attach_workspace(self._ws_nvec)

    def build(self):
        """Bin, re-order and build the neighbour list (grows k_max on overflow)."""
        for _ in range(4):
            api.rc_build_cells(self.ctx, self.pos, self.vel, self.image, self.rtag, self.box, self.ws)
            api.rc_clear_status(self.status)
            api.rc_build_nlist(self.ctx, self.pos, self.vel, self.box, self.ws, self.k_max, self.nlist,
                               self.nn, self.status)
            code, st = api.rc_read_status(self.status)
            if code == rcl.RC_ERR_NLIST_OVERFLOW:
                self._grow(st[rcl.RC_ST_KMAX])
                continue
            if code != rcl.RC_OK:
                raise RcError(code, "neighbour list build")
            self.built = True
            self._continues = False
            if self.step_form == "auto":
                self.ctx.set_step_form(self._form_for(int(st[rcl.RC_ST_NSWAP])))
            return st[rcl.RC_ST_KMAX]
        raise RcError(rcl.RC_ERR_NLIST_OVERFLOW, "could not size the neighbour list")

    # ---- single evaluations -----------------------------------------------------
    def compute_forces(self, gather=False, ev: bool = True):
        """Forces (N,4: xyz + per-particle energy) and, if ev, [E, W(6)] (float64).

        gather: False = triplet kernel, True = gather kernel, "sums" = the
        gather in the two-pass form."""
        if not self.built:
            self.build()
        flags = rcl.RC_FORCE_SUMS if gather == "sums" else (rcl.RC_FORCE_GATHER if gather else 0)
        api.rc_compute_forces(self.ctx, self.pos, self.nlist, self.nn, self.box, self.force,
                              self.ev if ev else None, flags, self.status)
        if self.bonds is not None:      # springs on top (accumulated)
            api.rc_fene_forces(self.ctx, self.pos, self.box, self.force, self.ev_fene if ev else None)
            if ev:
                self.ev[:7] += self.ev_fene
        return self.force, (self.ev[:7] if ev else None)

    def bond_partners(self) -> np.ndarray:
        """Bond partner of every particle, by tag (the partner's tag; -1 none, -2 several)."""
        out = torch.empty(self.N, dtype=torch.int32, device=self.device)
        api.rc_bond_partners(self.ctx, self.pos, self.nlist, self.nn, self.box, out)
        return out.cpu().numpy()

    def partner_counts(self, p0, pt, select=None):
        """(bonded at 0, unchanged, swapped) between two partner snapshots by tag (bond_partners()
        output), over the tags where select is true (None: all).  unchanged / bonded is the bond
        autocorrelation; swapped counts bonded sites whose partner changed."""
        dev = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt).to(self.device)  # noqa: E731
        sel = None if select is None else dev(np.asarray(select, bool).astype(np.uint8), torch.uint8)
        counts = torch.zeros(3, dtype=torch.int64, device=self.device)
        api.rc_partner_counts(self.ctx, dev(p0, torch.int32), dev(pt, torch.int32), sel, counts)
        return tuple(int(x) for x in counts.cpu().numpy())

    def stress_autocorrelation(self, rows, kT: float, max_lag: int) -> np.ndarray:
        """G(t), t = 0 .. max_lag log rows, of logged rows (E, W(6), K(6)) such as RunResult.ev."""
        r = torch.as_tensor(np.ascontiguousarray(rows, dtype=np.float64)).to(self.device)
        G = torch.empty(max_lag + 1, dtype=torch.float64, device=self.device)
        volume = float(self.box.L[0]) * float(self.box.L[1]) * float(self.box.L[2])
        api.rc_stress_autocorrelation(self.ctx, r, volume, kT, max_lag, G)
        return G.cpu().numpy()

    def bond_count(self) -> int:
        if not self.built:
            self.build()
        api.rc_bond_count(self.ctx, self.pos, self.nlist, self.nn, self.box, self.count)
        return int(self.count.item())

    def hvp(self, v: torch.Tensor) -> torch.Tensor:
        """H v for v of shape (N,4) in the engine's particle order."""
        if not self.built:
            self.build()
        out = torch.empty_like(self.pos)
        api.rc_force_hvp(self.ctx, self.pos, self.nlist, self.nn, self.box, v.contiguous(), out)
        return out

    def reserve_hvp_vectors(self, nvec: int):
        """Grow the caller-owned workspace so that batched products of up to
        ``nvec`` tangent vectors fit (raw rc_force_hvp_batch calls need it)."""
        if int(nvec) > self._ws_nvec:
            self._attach_workspace(int(nvec))

    def hvp_batch(self, V: torch.Tensor) -> torch.Tensor:
        """H V[k] for V of shape (nvec, N, 4) in the engine's particle order, one launch per pass."""
        if not self.built:
            self.build()
        V = V.contiguous()
        self.reserve_hvp_vectors(V.shape[0])
        out = torch.empty_like(V)
        api.rc_force_hvp_batch(self.ctx, self.pos, self.nlist, self.nn, self.box, V, out)
        return out

    def param_grad(self) -> np.ndarray:
        if not self.built:
            self.build()
        nt = self.ctx.ntypes
        g = torch.zeros(nt * nt * 3, dtype=torch.float64, device=self.device)
        api.rc_param_grad(self.ctx, self.pos, self.nlist, self.nn, self.box, g)
        return g.cpu().numpy().reshape(nt, nt, 3)

    def param_vjp(self, adj: torch.Tensor) -> np.ndarray:
        """sum_m adj_m . dF_m/dtheta for theta = (eps, sigma, lambda) of every entry, adj (N,4) in engine order."""
        if not self.built:
            self.build()
        nt = self.ctx.ntypes
        g = torch.zeros(nt * nt * 3, dtype=torch.float64, device=self.device)
        api.rc_param_vjp(self.ctx, self.pos, self.nlist, self.nn, self.box, adj.contiguous(), g)
        return g.cpu().numpy().reshape(nt, nt, 3)

    def soft_bonds(self, grad: bool = False):
        """Soft bond count (float64 device scalar) and, if grad, its gradient (N,4) in engine order."""
        if not self.built:
            self.build()
        val = torch.zeros(1, dtype=torch.float64, device=self.device)
        g = torch.empty_like(self.pos) if grad else None
        api.rc_soft_bonds(self.ctx, self.pos, self.nlist, self.nn, self.box, val, g)
        return val, g

    def set_table(self, table):
        """Replace eps, sigma, lambda (kinds, exponents and cutoffs unchanged)."""
        self.ctx.set_table(table)
        self.table = table

    # ---- dynamics ------------------------------------------------------------------
    def set_gather_width(self, width: int):
        """Entries per lane and pass of the fused step kernel (1, 2, 4): speed only."""
        self.ctx.set_gather_width(width)

    def set_step_form(self, form: str):
        """"walk" (one pass, partner sums by list walks), "sums" (two passes) or "auto" (walk or sums by
        the mean swap-range length of the list, chosen at every build from the status word it writes and
        after every run that rebuilt): speed only."""
        self.step_form = form
        if form == "auto":
            if self.built:
                self.ctx.set_step_form(self.auto_step_form())
        else:
            self.ctx.set_step_form(form)

    def auto_step_form(self) -> str:
        """The form "auto" picks for the current list: "sums" or "walk"."""
        return "sums" if self.mean_swap_length() >= self.AUTO_SUMS_KSWAP else "walk"

    def _form_for(self, nswap: int) -> str:
        """The auto form for a list whose swap ranges hold nswap entries in all (the status word the
        list build writes, so no device work is needed to choose)."""
        return "sums" if nswap >= self.AUTO_SUMS_KSWAP * self.N else "walk"

    def mean_swap_length(self) -> float:
        """Mean length of the swap range of the last list build."""
        return float((self.nn & 0xFFFF).float().mean().item())

    def mean_list_length(self) -> float:
        """Mean neighbour-list length of the last build (swap and other ranges)."""
        nn = self.nn
        return float(((nn & 0xFFFF) + (nn >> 16)).float().mean().item())

    def integrator(self, kind="langevin", dt=0.002, kT=1.0, gamma=1.0, seed=0, dim=3):
        return api.integrator(kind, dt, kT, gamma, seed, list(self.mass), dim=dim)

    def md_buffers(self, ev_log=None, bonds_log=None) -> rcl.MdBuffers:
        b = rcl.MdBuffers()
        p = lambda t: None if t is None else t.data_ptr()  # noqa: E731
        b.pos, b.pos_alt, b.vel = p(self.pos), p(self.pos_alt), p(self.vel)
        b.image, b.rtag, b.nlist, b.nn = p(self.image), p(self.rtag), p(self.nlist), p(self.nn)
        b.k_max = self.k_max
        b.cells_ws = p(self.ws)
        b.cells_ws_bytes = self.ws.numel()
        if self.rollback:
            b.snap_pos, b.snap_vel, b.snap_image = p(self.snap_pos), p(self.snap_vel), p(self.snap_image)
        b.status = p(self.status)
        b.ev_log, b.bonds_log = p(ev_log), p(bonds_log)
        return b

    def _run_buffers(self, rows: int) -> rcl.MdBuffers:
        """md_buffers for a run with `rows` log rows in the pinned log buffer (ev rows, then the bond
        counts).  The struct is kept while the same tensors hold the state (a replaced tensor, as after a
        list growth, rebuilds it): filling it costs more host time than a short run's steps leave idle."""
        key = (self.pos, self.pos_alt, self.vel, self.image, self.rtag, self.nlist, self.nn, self.ws,
               self.status, self._log) + ((self.snap_pos, self.snap_vel, self.snap_image) if self.rollback else ())
        c = self._bufs_cache
        if (c is None or c[3] != self.k_max or len(c[0]) != len(key)
                or not all(x is y for x, y in zip(c[0], key))):
            c = self._bufs_cache = (key, self.md_buffers(), self._log.data_ptr(), self.k_max)
        b, base = c[1], c[2]
        b.ev_log = base
        b.bonds_log = base + rows * 13 * 8   # u64 counts after the rows
        return b

    def run(self, n_steps: int, cfg, step0: int = 0, log_period: int = 0, use_graph: bool = True,
            graph_steps: int = 16, max_chunk: int = 256, soft_frac: float = 0.8, adapt: bool = True,
            one_block: bool = True, keep_list: bool = True, time_kernels: bool = False) -> RunResult:
        """Advance n_steps with the fused step kernel under the chunked driver.

        Log rows are taken at the step indices in [step0, step0 + n_steps) that are multiples of
        log_period (none for 0) and at the end; a continued run (keep_list) does not repeat the last
        run's final row.
        one_block: with use_graph, systems of at most 1024 particles run each replay of graph_steps
        steps in one workgroup launch (same results, bit for bit).
        keep_list: a run that starts where the last one ended (step0 = its last step) continues on
        its neighbour list instead of building one at entry; code that writes the state tensors
        directly calls invalidate() first.
        time_kernels: launch every step directly with events around its kernels; the stats then
        hold the summed kernel time (kernel_ms over kernel_launches)."""
        if self.step_form == "auto" and not self.built:
            self.build()    # picks the form from the new list
        rows = (n_steps // log_period + 2) if log_period > 0 else 1
        if self._log is None or self._log.shape[0] < rows * 14:
            # pinned host memory, which the driver's kernels write directly: the rows are on the host when
            # the run returns (its last status read waits for them), with no copy back
            self._log = torch.zeros(max(rows, 64) * 14, dtype=torch.float64, pin_memory=True)
            self._log_np = self._log.numpy()
        opts = rcl.MdOptions(int(use_graph), int(graph_steps), int(max_chunk), int(log_period), float(soft_frac),
                             int(adapt), int(one_block), 0, int(keep_list and self._continues), int(time_kernels))
        self._continues = False
        for _ in range(4):
            try:
                st = api.rc_md_run(self.ctx, self._run_buffers(rows), self.N, self.box, cfg, step0, n_steps,
                                   opts)
                break
            except RcError as e:
                if e.code != rcl.RC_ERR_NLIST_OVERFLOW:
                    raise
                done = int(e.stats.steps_done)
                if done > 0:        # the state owes its last step's final half kick
                    opts.resume = 1
                self._grow(int(e.stats.k_needed))
                step0 += done
                n_steps -= done
        else:
            raise RcError(rcl.RC_ERR_NLIST_OVERFLOW, "could not size the neighbour list")
        self.built = True
        self._continues = True
        if self.step_form == "auto" and st.rebuilds > 0:   # the next run takes the form of the last list
            self.ctx.set_step_form(self._form_for(st.nswap))
        n = int(st.log_rows)
        ev = self._log_np[:rows * 13].reshape(rows, 13)[:n].copy()
        bonds = self._log_np[rows * 13:rows * 14].view(np.int64)[:n].copy()
        return RunResult(stats=st, ev=ev, bonds=bonds)

    def invalidate(self):
        """Mark the state as changed outside the engine: the next run builds its list at entry."""
        self._continues = False

    # ---- state in tag order ----------------------------------------------------------
    def state_by_tag(self):
        """(pos (N,3) float32, vel (N,3), image (N,3), types) in tag order."""
        xyz, types, tags = api.unpack_positions(self.pos)
        order = np.argsort(tags)
        v = self.vel.cpu().numpy()[:, :3]
        im = self.image.cpu().numpy()[:, :3]
        return xyz[order], v[order], im[order], types[order]

    def by_tag(self, arr: torch.Tensor) -> np.ndarray:
        """Re-order a per-particle device array into tag order (numpy)."""
        _, _, tags = api.unpack_positions(self.pos)
        a = arr.detach().cpu().numpy()
        out = np.empty_like(a)
        out[tags] = a
        return out

    def to_engine_order(self, arr_by_tag: np.ndarray) -> torch.Tensor:
        _, _, tags = api.unpack_positions(self.pos)
        return torch.from_numpy(np.ascontiguousarray(np.asarray(arr_by_tag)[tags])).to(self.device)
