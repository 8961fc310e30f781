"""``Batch``: device buffers of R independent replicas and calls into the engine.

Replica r occupies the slots ``offsets[r] .. offsets[r] + counts[r]`` of every
per-particle array (slot ranges start at multiples of 64; the slots between
replicas are unused).  Tags are global, ``offsets[r] + local tag``.  No
arithmetic of the method happens here.
"""
from __future__ import annotations

import dataclasses
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib as rcl
from . import api
from ._lib import RcError


@dataclasses.dataclass
class BatchResult:
    stats: rcl.MdStats
    ev: Optional[np.ndarray]        # [rows, R, 13]: E, W(6), K(6) per replica
    bonds: Optional[np.ndarray]     # [rows, R]


class Batch:
    """R periodic systems on the current GPU, advanced by one launch per step.

    ``systems`` is a sequence of objects with ``pos`` (N_r,3), ``types``,
    ``L``, ``table`` and optionally ``vel`` and ``mass``; all tables have the
    same number of types and all replicas the same per-type masses.
    """

    def __init__(self, systems: Sequence, r_buff: float = 0.3, k_max: int = 32, rollback: bool = True,
                 device: str = "cuda", seeds=None, rebuild_margin: float = 0.3):
        self.device = torch.device(device)
        R = len(systems)
        self.R = R
        tables = [s.table for s in systems]
        counts = [int(np.asarray(s.pos).shape[0]) for s in systems]
        boxes = [api.box(s.L) for s in systems]
        self.bc = api.BatchContext(tables, counts, boxes, r_buff)
        self.counts = self.bc.counts
        self.offsets = self.bc.offsets
        self.n_slots = self.bc.n_slots
        nt = self.bc.ntypes
        m0 = getattr(systems[0], "mass", None)
        self.mass = np.ones(nt) if m0 is None else np.asarray(m0, dtype=np.float64)
        for s in systems[1:]:
            m = getattr(s, "mass", None)
            if m is not None and not np.array_equal(np.asarray(m, dtype=np.float64), self.mass):
                raise ValueError("all replicas must share the per-type masses")
        S = self.n_slots
        pos = np.zeros((S, 4), np.float32)
        vel = np.zeros((S, 4), np.float32)
        for r, s in enumerate(systems):
            o, n = int(self.offsets[r]), counts[r]
            ty = np.asarray(s.types)
            if ty.size and (ty.min() < 0 or ty.max() >= nt):
                raise ValueError(f"replica {r}: particle types must lie in [0, {nt})")
            p = api.pack_positions(s.pos, ty, tags=o + np.arange(n), device="cpu").numpy()
            pos[o:o + n] = p
            if getattr(s, "vel", None) is not None:
                vel[o:o + n, :3] = np.asarray(s.vel, dtype=np.float32)
        dev = self.device
        self.pos = torch.from_numpy(pos).to(dev)
        self.pos_alt = torch.zeros_like(self.pos)
        self.vel = torch.from_numpy(vel).to(dev)
        self.image = torch.zeros((S, 4), dtype=torch.int32, device=dev)
        self.rtag = torch.zeros(S, dtype=torch.int32, device=dev)
        self.k_max = int(k_max)
        self.nlist = torch.zeros(self.k_max * S, dtype=torch.int32, device=dev)
        self.nn = torch.zeros(S, dtype=torch.int32, device=dev)
        self.ws = torch.empty(api.rc_batch_cells_workspace_bytes(self.bc), dtype=torch.uint8, device=dev)
        self.status = torch.zeros(rcl.RC_STATUS_WORDS, dtype=torch.int32, device=dev)
        self.force = torch.zeros((S, 4), dtype=torch.float32, device=dev)
        self.ev = torch.zeros((R, 13), dtype=torch.float64, device=dev)
        self.bonds = torch.zeros(R, dtype=torch.int64, device=dev)
        self.rollback = rollback
        if rollback:
            self.snap_pos = torch.empty_like(self.pos)
            self.snap_vel = torch.empty_like(self.vel)
            self.snap_image = torch.empty_like(self.image)
        if seeds is not None:
            self.bc.set_seeds(seeds)
        self.bc.set_rebuild_margin(rebuild_margin)
        self.built = False
        self._continues = False     # the state is what the last run left (its list may be kept)
        self._attach_workspace()

    @classmethod
    def from_workloads(cls, systems, **kw):
        return cls(systems, **kw)

    # ---- neighbour lists -------------------------------------------------------------
    def _grow(self, k_needed: int):
        """Larger lists; the current lists are carried over (a resumed run rebuilds only the replicas of
        the build that overflowed, the others keep theirs)."""
        k_old, old = self.k_max, self.nlist
        self.k_max = int(max(k_needed + 4, int(self.k_max * 1.5)))
        self.nlist = torch.zeros(self.k_max * self.n_slots, dtype=torch.int32, device=self.device)
        self._attach_workspace()
        api.rc_batch_relayout_lists(self.bc, old, k_old, self.nlist, self.k_max, self.nn)

    def _attach_workspace(self):
        """The batch's large scratch (packed lists, switching sums) in a torch-owned buffer."""
        self.work = None
        api.rc_batch_set_workspace(self.bc, None)
        self.work = torch.empty(api.rc_batch_workspace_bytes(self.bc, self.k_max), dtype=torch.uint8,
                                device=self.device)
        api.rc_batch_set_workspace(self.bc, self.work, self.k_max)

    def build(self):
        """Bin, re-order and build every replica's list (grows k_max on overflow)."""
        for _ in range(4):
            api.rc_batch_build_cells(self.bc, self.pos, self.vel, self.image, self.rtag, self.ws)
            api.rc_clear_status(self.status)
            api.rc_batch_build_nlist(self.bc, self.pos, self.vel, self.ws, self.k_max, self.nlist, self.nn,
                                     self.status)
            code, st = api.rc_read_status(self.status)
            if code == rcl.RC_ERR_NLIST_OVERFLOW:
                self._grow(st[rcl.RC_ST_KMAX])
                continue
            if code != rcl.RC_OK:
                raise RcError(code, "batch neighbour list build")
            self.built = True
            self._continues = False
            return st[rcl.RC_ST_KMAX]
        raise RcError(rcl.RC_ERR_NLIST_OVERFLOW, "could not size the neighbour lists")

    # ---- single evaluations ----------------------------------------------------------------
    def compute_forces(self):
        """Forces (slots,4) and per-replica [E, W(6)] (R,7) float64."""
        if not self.built:
            self.build()
        ev = torch.zeros((self.R, 7), dtype=torch.float64, device=self.device)
        api.rc_batch_compute_forces(self.bc, self.pos, self.nlist, self.nn, self.force, ev, self.status)
        return self.force, ev

    def bond_count(self) -> np.ndarray:
        if not self.built:
            self.build()
        api.rc_batch_bond_count(self.bc, self.pos, self.nlist, self.nn, self.bonds)
        return self.bonds.cpu().numpy().astype(np.int64)

    # ---- dynamics -----------------------------------------------------------------------------
    def set_gather_width(self, width: int):
        """Entries per lane and pass of the fused step kernel (1, 2, 4): speed only."""
        self.bc.set_gather_width(width)

    def set_step_form(self, form: str):
        """"walk" (one pass, partner sums by list walks) or "sums" (two passes): speed only."""
        self.bc.set_step_form(form)

    def set_rebuild_margin(self, margin: float):
        """Replicas whose largest path length since their last list build exceeds margin x the rebuild
        threshold are rebuilt with the ones that crossed it (0: every replica at every build)."""
        self.bc.set_rebuild_margin(margin)

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

    def run(self, n_steps: int, cfg, step0: int = 0, log_period: int = 0, use_graph: bool = True,
            graph_steps: int = 16, max_chunk: int = 256, soft_frac: float = 0.8, adapt: bool = True,
            keep_list: bool = True, time_kernels: bool = False) -> BatchResult:
        """Advance every replica n_steps under the chunked driver (log rows and keep_list as
        System.run)."""
        rows = (n_steps // log_period + 2) if log_period > 0 else 1
        ev_log = torch.zeros((rows, self.R, 13), dtype=torch.float64, device=self.device)
        bonds_log = torch.zeros((rows, self.R), dtype=torch.int64, device=self.device)
        opts = rcl.MdOptions(int(use_graph), int(graph_steps), int(max_chunk), int(log_period), float(soft_frac),
                             int(adapt), 0, 0, int(keep_list and self._continues), int(time_kernels))
        self._continues = False
        for _ in range(4):
            try:
                st = api.rc_batch_run(self.bc, self.md_buffers(ev_log, bonds_log), cfg, step0, n_steps, opts)
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
            raise RcError(rcl.RC_ERR_NLIST_OVERFLOW, "could not size the neighbour lists")
        self.built = True
        self._continues = True
        n = int(st.log_rows)
        return BatchResult(stats=st, ev=ev_log[:n].cpu().numpy(), bonds=bonds_log[:n].cpu().numpy())

    # ---- per-replica views in tag order ------------------------------------------------------
    def slots(self, r: int) -> slice:
        o = int(self.offsets[r])
        return slice(o, o + int(self.counts[r]))

    def state_by_tag(self, r: int):
        """(pos (n,3), vel (n,3), image (n,3), types) of replica r in its own tag order."""
        sl = self.slots(r)
        xyz, types, tags = api.unpack_positions(self.pos[sl])
        order = np.argsort(tags)
        v = self.vel[sl].cpu().numpy()[:, :3]
        im = self.image[sl].cpu().numpy()[:, :3]
        return xyz[order], v[order], im[order], types[order]

    def by_tag(self, arr: torch.Tensor, r: int) -> np.ndarray:
        """Replica r's rows of a per-slot device array, in its tag order (numpy)."""
        sl = self.slots(r)
        _, _, tags = api.unpack_positions(self.pos[sl])
        a = arr[sl].detach().cpu().numpy()
        out = np.empty_like(a)
        out[tags - int(self.offsets[r])] = a
        return out
