"""Python binding of the C ABI: the same entry points, taking torch tensors.

Each ``rc_*`` function here marshals torch device tensors into the pointers
and sizes of the matching C function in ``include/rc.h`` and raises
``RcError`` on a non-zero status.  torch supplies device memory and the
current HIP stream; all arithmetic happens in ``librc.so``.
"""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib as L
from ._lib import RcError, check

__all__ = [
    "Context", "RcError", "box", "integrator", "pack_positions", "unpack_positions",
    "rc_cells_workspace_bytes", "rc_build_cells", "rc_build_nlist", "rc_compute_forces",
    "rc_compute_forces_noalloc", "rc_thermostat_normals", "rc_workspace_bytes", "rc_set_workspace",
    "rc_ctx_device_bytes", "rc_batch_workspace_bytes", "rc_batch_set_workspace",
    "rc_integrate_step", "rc_step_fused", "rc_bond_count", "rc_md_run", "rc_force_hvp", "rc_force_hvp_batch", "rc_partner_counts", "rc_stress_autocorrelation",
    "rc_param_grad", "rc_clear_status", "rc_read_status", "rc_time_fused_steps",
    "rc_param_vjp", "rc_soft_bonds", "rc_bond_partners", "rc_set_bonds", "rc_fene_forces", "BatchContext", "rc_batch_cells_workspace_bytes", "rc_batch_build_cells", "rc_batch_build_nlist",
    "rc_batch_compute_forces", "rc_batch_bond_count", "rc_batch_step_fused", "rc_batch_run",
    "rc_batch_time_fused_steps", "rc_batch_relayout_lists",
]


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("engine buffers must be device tensors")
    if not t.is_contiguous():
        raise ValueError("engine buffers must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def box(edges) -> L.Box:
    """Box from a scalar edge or three edges (each must be an FP32 value)."""
    v = [float(edges)] * 3 if np.isscalar(edges) else [float(x) for x in edges]
    out = L.Box()
    for d in range(3):
        out.L[d] = v[d]
    return out


def integrator(kind="langevin", dt=0.002, kT=1.0, gamma=1.0, seed=0, mass: Sequence[float] = (1.0,), dim: int = 3):
    """rc_integrator; dim = 2 keeps motion in the xy plane (no thermostat noise along z)."""
    cfg = L.Integrator()
    cfg.kind = L.RC_INTEGRATOR_LANGEVIN if kind == "langevin" else L.RC_INTEGRATOR_NVE
    cfg.dim = int(dim)
    cfg.dt, cfg.kT, cfg.gamma, cfg.seed = float(dt), float(kT), float(gamma), int(seed)
    for t in range(L.RC_MAX_TYPES):
        cfg.mass[t] = float(mass[t]) if t < len(mass) else 1.0
    return cfg


def pack_positions(xyz, types, tags=None, device="cuda") -> torch.Tensor:
    """(N,3) FP32 coordinates + types (+ tags) -> (N,4) float32 with w = (tag << 4) | type."""
    xyz = np.ascontiguousarray(xyz, dtype=np.float32)
    N = xyz.shape[0]
    tags = np.arange(N, dtype=np.int64) if tags is None else np.asarray(tags, dtype=np.int64)
    w = ((tags << L.RC_TYPE_BITS) | np.asarray(types, dtype=np.int64)).astype(np.int32)
    buf = np.empty((N, 4), dtype=np.float32)
    buf[:, :3] = xyz
    buf[:, 3] = w.view(np.float32)
    return torch.from_numpy(buf).to(device)


def unpack_positions(pos: torch.Tensor):
    """(N,4) device tensor -> (xyz float32 (N,3), types, tags) as numpy."""
    a = pos.detach().cpu().numpy()
    w = a[:, 3].copy().view(np.int32)
    return a[:, :3].copy(), (w & ((1 << L.RC_TYPE_BITS) - 1)).astype(np.int32), (w >> L.RC_TYPE_BITS).astype(np.int64)


def _fill_table(arr, base, table, nt):
    for a in range(nt):
        for b in range(nt):
            e = arr[base + a * nt + b]
            e.kind = int(table.kind[a, b])
            e.n = int(table.n[a, b])
            e.epsilon = float(table.epsilon[a, b])
            e.sigma = float(table.sigma[a, b])
            e.r_cut = float(table.rcut[a, b])
            e.lam = float(table.lam[a, b])


class Context:
    """An rc_ctx: the compiled per-type-pair coefficient table."""

    def __init__(self, table, r_buff: float = 0.3):
        lib = L.load()
        nt = int(np.asarray(table.kind).shape[0])
        arr = (L.PairCoeff * (nt * nt))()
        _fill_table(arr, 0, table, nt)
        h = ctypes.c_void_p()
        code = lib.rc_create(ctypes.byref(h), nt, arr, float(r_buff))
        if code != L.RC_OK:
            raise RcError(code, "rc_create rejected the table")
        self.handle = h
        self.ntypes = nt
        self.r_buff = float(r_buff)
        self.step_form = "walk"   # the library's default form

    def close(self):
        if getattr(self, "handle", None):
            L.load().rc_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_lambda(self, lam):
        lam = np.ascontiguousarray(np.broadcast_to(np.asarray(lam, dtype=np.float64),
                                                   (self.ntypes, self.ntypes)))
        check(L.load().rc_set_lambda(self.handle, lam.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
              self.handle)

    def set_gather_width(self, width: int):
        check(L.load().rc_set_gather_width(self.handle, int(width)), self.handle)

    def workspace_bytes(self, N: int, k_max: int, nvec: int = 1) -> int:
        return rc_workspace_bytes(self, N, k_max, nvec)

    def set_workspace(self, ws: Optional[torch.Tensor], N: int = 0, k_max: int = 0, nvec: int = 0):
        rc_set_workspace(self, ws, N, k_max, nvec)

    def device_bytes(self) -> int:
        return rc_ctx_device_bytes(self)

    def set_table(self, table):
        """New eps, sigma, lambda (same kinds, exponents and cutoffs)."""
        nt = self.ntypes
        arr = (L.PairCoeff * (nt * nt))()
        _fill_table(arr, 0, table, nt)
        check(L.load().rc_set_table(self.handle, arr), self.handle)

    def set_step_form(self, form: str):
        f = {"walk": L.RC_FORM_WALK, "sums": L.RC_FORM_SUMS}[form]
        check(L.load().rc_set_step_form(self.handle, f), self.handle)
        self.step_form = form

    def rlist(self, a: int, b: int) -> float:
        out = ctypes.c_double()
        check(L.load().rc_get_rlist(self.handle, a, b, ctypes.byref(out)), self.handle)
        return out.value


# ---------------------------------------------------------------------------
# the C entry points
# ---------------------------------------------------------------------------

def rc_cells_workspace_bytes(ctx: Context, N: int, bx) -> int:
    out = ctypes.c_size_t()
    check(L.load().rc_cells_workspace_bytes(ctx.handle, int(N), bx, ctypes.byref(out)), ctx.handle)
    return int(out.value)


def rc_clear_status(status: torch.Tensor, stream=None):
    check(L.load().rc_clear_status(_ptr(status), _stream(stream)))


def rc_read_status(status: torch.Tensor, stream=None, raise_on_error=False):
    out = (ctypes.c_int * L.RC_STATUS_WORDS)()
    code = L.load().rc_read_status(_ptr(status), out, _stream(stream))
    if raise_on_error:
        check(code)
    return code, list(out)


def rc_build_cells(ctx: Context, pos, vel, image, rtag, bx, ws, stream=None):
    N = pos.shape[0]
    check(L.load().rc_build_cells(ctx.handle, _ptr(pos), _ptr(vel), _ptr(image), _ptr(rtag), N, bx,
                                  _ptr(ws), ws.numel() * ws.element_size(), _stream(stream)), ctx.handle)


def rc_build_nlist(ctx: Context, pos, vel, bx, ws, k_max, nlist, nn, status=None, stream=None):
    N = pos.shape[0]
    check(L.load().rc_build_nlist(ctx.handle, _ptr(pos), _ptr(vel), N, bx, _ptr(ws),
                                  ws.numel() * ws.element_size(), int(k_max), _ptr(nlist), _ptr(nn),
                                  _ptr(status), _stream(stream)), ctx.handle)


def _kmax(nlist, N):
    return int(nlist.numel() // max(N, 1))


def rc_rigid_step(ctx: Context, pos, vel, force, image, rtag, bodies, theta, omega, bx, cfg, step, half,
                  status=None, stream=None):
    """bodies: dict of device tensors centre, first, member, offset [M,2] float32, inertia."""
    N = pos.shape[0]
    check(L.load().rc_rigid_step(ctx.handle, _ptr(pos), _ptr(vel), _ptr(force), _ptr(image), _ptr(rtag),
                                 int(bodies["centre"].shape[0]), _ptr(bodies["centre"]), _ptr(bodies["first"]),
                                 _ptr(bodies["member"]), _ptr(bodies["offset"]), _ptr(bodies["inertia"]),
                                 _ptr(theta), _ptr(omega), N, bx, ctypes.byref(cfg), int(step), int(half),
                                 _ptr(status), _stream(stream)), ctx.handle)


def rc_compute_forces(ctx: Context, pos, nlist, nn, bx, force, ev=None, flags=0, status=None, stream=None):
    N = pos.shape[0]
    check(L.load().rc_compute_forces(ctx.handle, _ptr(pos), _ptr(nlist), _ptr(nn), _kmax(nlist, N), N, bx,
                                     _ptr(force),
                                     _ptr(ev), int(flags), _ptr(status), _stream(stream)), ctx.handle)


def rc_compute_forces_noalloc(ctx: Context, pos, nlist, nn, bx, force, ev=None, flags=0, status=None, stream=None):
    N = pos.shape[0]
    check(L.load().rc_compute_forces_noalloc(ctx.handle, _ptr(pos), _ptr(nlist), _ptr(nn), _kmax(nlist, N), N, bx,
                                             _ptr(force), _ptr(ev), int(flags), _ptr(status), _stream(stream)),
          ctx.handle)


def rc_workspace_bytes(ctx: "Context", N, k_max, nvec=1) -> int:
    out = ctypes.c_size_t()
    check(L.load().rc_workspace_bytes(ctx.handle, int(N), int(k_max), int(nvec), ctypes.byref(out)), ctx.handle)
    return int(out.value)


def rc_set_workspace(ctx: "Context", ws: Optional[torch.Tensor], N=0, k_max=0, nvec=0):
    """Attach a caller-owned device workspace (a uint8 tensor of rc_workspace_bytes) or detach (None)."""
    nbytes = 0 if ws is None else ws.numel() * ws.element_size()
    check(L.load().rc_set_workspace(ctx.handle, _ptr(ws), nbytes, int(N), int(k_max), int(nvec)), ctx.handle)


def rc_ctx_device_bytes(ctx: "Context") -> int:
    out = ctypes.c_size_t()
    check(L.load().rc_ctx_device_bytes(ctx.handle, ctypes.byref(out)), ctx.handle)
    return int(out.value)


def rc_batch_workspace_bytes(bc: "BatchContext", k_max) -> int:
    out = ctypes.c_size_t()
    check(L.load().rc_batch_workspace_bytes(bc.handle, int(k_max), ctypes.byref(out)), batch=bc.handle)
    return int(out.value)


def rc_batch_set_workspace(bc: "BatchContext", ws: Optional[torch.Tensor], k_max=0):
    nbytes = 0 if ws is None else ws.numel() * ws.element_size()
    check(L.load().rc_batch_set_workspace(bc.handle, _ptr(ws), nbytes, int(k_max)), batch=bc.handle)


def rc_thermostat_normals(seed, step0, steps, N, dim=3, device="cuda", stream=None) -> torch.Tensor:
    """(steps, N, 4) float32 device tensor: the integrators' thermostat normals of tags 0..N-1 at steps
    step0 .. step0 + steps - 1 (w = 0)."""
    out = torch.empty((int(steps), int(N), 4), dtype=torch.float32, device=device)
    code = L.load().rc_thermostat_normals(int(seed), int(step0), int(steps), int(N), int(dim), _ptr(out),
                                          _stream(stream))
    if code != L.RC_OK:
        raise RcError(code, "rc_thermostat_normals")
    return out


def rc_integrate_step(ctx: Context, pos, vel, force, image, bx, cfg, step, half, kin=None, status=None,
                      stream=None):
    N = pos.shape[0]
    check(L.load().rc_integrate_step(ctx.handle, _ptr(pos), _ptr(vel), _ptr(force), _ptr(image), N, bx,
                                     ctypes.byref(cfg), int(step), int(half), _ptr(kin), _ptr(status),
                                     _stream(stream)), ctx.handle)


def rc_step_fused(ctx: Context, pos_in, pos_out, vel, image, nlist, nn, bx, cfg, step, mode,
                  soft_frac=0.8, ev=None, status=None, stream=None):
    N = pos_in.shape[0]
    check(L.load().rc_step_fused(ctx.handle, _ptr(pos_in), _ptr(pos_out), _ptr(vel), _ptr(image),
                                 _ptr(nlist), _ptr(nn), _kmax(nlist, N), N, bx, ctypes.byref(cfg), int(step), int(mode),
                                 float(soft_frac), _ptr(ev), _ptr(status), _stream(stream)), ctx.handle)


def rc_bond_count(ctx: Context, pos, nlist, nn, bx, count, stream=None):
    N = pos.shape[0]
    check(L.load().rc_bond_count(ctx.handle, _ptr(pos), _ptr(nlist), _ptr(nn), _kmax(nlist, N), N, bx, _ptr(count),
                                 _stream(stream)), ctx.handle)


def rc_md_run(ctx: Context, bufs: L.MdBuffers, N, bx, cfg, step0, n_steps, opts: Optional[L.MdOptions] = None,
              stream=None) -> L.MdStats:
    st = L.MdStats()
    code = L.load().rc_md_run(ctx.handle, ctypes.byref(bufs), int(N), bx, ctypes.byref(cfg), int(step0),
                              int(n_steps), ctypes.byref(opts) if opts is not None else None,
                              ctypes.byref(st), _stream(stream))
    if code != L.RC_OK:
        err = RcError(code, L.load().rc_last_error(ctx.handle).decode())
        err.stats = st
        raise err
    return st


def rc_time_fused_steps(ctx: Context, pos_a, pos_b, vel, nlist, nn, bx, cfg, step0, reps, status,
                        stream=None) -> float:
    """Milliseconds for `reps` back-to-back fused step launches (HIP events)."""
    ms = ctypes.c_float()
    N = pos_a.shape[0]
    check(L.load().rc_time_fused_steps(ctx.handle, _ptr(pos_a), _ptr(pos_b), _ptr(vel), _ptr(nlist), _ptr(nn),
                                       _kmax(nlist, N), N, bx, ctypes.byref(cfg), int(step0), int(reps), _ptr(status),
                                       ctypes.byref(ms), _stream(stream)), ctx.handle)
    return float(ms.value)


def rc_force_hvp(ctx: Context, pos, nlist, nn, bx, v, hv, stream=None):
    N = pos.shape[0]
    check(L.load().rc_force_hvp(ctx.handle, _ptr(pos), _ptr(nlist), _ptr(nn), _kmax(nlist, N), N, bx, _ptr(v),
                                _ptr(hv),
                                _stream(stream)), ctx.handle)


def rc_force_hvp_batch(ctx: Context, pos, nlist, nn, bx, v, hv, stream=None):
    """hv[k] = H v[k] for v, hv of shape (nvec, N, 4), in one launch per pass."""
    N = pos.shape[0]
    if v.dim() != 3 or v.shape[1] != N or v.shape[2] != 4 or hv.shape != v.shape:
        raise ValueError("v and hv must be (nvec, N, 4)")
    check(L.load().rc_force_hvp_batch(ctx.handle, _ptr(pos), _ptr(nlist), _ptr(nn), _kmax(nlist, N), N, bx,
                                      int(v.shape[0]), _ptr(v), _ptr(hv), _stream(stream)), ctx.handle)


def rc_partner_counts(ctx: Context, p0, pt, select, counts, stream=None):
    """counts (3,) int64 device <- (bonded at 0, unchanged, swapped) over the selected tags."""
    N = p0.shape[0]
    if pt.shape[0] != N or (select is not None and select.shape[0] != N) or counts.numel() < 3:
        raise ValueError("p0, pt (and select) must have N entries, counts at least 3")
    check(L.load().rc_partner_counts(ctx.handle, _ptr(p0), _ptr(pt), _ptr(select), N, _ptr(counts),
                                     _stream(stream)), ctx.handle)


def rc_stress_autocorrelation(ctx: Context, rows, volume, kT, max_lag, G, stream=None):
    """G (max_lag + 1,) float64 device <- stress autocorrelation of logged rows (T, 13) float64 device."""
    if rows.dim() != 2 or rows.shape[1] != 13 or G.numel() < max_lag + 1:
        raise ValueError("rows must be (T, 13), G at least max_lag + 1 long")
    check(L.load().rc_stress_autocorrelation(ctx.handle, _ptr(rows), int(rows.shape[0]), float(volume), float(kT),
                                             int(max_lag), _ptr(G), _stream(stream)), ctx.handle)


def rc_param_vjp(ctx: Context, pos, nlist, nn, bx, adj, out, stream=None):
    N = pos.shape[0]
    check(L.load().rc_param_vjp(ctx.handle, _ptr(pos), _ptr(nlist), _ptr(nn), _kmax(nlist, N), N, bx, _ptr(adj),
                                _ptr(out), _stream(stream)), ctx.handle)


def rc_soft_bonds(ctx: Context, pos, nlist, nn, bx, value, grad=None, stream=None):
    N = pos.shape[0]
    check(L.load().rc_soft_bonds(ctx.handle, _ptr(pos), _ptr(nlist), _ptr(nn), _kmax(nlist, N), N, bx, _ptr(value),
                                 _ptr(grad), _stream(stream)), ctx.handle)


def rc_bond_partners(ctx: Context, pos, nlist, nn, bx, partner, stream=None):
    """partner: (N,) int32 device tensor, by tag: the bonded partner's tag, -1 none, -2 several."""
    N = pos.shape[0]
    check(L.load().rc_bond_partners(ctx.handle, _ptr(pos), _ptr(nlist), _ptr(nn), _kmax(nlist, N), N, bx,
                                    _ptr(partner), _stream(stream)), ctx.handle)


def rc_set_bonds(ctx: Context, bonds, rtag, K: float, R0: float):
    """bonds: (N, 2) int32 device tensor of partner tags (-1 none); rtag: the tag -> index map."""
    if bonds is None:
        check(L.load().rc_set_bonds(ctx.handle, None, None, 0, 0.0, 0.0), ctx.handle)
        return
    check(L.load().rc_set_bonds(ctx.handle, _ptr(bonds), _ptr(rtag), int(bonds.shape[0]), float(K), float(R0)),
          ctx.handle)


def rc_fene_forces(ctx: Context, pos, bx, force, ev=None, stream=None):
    N = pos.shape[0]
    check(L.load().rc_fene_forces(ctx.handle, _ptr(pos), N, bx, _ptr(force), _ptr(ev), _stream(stream)), ctx.handle)


def rc_param_grad(ctx: Context, pos, nlist, nn, bx, grad, stream=None):
    N = pos.shape[0]
    check(L.load().rc_param_grad(ctx.handle, _ptr(pos), _ptr(nlist), _ptr(nn), _kmax(nlist, N), N, bx,
                                 _ptr(grad),
                                 _stream(stream)), ctx.handle)


# ---------------------------------------------------------------------------
# batches
# ---------------------------------------------------------------------------

class BatchContext:
    """An rc_batch: R replicas with their own tables, particle counts and boxes."""

    def __init__(self, tables, counts, boxes, r_buff: float = 0.3):
        lib = L.load()
        R = len(tables)
        if not (len(counts) == R and len(boxes) == R and R > 0):
            raise ValueError("tables, counts and boxes need one entry per replica")
        nt = int(np.asarray(tables[0].kind).shape[0])
        arr = (L.PairCoeff * (R * nt * nt))()
        for r, t in enumerate(tables):
            if np.asarray(t.kind).shape[0] != nt:
                raise ValueError("every replica's table must have the same number of types")
            _fill_table(arr, r * nt * nt, t, nt)
        cnt = (ctypes.c_int * R)(*[int(c) for c in counts])
        bxs = (L.Box * R)()
        for r, b in enumerate(boxes):
            bxs[r] = b if isinstance(b, L.Box) else box(b)
        h = ctypes.c_void_p()
        code = lib.rc_batch_create(ctypes.byref(h), R, nt, arr, cnt, bxs, float(r_buff))
        if code != L.RC_OK:
            raise RcError(code, "rc_batch_create rejected the replicas")
        self.handle = h
        self.R = R
        self.ntypes = nt
        self.r_buff = float(r_buff)
        n = ctypes.c_int()
        offs = (ctypes.c_int * (R + 1))()
        check(lib.rc_batch_layout(h, ctypes.byref(n), offs), batch=h)
        self.n_slots = int(n.value)
        self.offsets = np.array(list(offs), dtype=np.int64)
        self.counts = np.array([int(c) for c in counts], dtype=np.int64)

    def set_seeds(self, seeds):
        arr = (ctypes.c_uint64 * self.R)(*[int(x) for x in seeds])
        check(L.load().rc_batch_set_seeds(self.handle, arr), batch=self.handle)

    def set_gather_width(self, width: int):
        check(L.load().rc_batch_set_gather_width(self.handle, int(width)), batch=self.handle)

    def set_step_form(self, form: str):
        f = {"walk": L.RC_FORM_WALK, "sums": L.RC_FORM_SUMS}[form]
        check(L.load().rc_batch_set_step_form(self.handle, f), batch=self.handle)

    def set_rebuild_margin(self, margin: float):
        check(L.load().rc_batch_set_rebuild_margin(self.handle, float(margin)), batch=self.handle)

    def close(self):
        if getattr(self, "handle", None):
            L.load().rc_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def rc_batch_cells_workspace_bytes(bc: BatchContext) -> int:
    out = ctypes.c_size_t()
    check(L.load().rc_batch_cells_workspace_bytes(bc.handle, ctypes.byref(out)), batch=bc.handle)
    return int(out.value)


def rc_batch_build_cells(bc: BatchContext, pos, vel, image, rtag, ws, stream=None):
    check(L.load().rc_batch_build_cells(bc.handle, _ptr(pos), _ptr(vel), _ptr(image), _ptr(rtag), _ptr(ws),
                                        ws.numel() * ws.element_size(), _stream(stream)), batch=bc.handle)


def rc_batch_build_nlist(bc: BatchContext, pos, vel, ws, k_max, nlist, nn, status=None, stream=None):
    check(L.load().rc_batch_build_nlist(bc.handle, _ptr(pos), _ptr(vel), _ptr(ws), ws.numel() * ws.element_size(),
                                        int(k_max), _ptr(nlist), _ptr(nn), _ptr(status), _stream(stream)),
          batch=bc.handle)


def rc_batch_compute_forces(bc: BatchContext, pos, nlist, nn, force, ev=None, status=None, stream=None):
    check(L.load().rc_batch_compute_forces(bc.handle, _ptr(pos), _ptr(nlist), _ptr(nn), _kmax(nlist, bc.n_slots),
                                           _ptr(force), _ptr(ev), _ptr(status), _stream(stream)), batch=bc.handle)


def rc_batch_bond_count(bc: BatchContext, pos, nlist, nn, counts, stream=None):
    check(L.load().rc_batch_bond_count(bc.handle, _ptr(pos), _ptr(nlist), _ptr(nn), _kmax(nlist, bc.n_slots),
                                       _ptr(counts), _stream(stream)), batch=bc.handle)


def rc_batch_step_fused(bc: BatchContext, pos_in, pos_out, vel, image, nlist, nn, cfg, step, mode, soft_frac=0.8,
                        ev=None, status=None, stream=None):
    check(L.load().rc_batch_step_fused(bc.handle, _ptr(pos_in), _ptr(pos_out), _ptr(vel), _ptr(image), _ptr(nlist),
                                       _ptr(nn), _kmax(nlist, bc.n_slots), ctypes.byref(cfg), int(step), int(mode),
                                       float(soft_frac), _ptr(ev), _ptr(status), _stream(stream)), batch=bc.handle)


def rc_batch_run(bc: BatchContext, bufs: L.MdBuffers, cfg, step0, n_steps, opts: Optional[L.MdOptions] = None,
                 stream=None) -> L.MdStats:
    st = L.MdStats()
    code = L.load().rc_batch_run(bc.handle, ctypes.byref(bufs), ctypes.byref(cfg), int(step0), int(n_steps),
                                 ctypes.byref(opts) if opts is not None else None, ctypes.byref(st), _stream(stream))
    if code != L.RC_OK:
        err = RcError(code, L.load().rc_batch_last_error(bc.handle).decode())
        err.stats = st
        raise err
    return st


def rc_batch_relayout_lists(bc: BatchContext, old_nlist, k_old, new_nlist, k_new, nn, stream=None):
    check(L.load().rc_batch_relayout_lists(bc.handle, _ptr(old_nlist), int(k_old), _ptr(new_nlist), int(k_new),
                                           _ptr(nn), _stream(stream)), batch=bc.handle)


def rc_batch_time_fused_steps(bc: BatchContext, pos_a, pos_b, vel, nlist, nn, cfg, step0, reps, status,
                              stream=None) -> float:
    """Milliseconds for `reps` back-to-back batch step launches (HIP events)."""
    ms = ctypes.c_float()
    check(L.load().rc_batch_time_fused_steps(bc.handle, _ptr(pos_a), _ptr(pos_b), _ptr(vel), _ptr(nlist), _ptr(nn),
                                             _kmax(nlist, bc.n_slots), ctypes.byref(cfg), int(step0), int(reps),
                                             _ptr(status), ctypes.byref(ms), _stream(stream)), batch=bc.handle)
    return float(ms.value)
