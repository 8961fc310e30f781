"""ctypes view of ``librc.so`` (the C ABI declared in ``include/rc.h``).

Argument marshalling only: every computation runs in the HIP library.  The
library must be built (``paper_1912_08569_amd.build.build()``); there is no
fallback path.
"""
from __future__ import annotations

import ctypes
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
# RC_LIBRARY selects another build of the same ABI (default: the in-tree librc.so)
LIB_PATH = os.environ.get("RC_LIBRARY") or os.path.join(HERE, "librc.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "rc.h")

RC_OK = 0
RC_ERR_ARG = -1
RC_ERR_HIP = -2
RC_ERR_NLIST_OVERFLOW = -3
RC_ERR_UNSUPPORTED = -4
RC_ERR_NONFINITE = -5
RC_ERR_LOST_PARTICLE = -6
RC_ERR_WORKSPACE = -7

RC_KIND_NONE, RC_KIND_SWAP, RC_KIND_WCA = 0, 1, 2
RC_TYPE_BITS = 4
RC_MAX_TYPES = 16
RC_STATUS_WORDS = 8
RC_ST_NSWAP = 5
RC_NOALLOC_MAX_N = 1048576
RC_ST_FLAGS, RC_ST_KMAX, RC_ST_MAXPATH, RC_ST_FIRST_SOFT, RC_ST_FIRST_HARD = 0, 1, 2, 3, 4
RC_FLAG_NLIST_OVERFLOW, RC_FLAG_REBUILD, RC_FLAG_NONFINITE, RC_FLAG_LOST, RC_FLAG_STALE = 1, 2, 4, 8, 16
RC_FORCE_ACCUMULATE, RC_FORCE_GATHER, RC_FORCE_SUMS = 1, 4, 8
RC_FORM_WALK, RC_FORM_SUMS = 0, 1
RC_HALF_FIRST, RC_HALF_SECOND = 0, 1
RC_STEP_START, RC_STEP_CONT, RC_STEP_FINISH, RC_STEP_OBSERVE = 0, 1, 2, 3
RC_INTEGRATOR_NVE, RC_INTEGRATOR_LANGEVIN = 0, 1

_ERR_NAMES = {
    RC_ERR_ARG: "invalid argument", RC_ERR_HIP: "HIP runtime error",
    RC_ERR_NLIST_OVERFLOW: "neighbour list overflow", RC_ERR_UNSUPPORTED: "unsupported",
    RC_ERR_NONFINITE: "non-finite values", RC_ERR_LOST_PARTICLE: "lost particle",
    RC_ERR_WORKSPACE: "workspace too small",
}


class RcError(RuntimeError):
    def __init__(self, code: int, msg: str = ""):
        super().__init__(f"{_ERR_NAMES.get(code, 'error')} ({code}): {msg}")
        self.code = code


class PairCoeff(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("n", ctypes.c_int), ("epsilon", ctypes.c_double),
                ("sigma", ctypes.c_double), ("r_cut", ctypes.c_double), ("lam", ctypes.c_double)]


class Box(ctypes.Structure):
    _fields_ = [("L", ctypes.c_double * 3)]


class Integrator(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("dim", ctypes.c_int), ("dt", ctypes.c_double),
                ("kT", ctypes.c_double), ("gamma", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("mass", ctypes.c_double * RC_MAX_TYPES)]


class MdBuffers(ctypes.Structure):
    _fields_ = [("pos", ctypes.c_void_p), ("pos_alt", ctypes.c_void_p), ("vel", ctypes.c_void_p),
                ("image", ctypes.c_void_p), ("rtag", ctypes.c_void_p), ("nlist", ctypes.c_void_p),
                ("nn", ctypes.c_void_p), ("k_max", ctypes.c_int), ("pad", ctypes.c_int),
                ("cells_ws", ctypes.c_void_p), ("cells_ws_bytes", ctypes.c_size_t),
                ("snap_pos", ctypes.c_void_p), ("snap_vel", ctypes.c_void_p),
                ("snap_image", ctypes.c_void_p), ("status", ctypes.c_void_p),
                ("ev_log", ctypes.c_void_p), ("bonds_log", ctypes.c_void_p)]


class MdOptions(ctypes.Structure):
    _fields_ = [("use_graph", ctypes.c_int), ("graph_steps", ctypes.c_int),
                ("max_chunk", ctypes.c_int), ("log_period", ctypes.c_int),
                ("soft_frac", ctypes.c_double), ("adapt", ctypes.c_int), ("one_block", ctypes.c_int),
                ("resume", ctypes.c_int), ("keep_list", ctypes.c_int), ("time_kernels", ctypes.c_int)]


class MdStats(ctypes.Structure):
    _fields_ = [("steps_done", ctypes.c_int64), ("rebuilds", ctypes.c_int64),
                ("rollbacks", ctypes.c_int64), ("chunks", ctypes.c_int64),
                ("log_rows", ctypes.c_int64), ("k_needed", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("kernel_launches", ctypes.c_int64), ("kernel_ms", ctypes.c_double),
                ("sums_ms", ctypes.c_double), ("list_kept", ctypes.c_int32), ("nswap", ctypes.c_int32),
                ("particles_rebuilt", ctypes.c_int64)]


_VP = ctypes.c_void_p
_I = ctypes.c_int
_U = ctypes.c_uint
_U64 = ctypes.c_uint64
_D = ctypes.c_double

_SIGS = {
    "rc_version": ([], _I),
    "rc_create": ([ctypes.POINTER(_VP), _I, ctypes.POINTER(PairCoeff), _D], _I),
    "rc_destroy": ([_VP], _I),
    "rc_last_error": ([_VP], ctypes.c_char_p),
    "rc_set_lambda": ([_VP, ctypes.POINTER(_D)], _I),
    "rc_get_rlist": ([_VP, _I, _I, ctypes.POINTER(_D)], _I),
    "rc_set_gather_width": ([_VP, _I], _I),
    "rc_set_step_form": ([_VP, _I], _I),
    "rc_clear_status": ([_VP, _VP], _I),
    "rc_read_status": ([_VP, ctypes.POINTER(_I), _VP], _I),
    "rc_cells_workspace_bytes": ([_VP, _I, Box, ctypes.POINTER(ctypes.c_size_t)], _I),
    "rc_build_cells": ([_VP, _VP, _VP, _VP, _VP, _I, Box, _VP, ctypes.c_size_t, _VP], _I),
    "rc_build_nlist": ([_VP, _VP, _VP, _I, Box, _VP, ctypes.c_size_t, _I, _VP, _VP, _VP, _VP], _I),
    "rc_compute_forces": ([_VP, _VP, _VP, _VP, _I, _I, Box, _VP, _VP, _U, _VP, _VP], _I),
    "rc_thermostat_normals": ([_U64, _U64, _I, _I, _I, _VP, _VP], _I),
    "rc_workspace_bytes": ([_VP, _I, _I, _I, ctypes.POINTER(ctypes.c_size_t)], _I),
    "rc_set_workspace": ([_VP, _VP, ctypes.c_size_t, _I, _I, _I], _I),
    "rc_ctx_device_bytes": ([_VP, ctypes.POINTER(ctypes.c_size_t)], _I),
    "rc_batch_workspace_bytes": ([_VP, _I, ctypes.POINTER(ctypes.c_size_t)], _I),
    "rc_batch_set_workspace": ([_VP, _VP, ctypes.c_size_t, _I], _I),
    "rc_compute_forces_noalloc": ([_VP, _VP, _VP, _VP, _I, _I, Box, _VP, _VP, _U, _VP, _VP], _I),
    "rc_integrate_step": ([_VP, _VP, _VP, _VP, _VP, _I, Box, ctypes.POINTER(Integrator), _U64, _I,
                           _VP, _VP, _VP], _I),
    "rc_step_fused": ([_VP, _VP, _VP, _VP, _VP, _VP, _VP, _I, _I, Box, ctypes.POINTER(Integrator), _U64,
                       _I, _D, _VP, _VP, _VP], _I),
    "rc_bond_count": ([_VP, _VP, _VP, _VP, _I, _I, Box, _VP, _VP], _I),
    "rc_time_fused_steps": ([_VP, _VP, _VP, _VP, _VP, _VP, _I, _I, Box, ctypes.POINTER(Integrator), _U64, _I,
                             _VP, ctypes.POINTER(ctypes.c_float), _VP], _I),
    "rc_md_run": ([_VP, ctypes.POINTER(MdBuffers), _I, Box, ctypes.POINTER(Integrator), _U64, _I,
                   ctypes.POINTER(MdOptions), ctypes.POINTER(MdStats), _VP], _I),
    "rc_force_hvp": ([_VP, _VP, _VP, _VP, _I, _I, Box, _VP, _VP, _VP], _I),
    "rc_force_hvp_batch": ([_VP, _VP, _VP, _VP, _I, _I, Box, _I, _VP, _VP, _VP], _I),
    "rc_partner_counts": ([_VP, _VP, _VP, _VP, _I, _VP, _VP], _I),
    "rc_rigid_step": ([_VP, _VP, _VP, _VP, _VP, _VP, _I, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _I, Box,
                       ctypes.POINTER(Integrator), _U64, _I, _VP, _VP], _I),
    "rc_stress_autocorrelation": ([_VP, _VP, _I, ctypes.c_double, ctypes.c_double, _I, _VP, _VP], _I),
    "rc_param_grad": ([_VP, _VP, _VP, _VP, _I, _I, Box, _VP, _VP], _I),
    "rc_param_vjp": ([_VP, _VP, _VP, _VP, _I, _I, Box, _VP, _VP, _VP], _I),
    "rc_set_table": ([_VP, ctypes.POINTER(PairCoeff)], _I),
    "rc_soft_bonds": ([_VP, _VP, _VP, _VP, _I, _I, Box, _VP, _VP, _VP], _I),
    "rc_set_bonds": ([_VP, _VP, _VP, _I, _D, _D], _I),
    "rc_bond_partners": ([_VP, _VP, _VP, _VP, _I, _I, Box, _VP, _VP], _I),
    "rc_fene_forces": ([_VP, _VP, _I, Box, _VP, _VP, _VP], _I),
    # batches
    "rc_batch_create": ([ctypes.POINTER(_VP), _I, _I, ctypes.POINTER(PairCoeff), ctypes.POINTER(_I),
                         ctypes.POINTER(Box), _D], _I),
    "rc_batch_destroy": ([_VP], _I),
    "rc_batch_last_error": ([_VP], ctypes.c_char_p),
    "rc_batch_layout": ([_VP, ctypes.POINTER(_I), ctypes.POINTER(_I)], _I),
    "rc_batch_set_seeds": ([_VP, ctypes.POINTER(_U64)], _I),
    "rc_batch_set_gather_width": ([_VP, _I], _I),
    "rc_batch_set_step_form": ([_VP, _I], _I),
    "rc_batch_cells_workspace_bytes": ([_VP, ctypes.POINTER(ctypes.c_size_t)], _I),
    "rc_batch_build_cells": ([_VP, _VP, _VP, _VP, _VP, _VP, ctypes.c_size_t, _VP], _I),
    "rc_batch_build_nlist": ([_VP, _VP, _VP, _VP, ctypes.c_size_t, _I, _VP, _VP, _VP, _VP], _I),
    "rc_batch_compute_forces": ([_VP, _VP, _VP, _VP, _I, _VP, _VP, _VP, _VP], _I),
    "rc_batch_bond_count": ([_VP, _VP, _VP, _VP, _I, _VP, _VP], _I),
    "rc_batch_step_fused": ([_VP, _VP, _VP, _VP, _VP, _VP, _VP, _I, ctypes.POINTER(Integrator), _U64, _I, _D,
                             _VP, _VP, _VP], _I),
    "rc_batch_run": ([_VP, ctypes.POINTER(MdBuffers), ctypes.POINTER(Integrator), _U64, _I,
                      ctypes.POINTER(MdOptions), ctypes.POINTER(MdStats), _VP], _I),
    "rc_batch_time_fused_steps": ([_VP, _VP, _VP, _VP, _VP, _VP, _I, ctypes.POINTER(Integrator), _U64, _I, _VP,
                                   ctypes.POINTER(ctypes.c_float), _VP], _I),
    "rc_batch_set_rebuild_margin": ([_VP, _D], _I),
    "rc_batch_relayout_lists": ([_VP, _VP, _I, _VP, _I, _VP, _VP], _I),
}

_lib = None


def declared_symbols():
    """Names of every function declared in include/rc.h."""
    with open(HEADER) as f:
        text = f.read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?(?:int|char\s*\*|const char\s*\*)\s*(rc_\w+)\s*\(",
                                 text, flags=re.M)))


def load():
    """Load librc.so; raises if it has not been built.

    torch is imported first: its wheel carries its own HIP and HSA runtimes,
    and librc.so must bind to those (the ones that own the device memory it
    is handed).  Loaded before torch, librc.so would map the system ROCm
    runtime, and torch would then map its own beside it: two HIP runtimes in
    one process, which can fail to bring up the device."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build the HIP engine first "
                           "(python -m paper_1912_08569_amd.build)")
    import torch  # noqa: F401  (its HIP runtime first)
    lib = ctypes.CDLL(LIB_PATH)
    for name, (args, res) in _SIGS.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def check(code: int, ctx=None, batch=None):
    if code != RC_OK:
        msg = ""
        if ctx is not None:
            raw = load().rc_last_error(ctx)
            msg = raw.decode() if raw else ""
        elif batch is not None:
            raw = load().rc_batch_last_error(batch)
            msg = raw.decode() if raw else ""
        raise RcError(code, msg)
