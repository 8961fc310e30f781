"""ctypes front end of the C brute-force oracle (``brute.c``).

TEST INFRASTRUCTURE ONLY.  ``build()`` compiles ``brute.c`` with gcc into
``oracle/_brute.so`` (``-O2 -fopenmp -ffp-contract=off``).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "brute.c")
_LIB = os.path.join(_HERE, "_brute.so")
_lib = None


def build(force: bool = True) -> str:
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
                               "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        _lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        lp = ctypes.POINTER(ctypes.c_longlong)
        _lib.orc_evaluate.argtypes = [ctypes.c_int, dp, ip, dp, ctypes.c_int, ip, dp, dp, ip, dp,
                                      dp, ctypes.c_int, dp, dp, dp, lp, lp]
        _lib.orc_evaluate.restype = ctypes.c_int
        _lib.orc_forces_subset.argtypes = [ctypes.c_int, dp, ip, dp, ctypes.c_int, ip, dp, dp, ip,
                                           dp, dp, ctypes.c_int, ctypes.c_int, ip, dp, dp, ip]
        _lib.orc_forces_subset.restype = ctypes.c_int
    return _lib


def _p(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def _table_arrays(table):
    nt = table.kind.shape[0]
    return (nt,
            np.ascontiguousarray(table.kind, dtype=np.int32).ravel(),
            np.ascontiguousarray(table.epsilon, dtype=np.float64).ravel(),
            np.ascontiguousarray(table.sigma, dtype=np.float64).ravel(),
            np.ascontiguousarray(table.n, dtype=np.int32).ravel(),
            np.ascontiguousarray(table.rcut, dtype=np.float64).ravel(),
            np.ascontiguousarray(table.lam, dtype=np.float64).ravel())


def evaluate(pos, types, L, table, nthreads: int = 0):
    """Full O(N^2) evaluation: dict(E, E2, E3, W[6], F[N,3], pe[N], bonds, n_triplets)."""
    lib = _load()
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    N = pos.shape[0]
    ty = np.ascontiguousarray(types, dtype=np.int32)
    Lv = np.ascontiguousarray(np.broadcast_to(np.asarray(L, dtype=np.float64), (3,)))
    nt, k, e, s, n, rc, lm = _table_arrays(table)
    F = np.zeros((N, 3))
    pe = np.zeros(N)
    out = np.zeros(9)
    bonds = ctypes.c_longlong(0)
    ntr = ctypes.c_longlong(0)
    rc_ = lib.orc_evaluate(N, _p(pos, ctypes.c_double), _p(ty, ctypes.c_int),
                           _p(Lv, ctypes.c_double), nt, _p(k, ctypes.c_int),
                           _p(e, ctypes.c_double), _p(s, ctypes.c_double), _p(n, ctypes.c_int),
                           _p(rc, ctypes.c_double), _p(lm, ctypes.c_double), int(nthreads),
                           _p(F, ctypes.c_double), _p(pe, ctypes.c_double),
                           _p(out, ctypes.c_double), ctypes.byref(bonds), ctypes.byref(ntr))
    if rc_ != 0:
        raise RuntimeError("brute-force oracle failed")
    return dict(E=out[0], E2=out[1], E3=out[2], W=out[3:9].copy(), F=F, pe=pe,
                bonds=int(bonds.value), n_triplets=int(ntr.value))


def forces_subset(pos, types, L, table, idx, nthreads: int = 0):
    """Forces, per-particle energies and bond degrees of the particles ``idx``."""
    lib = _load()
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    N = pos.shape[0]
    ty = np.ascontiguousarray(types, dtype=np.int32)
    Lv = np.ascontiguousarray(np.broadcast_to(np.asarray(L, dtype=np.float64), (3,)))
    nt, k, e, s, n, rc, lm = _table_arrays(table)
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    M = idx.shape[0]
    F = np.zeros((M, 3))
    pe = np.zeros(M)
    deg = np.zeros(M, np.int32)
    rc_ = lib.orc_forces_subset(N, _p(pos, ctypes.c_double), _p(ty, ctypes.c_int),
                                _p(Lv, ctypes.c_double), nt, _p(k, ctypes.c_int),
                                _p(e, ctypes.c_double), _p(s, ctypes.c_double),
                                _p(n, ctypes.c_int), _p(rc, ctypes.c_double),
                                _p(lm, ctypes.c_double), int(nthreads), M, _p(idx, ctypes.c_int),
                                _p(F, ctypes.c_double), _p(pe, ctypes.c_double),
                                _p(deg, ctypes.c_int))
    if rc_ != 0:
        raise RuntimeError("brute-force oracle subset failed")
    return dict(F=F, pe=pe, degree=deg)
