"""Literal triple-loop energy of the swap potential, for a handful of particles.

TEST INFRASTRUCTURE ONLY.  Written independently of ``swap_ref`` with the
``math`` module and plain Python loops, straight from the paper's sums:

    E = sum_{i<j} phi(r_ij)                                   (Sec. 2, eq. 2b)
      + sum_i sum_{j<k; j,k != i} lambda eps vhat(r_ij) vhat(r_ik)   (eq. 3bp, eq. pot)

Only for N <= ~30 (O(N^3)).  Parity status: pinned by closed forms (dimer,
symmetric and collinear triplets, flat swap barrier) in the tests.
"""
from __future__ import annotations

import math

KIND_NONE, KIND_SWAP, KIND_WCA = 0, 1, 2


def _sep(xi, xj, L):
    out = []
    for a in range(3):
        d = float(xj[a]) - float(xi[a])
        if d > 0.5 * L[a]:
            d -= L[a]
        elif d < -0.5 * L[a]:
            d += L[a]
        out.append(d)
    return out


def _r2(d):
    return (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]


def _phi(kind, r, eps, sigma, n):
    if kind == KIND_SWAP:
        q = (sigma / r) ** n
        return 4.0 * eps * (q * q - q)
    if kind == KIND_WCA:
        q = (sigma / r) ** 6
        return 4.0 * eps * (q * q - q) + eps
    return 0.0


def _vhat(r2, eps, sigma, n, rcut):
    if r2 >= rcut * rcut:
        return 0.0
    if r2 <= (sigma * sigma) * math.pow(2.0, 2.0 / n):
        return 1.0
    r = math.sqrt(r2)
    q = (sigma / r) ** n
    return -(4.0 * eps * (q * q - q)) / eps


def literal_energy(pos, types, L, table):
    """Return (E2, E3) by explicit loops over i<j and over i, j<k."""
    N = len(pos)
    Lv = [float(L)] * 3 if not hasattr(L, "__len__") else [float(x) for x in L]
    E2 = 0.0
    for i in range(N):
        for j in range(i + 1, N):
            a, b = int(types[i]), int(types[j])
            kind = int(table.kind[a, b])
            if kind == KIND_NONE:
                continue
            d = _sep(pos[i], pos[j], Lv)
            r2 = _r2(d)
            rc = float(table.rcut[a, b])
            if r2 < rc * rc:
                E2 += _phi(kind, math.sqrt(r2), float(table.epsilon[a, b]),
                           float(table.sigma[a, b]), int(table.n[a, b]))
    E3 = 0.0
    for i in range(N):
        for j in range(N):
            for k in range(j + 1, N):
                if j == i or k == i:
                    continue
                ti, tj, tk = int(types[i]), int(types[j]), int(types[k])
                if table.kind[ti, tj] != KIND_SWAP or table.kind[ti, tk] != KIND_SWAP:
                    continue
                dij = _sep(pos[i], pos[j], Lv)
                dik = _sep(pos[i], pos[k], Lv)
                uj = _vhat(_r2(dij), float(table.epsilon[ti, tj]), float(table.sigma[ti, tj]),
                           int(table.n[ti, tj]), float(table.rcut[ti, tj]))
                uk = _vhat(_r2(dik), float(table.epsilon[ti, tk]), float(table.sigma[ti, tk]),
                           int(table.n[ti, tk]), float(table.rcut[ti, tk]))
                Lj = float(table.lam[ti, tj]) * float(table.epsilon[ti, tj])
                Lk = float(table.lam[ti, tk]) * float(table.epsilon[ti, tk])
                Lam = Lj if Lj == Lk else math.sqrt(Lj * Lk)
                E3 += Lam * uj * uk
    return E2, E3
