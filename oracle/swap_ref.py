"""FP64 numpy evaluator of the swap potential -- the oracle's definition.

TEST INFRASTRUCTURE ONLY (see the package docstring).  No blocking, fusion or
reordering beyond the definition: every pair term and every triplet term is
formed explicitly and summed.

Definition (paper, Sec. 2):

* pair term, kind SWAP: the generalized LJ of eq. (2b),
  v(r) = 4 eps [(sigma/r)^(2n) - (sigma/r)^n] for r < r_cut, zero beyond
  (truncated, not shifted: the paper states no shift).
* pair term, kind WCA: 4 eps [(sigma/r)^12 - (sigma/r)^6] + eps for r < r_cut
  (the repulsive inert species of Sec. 3.1 / 3.2).
* switching factor, eq. (pot): vhat(r) = 1 for r <= r_min = sigma 2^(1/n),
  -v(r)/eps for r_min < r < r_cut, 0 for r >= r_cut.
* three-body term, eq. (3bp): for every centre i and every unordered pair
  {j, k} of distinct partners of i (j, k != i, both swap pairs with i and
  inside r_cut): Lambda_ijk * vhat(r_ij) * vhat(r_ik), with Lambda = lambda*eps.
  When the (i,j) and (i,k) entries differ Lambda_ijk = sqrt(Lambda_ij Lambda_ik)
  (a reading: the paper gives one lambda per type pair; see the design notes).
* forces F = -grad E, analytic per term; configurational virial
  W_ab = sum over terms of sum_m (x_m - x_centre)_a F_m,b, i.e. for a pair
  (r_ij)_a (F_j)_b and for a triplet (r_ij)_a (F_j)_b + (r_ik)_a (F_k)_b --
  the two-body virial plus the triplet bracket of eq. (p3); the stress is
  sigma_ab = -(kinetic + W_ab)/V (sign convention of eq. p3).
* per-particle energy: half of every pair term to each particle, every
  triplet term to its centre (a reading; only totals are fixed by the paper).
* bond count: swap pairs i<j with r^2 < r_min^2 (the bond length of Sec. 2).

Cut and bond decisions use the *canonical FP64 predicate*: minimum image
dx = x_j - x_i, folded once by +-L; r^2 = (dx*dx + dy*dy) + dz*dz with no
fused multiply-add; compared with r_cut*r_cut and
r_min^2 = (sigma*sigma) * pow(2, 2/n).  Any implementation that follows these
IEEE operations reaches the same integer decisions.

Parity status: pinned (closed forms, finite differences of the energy, strain
derivatives, the flat swap barrier, literal triple loops).  The error scales
A_F, A_E, A_W and A_pe are pinned by the bounds they must satisfy, their
units (eps and length scaling) and their equality with the quantity itself
where one sub-term dominates (tests/test_oracle_scales.py).
"""
from __future__ import annotations

import math
from typing import Dict

import numpy as np
from scipy.spatial import cKDTree

KIND_NONE, KIND_SWAP, KIND_WCA = 0, 1, 2

# ----------------------------------------------------------------------------
# scalar / vectorized pair functions
# ----------------------------------------------------------------------------


def rmin(sigma, n):
    """Location of the minimum of eq. (2b): sigma * 2^(1/n)."""
    return sigma * 2.0 ** (1.0 / n)


def rmin2_canonical(sigma: float, n: int) -> float:
    """r_min^2 as the canonical double (sigma*sigma) * pow(2, 2/n)."""
    return (float(sigma) * float(sigma)) * math.pow(2.0, 2.0 / float(n))


def mie(r, eps, sigma, n):
    """Eq. (2b): 4 eps [(sigma/r)^(2n) - (sigma/r)^n]."""
    s = np.power(sigma / r, n)
    return 4.0 * eps * (s * s - s)


def mie_d1(r, eps, sigma, n):
    """d/dr of eq. (2b)."""
    s = np.power(sigma / r, n)
    return 4.0 * eps * n * (s - 2.0 * s * s) / r


def mie_d2(r, eps, sigma, n):
    """d^2/dr^2 of eq. (2b)."""
    s = np.power(sigma / r, n)
    return 4.0 * eps * (2.0 * n * (2.0 * n + 1.0) * s * s - n * (n + 1.0) * s) / (r * r)


def mie_dsigma(r, eps, sigma, n):
    """d/dsigma of eq. (2b) at fixed r."""
    s = np.power(sigma / r, n)
    return 4.0 * eps * n * (2.0 * s * s - s) / sigma


def pair_phi(kind, r, eps, sigma, n):
    """Pair energy and its first two r-derivatives (inside the cutoff)."""
    kind = np.asarray(kind)
    nn = np.where(kind == KIND_WCA, 6, n)
    phi = mie(r, eps, sigma, nn) + np.where(kind == KIND_WCA, eps, 0.0)
    d1 = mie_d1(r, eps, sigma, nn)
    d2 = mie_d2(r, eps, sigma, nn)
    return phi, d1, d2


def pair_scales(kind, r, eps, sigma, n):
    """Absolute-summed magnitudes of the energy and force sub-terms."""
    kind = np.asarray(kind)
    nn = np.where(kind == KIND_WCA, 6, n)
    s = np.power(sigma / r, nn)
    e_scale = 4.0 * eps * (s * s + s) + np.where(kind == KIND_WCA, eps, 0.0)
    f_scale = 4.0 * eps * nn * (2.0 * s * s + s) / r
    return e_scale, f_scale


def vhat_terms(r2, r, eps, sigma, n, rmin2):
    """Eq. (pot) inside the cutoff: u, u', u'' and magnitude scales of u, u'.

    u = 1 for r^2 <= r_min^2 (canonical), else -v/eps.
    """
    inside = r2 <= rmin2
    s = np.power(sigma / r, n)
    u_out = -4.0 * (s * s - s)
    d1_out = -4.0 * n * (s - 2.0 * s * s) / r
    d2_out = -4.0 * (2.0 * n * (2.0 * n + 1.0) * s * s - n * (n + 1.0) * s) / (r * r)
    u = np.where(inside, 1.0, u_out)
    d1 = np.where(inside, 0.0, d1_out)
    d2 = np.where(inside, 0.0, d2_out)
    us = np.where(inside, 1.0, 4.0 * (s * s + s))
    d1s = np.where(inside, 0.0, 4.0 * n * (2.0 * s * s + s) / r)
    return u, d1, d2, us, d1s


def vhat_scalar(r, eps, sigma, n, rcut):
    """Eq. (pot) for one distance (reals, r > 0); used by closed-form checks."""
    if r >= rcut:
        return 0.0
    if r <= rmin(sigma, n):
        return 1.0
    return -float(mie(r, eps, sigma, n)) / eps


# ----------------------------------------------------------------------------
# geometry
# ----------------------------------------------------------------------------


def min_image(xi: np.ndarray, xj: np.ndarray, L: np.ndarray) -> np.ndarray:
    """Canonical minimum-image separation x_j - x_i (FP64, one fold by +-L)."""
    d = xj - xi
    half = 0.5 * L
    d = np.where(d > half, d - L, np.where(d < -half, d + L, d))
    return d


def r2_canonical(d: np.ndarray) -> np.ndarray:
    """(dx*dx + dy*dy) + dz*dz, evaluated left to right (numpy never fuses)."""
    return (d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1]) + d[..., 2] * d[..., 2]


def candidate_pairs(pos64: np.ndarray, L: np.ndarray, rmax: float):
    """All unordered pairs (i<j) whose periodic distance may be below rmax.

    A superset: the exact decision is taken afterwards with the canonical
    predicate.  Small systems: every pair; larger: a periodic k-d tree query
    (library primitive) with a relative margin of 1e-9.
    """
    N = pos64.shape[0]
    if N < 2:
        return np.zeros(0, np.int64), np.zeros(0, np.int64)
    if N <= 2500 or rmax >= 0.45 * float(np.min(L)):
        i, j = np.triu_indices(N, k=1)
        return i.astype(np.int64), j.astype(np.int64)
    Lv = np.broadcast_to(np.asarray(L, dtype=np.float64), (3,))
    p = pos64 + 0.5 * Lv
    p = np.minimum(np.maximum(p, 0.0), np.nextafter(Lv, 0.0))
    tree = cKDTree(p, boxsize=Lv)   # periodic along each axis (orthorhombic boxes)
    pairs = tree.query_pairs(rmax * (1.0 + 1e-9) + 1e-12, output_type="ndarray")
    if pairs.size == 0:
        return np.zeros(0, np.int64), np.zeros(0, np.int64)
    i = np.minimum(pairs[:, 0], pairs[:, 1]).astype(np.int64)
    j = np.maximum(pairs[:, 0], pairs[:, 1]).astype(np.int64)
    return i, j


# ----------------------------------------------------------------------------
# table helpers
# ----------------------------------------------------------------------------


def _entry_arrays(table, ti, tj):
    kind = table.kind[ti, tj].astype(np.int64)
    eps = table.epsilon[ti, tj].astype(np.float64)
    sig = table.sigma[ti, tj].astype(np.float64)
    n = table.n[ti, tj].astype(np.float64)
    rc = table.rcut[ti, tj].astype(np.float64)
    lam = table.lam[ti, tj].astype(np.float64)
    return kind, eps, sig, n, rc, lam


def rmin2_table(table) -> np.ndarray:
    nt = table.kind.shape[0]
    out = np.zeros((nt, nt))
    for a in range(nt):
        for b in range(nt):
            out[a, b] = rmin2_canonical(table.sigma[a, b], int(table.n[a, b]))
    return out


# ----------------------------------------------------------------------------
# the evaluator
# ----------------------------------------------------------------------------


def interacting_pairs(pos, types, L, table):
    """Pairs i<j inside their cutoff, with the quantities every term needs."""
    pos64 = np.asarray(pos, dtype=np.float64)
    types = np.asarray(types, dtype=np.int64)
    Lv = np.broadcast_to(np.asarray(L, dtype=np.float64), (3,)).copy()
    active = table.kind != KIND_NONE
    rmax = float(np.max(np.where(active, table.rcut, 0.0))) if active.any() else 0.0
    i, j = candidate_pairs(pos64, Lv, rmax)
    d = min_image(pos64[i], pos64[j], Lv)
    r2 = r2_canonical(d)
    ti, tj = types[i], types[j]
    kind, eps, sig, n, rc, lam = _entry_arrays(table, ti, tj)
    keep = (kind != KIND_NONE) & (r2 < rc * rc)
    sel = np.nonzero(keep)[0]
    rm2 = rmin2_table(table)[ti[sel], tj[sel]]
    return dict(i=i[sel], j=j[sel], d=d[sel], r2=r2[sel], kind=kind[sel], eps=eps[sel],
                sigma=sig[sel], n=n[sel], rcut=rc[sel], lam=lam[sel], rmin2=rm2,
                N=pos64.shape[0], L=Lv)


def directed_swap_edges(P):
    """Both directions of every interacting swap pair, grouped by centre."""
    sw = np.nonzero(P["kind"] == KIND_SWAP)[0]
    i, j, d = P["i"][sw], P["j"][sw], P["d"][sw]
    r2 = P["r2"][sw]
    r = np.sqrt(r2)
    eps, sig, n, lam, rm2 = P["eps"][sw], P["sigma"][sw], P["n"][sw], P["lam"][sw], P["rmin2"][sw]
    u, u1, u2, us, u1s = vhat_terms(r2, r, eps, sig, n, rm2)
    Lam = lam * eps
    # centre, partner, vector centre->partner
    c = np.concatenate([i, j])
    p = np.concatenate([j, i])
    dv = np.concatenate([d, -d])
    rep = lambda a: np.concatenate([a, a])  # noqa: E731
    order = np.argsort(c, kind="stable")
    E = dict(c=c[order], p=p[order], d=dv[order], r=rep(r)[order], u=rep(u)[order],
             u1=rep(u1)[order], u2=rep(u2)[order], us=rep(us)[order], u1s=rep(u1s)[order],
             Lam=rep(Lam)[order], eps=rep(eps)[order], sigma=rep(sig)[order], n=rep(n)[order],
             lam=rep(lam)[order], r2=rep(r2)[order], rmin2=rep(rm2)[order],
             pair_index=rep(sw)[order])
    return E


def triplets(E, N):
    """Every (centre, a, b) with a < b indexing the directed edge arrays."""
    c = E["c"]
    counts = np.bincount(c, minlength=N) if c.size else np.zeros(N, np.int64)
    starts = np.concatenate([[0], np.cumsum(counts)])
    ea, eb = [], []
    for k in np.unique(counts[counts >= 2]):
        cen = np.nonzero(counts == k)[0]
        aa, bb = np.triu_indices(int(k), k=1)
        base = starts[cen][:, None]
        ea.append((base + aa[None, :]).ravel())
        eb.append((base + bb[None, :]).ravel())
    if not ea:
        return np.zeros(0, np.int64), np.zeros(0, np.int64)
    return np.concatenate(ea), np.concatenate(eb)


def triplet_lambda(E, a, b):
    La, Lb = E["Lam"][a], E["Lam"][b]
    return np.where(La == Lb, La, np.sqrt(La * Lb))


def evaluate(pos, types, L, table, scales: bool = True) -> Dict[str, np.ndarray]:
    """Energy, per-particle energy, forces, virial and bond count (FP64).

    Returns a dict with E, E2, E3, pe [N], F [N,3], W [6] ordered
    (xx, yy, zz, xy, xz, yz), bonds (int), n_triplets, and, if ``scales``,
    the error scales A_E, A_pe [N], A_F [N], A_W used by parity tolerances.
    """
    P = interacting_pairs(pos, types, L, table)
    N = P["N"]
    F = np.zeros((N, 3))
    pe = np.zeros(N)
    Wt = np.zeros((3, 3))
    A_pe = np.zeros(N)
    A_F = np.zeros(N)
    A_W = 0.0

    # ---- pair terms ---------------------------------------------------------
    i, j, d = P["i"], P["j"], P["d"]
    r = np.sqrt(P["r2"])
    phi, dphi, _ = pair_phi(P["kind"], r, P["eps"], P["sigma"], P["n"])
    rhat = d / r[:, None]
    Fj = -dphi[:, None] * rhat            # force on j from the pair term
    np.add.at(F, j, Fj)
    np.add.at(F, i, -Fj)
    np.add.at(pe, i, 0.5 * phi)
    np.add.at(pe, j, 0.5 * phi)
    Wt += np.einsum("pa,pb->ab", d, Fj)
    E2 = float(phi.sum())
    if scales:
        es, fs = pair_scales(P["kind"], r, P["eps"], P["sigma"], P["n"])
        np.add.at(A_pe, i, 0.5 * es)
        np.add.at(A_pe, j, 0.5 * es)
        np.add.at(A_F, i, fs)
        np.add.at(A_F, j, fs)
        A_W += float((r * fs).sum())
        A_E = float(es.sum())

    # ---- three-body terms ---------------------------------------------------
    E = directed_swap_edges(P)
    a, b = triplets(E, N)
    E3 = 0.0
    if a.size:
        Lt = triplet_lambda(E, a, b)
        cen, pa, pb = E["c"][a], E["p"][a], E["p"][b]
        ua, ub = E["u"][a], E["u"][b]
        ra, rb = E["r"][a], E["r"][b]
        da, db = E["d"][a], E["d"][b]
        e = Lt * ua * ub
        Fa = -(Lt * E["u1"][a] * ub / ra)[:, None] * da
        Fb = -(Lt * ua * E["u1"][b] / rb)[:, None] * db
        np.add.at(F, pa, Fa)
        np.add.at(F, pb, Fb)
        np.add.at(F, cen, -(Fa + Fb))
        np.add.at(pe, cen, e)
        Wt += np.einsum("pa,pb->ab", da, Fa) + np.einsum("pa,pb->ab", db, Fb)
        E3 = float(e.sum())
        if scales:
            usa, usb = E["us"][a], E["us"][b]
            fsa = np.abs(Lt) * E["u1s"][a] * usb
            fsb = np.abs(Lt) * usa * E["u1s"][b]
            es3 = np.abs(Lt) * usa * usb
            A_E += float(es3.sum())
            np.add.at(A_pe, cen, es3)
            np.add.at(A_F, pa, fsa)
            np.add.at(A_F, pb, fsb)
            np.add.at(A_F, cen, fsa + fsb)
            A_W += float((ra * fsa + rb * fsb).sum())

    bonds = int(np.count_nonzero((P["kind"] == KIND_SWAP) & (P["r2"] < P["rmin2"])))
    W = np.array([Wt[0, 0], Wt[1, 1], Wt[2, 2], Wt[0, 1], Wt[0, 2], Wt[1, 2]])
    out = dict(E=E2 + E3, E2=E2, E3=E3, pe=pe, F=F, W=W, W_full=Wt, bonds=bonds,
               n_pairs=int(i.size), n_triplets=int(a.size))
    if scales:
        out.update(A_E=A_E, A_pe=A_pe, A_F=A_F, A_W=A_W)
    return out


def energy(pos, types, L, table) -> float:
    return evaluate(pos, types, L, table, scales=False)["E"]


def bond_count(pos, types, L, table) -> int:
    """Number of swap pairs i<j with r^2 < r_min^2 (canonical predicate)."""
    P = interacting_pairs(pos, types, L, table)
    return int(np.count_nonzero((P["kind"] == KIND_SWAP) & (P["r2"] < P["rmin2"])))


def bond_partners(pos, types, L, table) -> np.ndarray:
    """Per particle (in the order of pos): the index of its single bonded swap partner
    (r^2 < r_min^2), -1 without a bond, -2 with more than one."""
    P = interacting_pairs(pos, types, L, table)
    m = (P["kind"] == KIND_SWAP) & (P["r2"] < P["rmin2"])
    i, j = P["i"][m], P["j"][m]
    deg = np.zeros(P["N"], np.int64)
    np.add.at(deg, i, 1)
    np.add.at(deg, j, 1)
    out = np.full(P["N"], -1, np.int64)
    out[i] = j
    out[j] = i
    out[deg > 1] = -2
    return out


def bond_autocorrelation(partners0, partners_t, mask=None) -> float:
    """Fraction of the bonds present in partners0 that are still present (same partner) in
    partners_t (the bond autocorrelation of the paper's swap test, Sec. 3.1); mask selects the
    particles counted (e.g. the minority species, whose every member is bonded)."""
    p0 = np.asarray(partners0)
    pt = np.asarray(partners_t)
    keep = p0 >= 0
    if mask is not None:
        keep &= np.asarray(mask, bool)
    if not np.any(keep):
        return float("nan")
    return float(np.mean(pt[keep] == p0[keep]))


def bond_degree(pos, types, L, table) -> np.ndarray:
    """Per-particle number of bonded swap partners (r^2 < r_min^2)."""
    P = interacting_pairs(pos, types, L, table)
    m = (P["kind"] == KIND_SWAP) & (P["r2"] < P["rmin2"])
    deg = np.zeros(P["N"], np.int64)
    np.add.at(deg, P["i"][m], 1)
    np.add.at(deg, P["j"][m], 1)
    return deg
