"""Second derivatives of the swap-potential energy, per term, in FP64.

TEST INFRASTRUCTURE ONLY.  The paper defines the energy (Sec. 2: eq. 2b,
eq. pot, eq. 3bp); its derivatives are the plain calculus of those terms.

* ``hvp``: H v with H = d^2 E / dx dx (so the force JVP is -H v).  Pair term
  phi(r), r = |x_j - x_i|, D = v_j - v_i, dr = rhat.D:
      (Hv)_j = phi'' dr rhat + (phi'/r)(D - dr rhat),   (Hv)_i = -(Hv)_j.
  Triplet term Lambda u(r_a) u(r_b) with centre c and partners a, b,
  D_a = v_a - v_c, dr_a = rhat_a.D_a:
      (Hv)_a = Lambda [(u''_a dr_a u_b + u'_a u'_b dr_b) rhat_a
                       + u'_a u_b (D_a - dr_a rhat_a)/r_a],
      (Hv)_b symmetric, (Hv)_c = -((Hv)_a + (Hv)_b).
  u'' jumps at r_min and the pair energy jumps at r_cut, so H is defined
  almost everywhere; tests keep finite-difference stencils away from both.
* ``param_grad``: dE/d(eps, sigma, lambda) of every table entry at fixed
  r_cut.  u = vhat does not depend on eps; d u / d sigma = -(dv/dsigma)/eps
  beyond r_min (u is continuous at the moving r_min, so the boundary adds
  nothing); Lambda_ijk = sqrt(Lambda_ij Lambda_ik) contributes half of
  Lambda_ijk/lambda (or /eps) for each of its two entries that is the entry.
* ``force_param_vjp``: a . dF/d(theta) for theta = (eps, sigma, lambda) of
  every entry, by central differences of ``swap_ref`` forces in the
  parameters (used only on small systems).
* ``soft_bonds``: B = sum over interacting swap pairs of vhat(r) (eq. pot)
  and dB/dx_m = -sum_j vhat'(r_mj) (x_j - x_m)/r_mj.

Parity status: pinned by central finite differences of ``swap_ref`` (forces
for ``hvp``, energy for ``param_grad``, ``soft_bonds`` for its own gradient,
and ``soft_bonds`` equals ``swap_ref.bond_count`` when every swap pair inside
r_cut is bonded) and by the identities
dE/dlambda = E3/lambda and dE/deps = (E2_swap + E3)/eps of a one-entry system.
The error scale of ``hvp`` is pinned by its bound on |Hv|, its units and its
closed-form ratio to |Hv| along a bond far beyond r_min
(tests/test_oracle_scales.py).
"""
from __future__ import annotations

import numpy as np

from . import swap_ref
from .swap_ref import KIND_SWAP, KIND_WCA


def hvp(pos, types, L, table, v, with_scale=False):
    """Hessian of the total energy applied to v [N,3] (FP64).

    With ``with_scale`` also returns, per particle, the sum of the magnitudes
    of the term contributions it receives, each taken with absolute-summed
    sub-terms (|phi''| |dr| + |phi'/r| |D_perp| for a pair; likewise for the
    factors of a triplet term): the error scale of a parity test.
    """
    P = swap_ref.interacting_pairs(pos, types, L, table)
    N = P["N"]
    v = np.asarray(v, dtype=np.float64)
    out = np.zeros((N, 3))
    i, j, d = P["i"], P["j"], P["d"]
    r = np.sqrt(P["r2"])
    _, d1, d2 = swap_ref.pair_phi(P["kind"], r, P["eps"], P["sigma"], P["n"])
    rh = d / r[:, None]
    D = v[j] - v[i]
    dr = np.einsum("pa,pa->p", rh, D)
    hj = (d2 * dr)[:, None] * rh + (d1 / r)[:, None] * (D - dr[:, None] * rh)
    np.add.at(out, j, hj)
    np.add.at(out, i, -hj)
    scale = np.zeros(N)
    if with_scale:
        nn_ = np.where(P["kind"] == KIND_WCA, 6.0, P["n"])
        q = np.power(P["sigma"] / r, nn_)
        d2s = 4.0 * P["eps"] * (2.0 * nn_ * (2.0 * nn_ + 1.0) * q * q + nn_ * (nn_ + 1.0) * q) / (r * r)
        d1s = 4.0 * P["eps"] * nn_ * (2.0 * q * q + q) / r
        Dn = np.linalg.norm(D, axis=1)
        sc = d2s * Dn + (d1s / r) * Dn
        np.add.at(scale, i, sc)
        np.add.at(scale, j, sc)

    E = swap_ref.directed_swap_edges(P)
    a, b = swap_ref.triplets(E, N)
    if a.size:
        Lt = swap_ref.triplet_lambda(E, a, b)
        c, pa, pb = E["c"][a], E["p"][a], E["p"][b]
        ra, rb = E["r"][a], E["r"][b]
        rha, rhb = E["d"][a] / ra[:, None], E["d"][b] / rb[:, None]
        Da, Db = v[pa] - v[c], v[pb] - v[c]
        dra = np.einsum("pa,pa->p", rha, Da)
        drb = np.einsum("pa,pa->p", rhb, Db)
        ua, ub = E["u"][a], E["u"][b]
        u1a, u1b = E["u1"][a], E["u1"][b]
        u2a, u2b = E["u2"][a], E["u2"][b]
        ha = (Lt * (u2a * dra * ub + u1a * u1b * drb))[:, None] * rha \
            + (Lt * u1a * ub / ra)[:, None] * (Da - dra[:, None] * rha)
        hb = (Lt * (u2b * drb * ua + u1b * u1a * dra))[:, None] * rhb \
            + (Lt * u1b * ua / rb)[:, None] * (Db - drb[:, None] * rhb)
        np.add.at(out, pa, ha)
        np.add.at(out, pb, hb)
        np.add.at(out, c, -(ha + hb))
        if with_scale:
            usa, usb = E["us"][a], E["us"][b]
            u1sa, u1sb = E["u1s"][a], E["u1s"][b]
            # |u''| scale beyond r_min: 4 (2n(2n+1) q^2 + n(n+1) q)/r^2 ; inside: 0
            def u2s(k):
                n_ = E["n"][k]
                q_ = np.power(E["sigma"][k] / E["r"][k], n_)
                inside = E["r2"][k] <= E["rmin2"][k]
                val = 4.0 * (2.0 * n_ * (2.0 * n_ + 1.0) * q_ * q_ + n_ * (n_ + 1.0) * q_) / E["r"][k] ** 2
                return np.where(inside, 0.0, val)
            Dan, Dbn = np.linalg.norm(Da, axis=1), np.linalg.norm(Db, axis=1)
            sa = np.abs(Lt) * ((u2s(a) * Dan * usb + u1sa * u1sb * Dbn) + u1sa * usb * Dan / ra)
            sb = np.abs(Lt) * ((u2s(b) * Dbn * usa + u1sb * u1sa * Dan) + u1sb * usa * Dbn / rb)
            np.add.at(scale, pa, sa)
            np.add.at(scale, pb, sb)
            np.add.at(scale, c, sa + sb)
    if with_scale:
        return out, scale
    return out


def param_grad(pos, types, L, table):
    """dE/d(eps, sigma, lambda) per table entry -> array [nt, nt, 3].

    Entry (a,b) and (b,a) are one parameter; the gradient is reported on both
    (symmetric), each holding the full derivative with respect to that shared
    parameter.
    """
    P = swap_ref.interacting_pairs(pos, types, L, table)
    nt = table.kind.shape[0]
    N = P["N"]
    g = np.zeros((nt, nt, 3))
    ty = np.asarray(types, dtype=np.int64)

    def entry_key(ti, tj):
        lo, hi = np.minimum(ti, tj), np.maximum(ti, tj)
        return lo * nt + hi

    acc = np.zeros((nt * nt, 3))
    r = np.sqrt(P["r2"])
    key = entry_key(ty[P["i"]], ty[P["j"]])
    kind, eps, sig, n = P["kind"], P["eps"], P["sigma"], P["n"]
    nn = np.where(kind == KIND_WCA, 6.0, n)
    phi = swap_ref.mie(r, eps, sig, nn) + np.where(kind == KIND_WCA, eps, 0.0)
    np.add.at(acc[:, 0], key, phi / eps)                                 # phi is linear in eps
    np.add.at(acc[:, 1], key, swap_ref.mie_dsigma(r, eps, sig, nn))

    E = swap_ref.directed_swap_edges(P)
    a, b = swap_ref.triplets(E, N)
    if a.size:
        Lt = swap_ref.triplet_lambda(E, a, b)
        c = E["c"][a]
        ka = entry_key(ty[c], ty[E["p"][a]])
        kb = entry_key(ty[c], ty[E["p"][b]])
        ua, ub = E["u"][a], E["u"][b]
        e = Lt * ua * ub
        # Lambda_ijk = sqrt(lam_a eps_a lam_b eps_b): d/dlam_a = Lambda/(2 lam_a)
        for kk, lamk, epsk in ((ka, E["lam"][a], E["eps"][a]), (kb, E["lam"][b], E["eps"][b])):
            with np.errstate(divide="ignore", invalid="ignore"):
                dl = np.where(lamk != 0.0, 0.5 * e / lamk, 0.0)
            np.add.at(acc[:, 2], kk, dl)
            np.add.at(acc[:, 0], kk, 0.5 * e / epsk)
        # d lambda-derivative when lambda = 0 : E3 is linear in sqrt(lam_a lam_b);
        # for a one-entry system dE/dlam = sum u_a u_b eps.
        zero = (E["lam"][a] == 0.0) & (E["lam"][b] == 0.0) & (ka == kb)
        if np.any(zero):
            np.add.at(acc[:, 2], ka[zero], (E["eps"][a] * ua * ub)[zero])
        # sigma through u beyond r_min
        ra, rb = E["r"][a], E["r"][b]
        inside_a = E["r2"][a] <= E["rmin2"][a]
        inside_b = E["r2"][b] <= E["rmin2"][b]
        dua = np.where(inside_a, 0.0, -swap_ref.mie_dsigma(ra, 1.0, E["sigma"][a], E["n"][a]))
        dub = np.where(inside_b, 0.0, -swap_ref.mie_dsigma(rb, 1.0, E["sigma"][b], E["n"][b]))
        np.add.at(acc[:, 1], ka, Lt * dua * ub)
        np.add.at(acc[:, 1], kb, Lt * ua * dub)
    for x in range(nt):
        for y in range(nt):
            g[x, y] = acc[min(x, y) * nt + max(x, y)]
    return g


def _with_param(table, a, b, which, value):
    t = table.copy()
    arr = {0: t.epsilon, 1: t.sigma, 2: t.lam}[which]
    arr[a, b] = value
    arr[b, a] = value
    return t


def force_param_vjp(pos, types, L, table, adj, h=1e-6):
    """sum_m adj_m . dF_m/dtheta for theta = (eps, sigma, lambda) of each entry."""
    nt = table.kind.shape[0]
    out = np.zeros((nt, nt, 3))
    adj = np.asarray(adj, dtype=np.float64)
    for a in range(nt):
        for b in range(a, nt):
            if table.kind[a, b] == 0:
                continue
            for w, arr in ((0, table.epsilon), (1, table.sigma), (2, table.lam)):
                if w == 2 and table.kind[a, b] != KIND_SWAP:
                    continue
                p0 = float(arr[a, b])
                step = h * max(1.0, abs(p0))
                Fp = swap_ref.evaluate(pos, types, L, _with_param(table, a, b, w, p0 + step),
                                       scales=False)["F"]
                Fm = swap_ref.evaluate(pos, types, L, _with_param(table, a, b, w, p0 - step),
                                       scales=False)["F"]
                val = float(np.sum(adj * (Fp - Fm))) / (2.0 * step)
                out[a, b, w] = val
                out[b, a, w] = val
    return out


def soft_bonds(pos, types, L, table):
    """(B, dB/dx [N,3]) with B = sum over interacting swap pairs of vhat(r)."""
    P = swap_ref.interacting_pairs(pos, types, L, table)
    E = swap_ref.directed_swap_edges(P)
    N = P["N"]
    B = 0.5 * float(np.sum(E["u"]))
    g = np.zeros((N, 3))
    if E["c"].size:
        # centre c: dvhat(r_cp)/dx_c = -vhat'(r) rhat_cp
        np.add.at(g, E["c"], -(E["u1"] / E["r"])[:, None] * E["d"])
    return B, g
