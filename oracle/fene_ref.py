"""FENE bond springs of a bead-spring network, in FP64.

TEST INFRASTRUCTURE ONLY.  The paper's vitrimer-like networks (Sec. 3,
polymer applications) use bead-spring chains; the springs follow the
finite-extensible nonlinear elastic form of Kremer & Grest (1990):

    U(r) = -(1/2) K R0^2 ln(1 - (r/R0)^2),   r < R0,

with the WCA repulsion of the pair table acting between all pairs, bonded
or not.  Force on bead i of bond (i, j), d = x_j - x_i (minimum image):
F_i = K d / (1 - r^2/R0^2); the virial of the bond is d (x) F_j = -K d d /
(1 - r^2/R0^2).  Bonds are pairs of tags; every bond is listed once.

Parity status: pinned by central finite differences of the energy, by the
closed-form force at a chosen extension, and by the Kremer-Grest bond length
(the minimum of FENE plus WCA with K = 30, R0 = 1.5, eps = sigma = 1 lies at
about 0.96 sigma).
"""
from __future__ import annotations

import numpy as np

from . import swap_ref


def bond_pairs(bonds_by_tag):
    """Unique (i, j) tag pairs, i < j, of a [N, 2] partner table (-1 = none)."""
    b = np.asarray(bonds_by_tag, dtype=np.int64)
    i = np.repeat(np.arange(b.shape[0]), b.shape[1])
    j = b.ravel()
    keep = (j >= 0) & (i < j)
    return i[keep], j[keep]


def evaluate(pos, L, bonds_by_tag, K, R0):
    """dict(E, F [N,3], W [6] (xx yy zz xy xz yz), pe [N], A_F [N]) of the springs.

    pos is in tag order.  A_F is the per-bead force scale (sum of |F| of its
    bonds), for parity tolerances."""
    x = np.asarray(pos, dtype=np.float64)
    N = x.shape[0]
    Lv = np.broadcast_to(np.asarray(L, dtype=np.float64), (3,))
    i, j = bond_pairs(bonds_by_tag)
    d = swap_ref.min_image(x[i], x[j], Lv)
    r2 = np.einsum("ba,ba->b", d, d)
    s = 1.0 - r2 / (R0 * R0)
    if np.any(s <= 0.0):
        raise ValueError("a bond is stretched beyond R0")
    E_b = -0.5 * K * R0 * R0 * np.log(s)
    g = K / s                      # F_i = g d, F_j = -g d
    F = np.zeros((N, 3))
    np.add.at(F, i, g[:, None] * d)
    np.add.at(F, j, -g[:, None] * d)
    W = np.array([np.sum(-g * d[:, a] * d[:, b]) for a, b in ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))])
    pe = np.zeros(N)
    np.add.at(pe, i, 0.5 * E_b)
    np.add.at(pe, j, 0.5 * E_b)
    A = np.zeros(N)
    fm = g * np.sqrt(r2)
    np.add.at(A, i, fm)
    np.add.at(A, j, fm)
    return dict(E=float(np.sum(E_b)), F=F, W=W, pe=pe, A_F=A, n_bonds=int(i.size))
