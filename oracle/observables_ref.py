"""FP64 oracle of the observables built on the step: the stress autocorrelation G(t) and the
bond-partner statistics (bond autocorrelation and swap events).

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain loops over the definitions, no
reordering beyond them.

Definitions:

* A logged row holds (E, W_xx, W_yy, W_zz, W_xy, W_xz, W_yz, K_xx, K_yy, K_zz, K_xy, K_xz, K_yz):
  energy, configurational virial and kinetic tensor of one step.  The stress tensor of the row is
  sigma_ab = -(K_ab + W_ab) / V (the pressure tensor of eq. p3 with its kinetic part, negated).
* G(t) (the stress relaxation modulus by the autocorrelation method, Sec. 2.2 after eq. p3):
  V / kT times the average of sigma_ab(t0) sigma_ab(t0 + t) over the three off-diagonal
  components ab = xy, xz, yz (the overline: a reading) and over every time origin t0 of the
  series with t0 + t inside it (the angle brackets: a reading).  t counts rows.
* Bond partners at times 0 and t are tag-indexed (-1: no bond, -2: several bonds).  A selected
  particle is bonded at 0 if p0 >= 0; it is unchanged if also pt == p0 (the bond autocorrelation
  of Sec. 3.1 / Fig. 3 is unchanged / bonded), and it has swapped if pt >= 0 and pt != p0 (its
  partner changed: the swap event of a bonded site).
"""
import numpy as np

OFF_DIAGONAL = ((4, 10), (5, 11), (6, 12))   # (W_ab, K_ab) columns of xy, xz, yz


def shear_stress(rows, volume):
    """(T, 3) off-diagonal stresses sigma_xy, sigma_xz, sigma_yz of the logged rows."""
    r = np.asarray(rows, np.float64)
    out = np.empty((r.shape[0], 3))
    for c, (w, k) in enumerate(OFF_DIAGONAL):
        out[:, c] = -(r[:, k] + r[:, w]) / volume
    return out


def stress_autocorrelation(rows, volume, kT, max_lag):
    """G(t) for t = 0 .. max_lag (max_lag < number of rows)."""
    s = shear_stress(rows, volume)
    T = s.shape[0]
    if not 0 <= max_lag < T:
        raise ValueError("max_lag must be in [0, T)")
    G = np.zeros(max_lag + 1)
    for t in range(max_lag + 1):
        acc = 0.0
        for t0 in range(T - t):
            for c in range(3):
                acc += s[t0, c] * s[t0 + t, c]
        G[t] = volume / kT * acc / (3 * (T - t))
    return G


def partner_counts(p0, pt, select=None):
    """(bonded at 0, unchanged, swapped) over the selected particles."""
    p0 = np.asarray(p0)
    pt = np.asarray(pt)
    sel = np.ones(p0.shape[0], bool) if select is None else np.asarray(select, bool)
    bonded = unchanged = swapped = 0
    for i in range(p0.shape[0]):
        if not sel[i] or p0[i] < 0:
            continue
        bonded += 1
        if pt[i] == p0[i]:
            unchanged += 1
        elif pt[i] >= 0:
            swapped += 1
    return bonded, unchanged, swapped
