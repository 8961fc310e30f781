"""Pins of the oracle's error scales and of the rigid-body thermostat.

Every GPU parity bar is a multiple of a scale the oracle computes: A_F per
particle, A_E, A_W and A_pe (``swap_ref.evaluate``) and the per-particle
scale of ``adjoint_ref.hvp(..., with_scale=True)``.  Each is defined as the
sum, over the terms that touch a quantity, of that term's sub-terms taken
with absolute values.  Three facts fix such a scale without retyping it:

* it bounds the quantity it scales (triangle inequality), on any
  configuration;
* it carries the quantity's units: multiplying every eps by c multiplies it
  by c, and stretching every length (sigma, r_cut, positions, box) by s
  divides a force scale by s, an HVP scale by s^2 and leaves energy and
  virial scales unchanged (a dropped 1/r or a stray factor r fails this);
* where one sub-term dominates (n = 100 far beyond r_min, where
  (sigma/r)^n << 1, or deep inside the core, where it is >> 1) the
  absolute sum equals the magnitude of the quantity itself, whose value
  the finite-difference and closed-form pins of the oracle already fix.
  Three-body scales are isolated by differencing lambda: the scales grow
  linearly in lambda from their pair part.

The rigid-body Langevin branch is pinned by equipartition of a free-body gas
(translation and rotation, with unequal mass and inertia).
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import adjoint_ref, rigid_ref, swap_ref


def ev(pos, types, L, table):
    return swap_ref.evaluate(np.asarray(pos, dtype=np.float64), np.asarray(types), L, table)


def mixed_table(lam, eps_scale=1.0, s=1.0):
    """Two swap entries of different exponents plus a WCA cross entry, all lengths times s."""
    tab = W.PairTable.empty(2)
    tab.set(0, 0, W.KIND_SWAP, 1.0 * eps_scale, 1.0 * s, 10, 1.5 * s, lam)
    tab.set(0, 1, W.KIND_WCA, 1.3 * eps_scale, 0.9 * s, 6)
    tab.set(1, 1, W.KIND_SWAP, 2.0 * eps_scale, 0.8 * s, 8, 1.2 * s, 0.5 * lam)
    return tab


def random_cluster(rng, N, box, min_r=0.78):
    while True:
        pos = rng.uniform(-box, box, size=(N, 3))
        ty = rng.integers(0, 2, size=N)
        d = pos[:, None, :] - pos[None, :, :]
        r = np.sqrt((d * d).sum(-1))
        if np.min(r[np.triu_indices(N, 1)]) > min_r:
            return pos, ty


# --------------------------------------------------------------------------
# bounds: every scale dominates what it scales
# --------------------------------------------------------------------------

@pytest.mark.parametrize("lam", [0.0, 0.7, 1.0, 2.5])
def test_scales_bound_the_quantities(lam):
    rng = np.random.default_rng(41)
    tab = mixed_table(lam)
    for trial in range(6):
        pos, ty = random_cluster(rng, 14, 1.6)
        out = ev(pos, ty, 40.0, tab)
        assert out["n_triplets"] > 0 or lam == 0.0
        Fn = np.linalg.norm(out["F"], axis=1)
        assert np.all(Fn <= out["A_F"] * (1 + 1e-12))
        assert abs(out["E"]) <= out["A_E"] * (1 + 1e-12)
        assert np.all(np.abs(out["pe"]) <= out["A_pe"] * (1 + 1e-12))
        assert np.abs(out["W"]).max() <= out["A_W"] * (1 + 1e-12)
        v = rng.standard_normal(pos.shape)
        hv, hs = adjoint_ref.hvp(pos, ty, 40.0, tab, v, with_scale=True)
        assert np.all(np.linalg.norm(hv, axis=1) <= hs * (1 + 1e-12))


# --------------------------------------------------------------------------
# units: eps and length scaling
# --------------------------------------------------------------------------

def test_scales_carry_the_units_of_their_quantities():
    rng = np.random.default_rng(43)
    pos, ty = random_cluster(rng, 14, 1.6)
    v = rng.standard_normal(pos.shape)
    base = ev(pos, ty, 40.0, mixed_table(1.3))
    _, hs = adjoint_ref.hvp(pos, ty, 40.0, mixed_table(1.3), v, with_scale=True)
    assert base["n_triplets"] > 0
    # energy scaling: everything linear in eps (lambda is dimensionless)
    c = 3.0
    o = ev(pos, ty, 40.0, mixed_table(1.3, eps_scale=c))
    _, hs_c = adjoint_ref.hvp(pos, ty, 40.0, mixed_table(1.3, eps_scale=c), v, with_scale=True)
    np.testing.assert_allclose(o["A_F"], c * base["A_F"], rtol=1e-12)
    np.testing.assert_allclose(o["A_pe"], c * base["A_pe"], rtol=1e-12)
    assert o["A_E"] == pytest.approx(c * base["A_E"], rel=1e-12)
    assert o["A_W"] == pytest.approx(c * base["A_W"], rel=1e-12)
    np.testing.assert_allclose(hs_c, c * hs, rtol=1e-12)
    # length scaling by s: forces 1/s, Hessian 1/s^2, energies and virials unchanged
    s = 0.37
    o = ev(s * pos, ty, 40.0 * s, mixed_table(1.3, s=s))
    _, hs_s = adjoint_ref.hvp(s * pos, ty, 40.0 * s, mixed_table(1.3, s=s), v, with_scale=True)
    assert o["n_pairs"] == base["n_pairs"] and o["n_triplets"] == base["n_triplets"]
    np.testing.assert_allclose(o["A_F"], base["A_F"] / s, rtol=1e-10)
    np.testing.assert_allclose(o["A_pe"], base["A_pe"], rtol=1e-10)
    assert o["A_E"] == pytest.approx(base["A_E"], rel=1e-10)
    assert o["A_W"] == pytest.approx(base["A_W"], rel=1e-10)
    np.testing.assert_allclose(hs_s, hs / s ** 2, rtol=1e-10)


# --------------------------------------------------------------------------
# tightness where one sub-term dominates
# --------------------------------------------------------------------------

def n100_table(lam=1.0, rcut=1.3):
    return W.swap_table_single(epsilon=1.0, sigma=1.0, n=100, rcut=rcut, lam=lam)


@pytest.mark.parametrize("r", [1.2, 1.25, 1.29])
def test_pair_scales_are_tight_far_beyond_rmin(r):
    # (1/r)^100 < 1.2e-8: the attractive sub-term is all there is
    out = ev([[0, 0, 0], [r, 0, 0]], [0, 0], 30.0, n100_table(lam=0.0))
    F = abs(out["F"][1, 0])
    assert F > 0
    assert out["A_F"][0] == pytest.approx(F, rel=1e-7)
    assert out["A_F"][1] == pytest.approx(F, rel=1e-7)
    assert out["A_E"] == pytest.approx(abs(out["E"]), rel=1e-7)
    assert out["A_pe"][0] == pytest.approx(abs(out["pe"][0]), rel=1e-7)
    assert out["A_W"] == pytest.approx(abs(out["W"][0]), rel=1e-7)   # pair along x: W_xx is all of it
    # Hessian along the bond: phi'' dominates phi'/r by (n + 1), so the scale
    # (|phi''| + |phi'|/r) |D| is |Hv| (n + 2) / (n + 1) to that order
    v = np.array([[0.0, 0, 0], [1.0, 0, 0]])
    hv, hs = adjoint_ref.hvp(np.array([[0, 0, 0], [r, 0, 0]], float), [0, 0], 30.0, n100_table(lam=0.0), v,
                             with_scale=True)
    assert hs[1] == pytest.approx(abs(hv[1, 0]) * 102.0 / 101.0, rel=1e-6)


@pytest.mark.parametrize("r", [0.85, 0.9])
def test_pair_scales_are_tight_deep_in_the_core(r):
    # (1/r)^100 > 3.7e4: the repulsive sub-term is all there is (to ~1/q)
    out = ev([[0, 0, 0], [r, 0, 0]], [0, 0], 30.0, n100_table(lam=0.0))
    F = abs(out["F"][1, 0])
    q = r ** -100
    assert out["A_F"][1] == pytest.approx(F, rel=2.0 / q)
    assert out["A_E"] == pytest.approx(abs(out["E"]), rel=3.0 / q)
    assert out["A_W"] == pytest.approx(abs(out["W"][0]), rel=2.0 / q)


def test_wca_scale_near_contact():
    tab = W.PairTable.empty(1)
    tab.set(0, 0, W.KIND_WCA, 2.0, 1.0, 6)
    out = ev([[0, 0, 0], [0.5, 0, 0]], [0, 0], 30.0, tab)
    F = abs(out["F"][1, 0])
    # q = (1/0.5)^6 = 64: force sub-terms 2q^2 and q, energy q^2, q and the shift
    assert 0.98 <= F / out["A_F"][1] <= 1.0
    assert 0.96 <= abs(out["E"]) / out["A_E"] <= 1.0
    assert out["E"] > 0


def _lambda_parts(pos, types, table_of):
    """Three-body parts of the values and scales: lambda-differenced (both are linear in lambda)."""
    a, b = ev(pos, types, 30.0, table_of(0.0)), ev(pos, types, 30.0, table_of(1.0))
    c = ev(pos, types, 30.0, table_of(2.0))
    for k in ("A_F", "A_pe"):
        # differences of sums whose pair part may be ~1e10 times the three-body part
        np.testing.assert_allclose(c[k] - a[k], 2.0 * (b[k] - a[k]), rtol=1e-9, atol=1e-14 * np.abs(c[k]).max())
    for k in ("A_E", "A_W"):
        assert c[k] - a[k] == pytest.approx(2.0 * (b[k] - a[k]), rel=1e-9, abs=1e-14 * c[k])
    return a, b


def test_triplet_scales_with_one_partner_bonded():
    # collinear A1 - B - A2, n = 100: A1 inside r_min (vhat = 1, vhat' = 0), A2 far beyond,
    # A1-A2 beyond r_cut.  At lambda = 1 the triplet force on A2 cancels its pair force
    # (the flat barrier), so the triplet parts equal the pair magnitudes there.
    pos = np.array([[-1.0, 0, 0], [0.0, 0, 0], [1.25, 0, 0]])
    ty = np.zeros(3, int)
    a, b = _lambda_parts(pos, ty, lambda lam: n100_table(lam=lam))
    assert b["n_triplets"] == 1
    dF = b["F"] - a["F"]
    tF = b["A_F"] - a["A_F"]
    assert tF[0] == 0.0 and np.abs(dF[0]).max() == 0.0          # no three-body force on the bonded partner
    assert tF[2] == pytest.approx(abs(dF[2, 0]), rel=1e-7)
    # the centre's pair scale (partner inside r_min) is ~1e10 times its three-body part:
    # the lambda difference keeps about 11 digits
    assert tF[1] == pytest.approx(abs(dF[1, 0]), rel=1e-5)
    assert abs(b["F"][2, 0]) < 1e-12 * a["A_F"][2]               # flat barrier
    assert tF[2] == pytest.approx(a["A_F"][2], rel=1e-12)
    assert b["A_E"] - a["A_E"] == pytest.approx(abs(b["E3"]), rel=1e-7)
    assert b["A_W"] - a["A_W"] == pytest.approx(abs(b["W"][0] - a["W"][0]), rel=1e-7)
    assert (b["A_pe"] - a["A_pe"])[1] == pytest.approx(abs(b["pe"][1] - a["pe"][1]), rel=1e-5)


def test_triplet_scales_with_both_partners_beyond_rmin():
    # both partners at (1/r)^100 = 1e-3: every three-body factor is within 0.4 % of its
    # dominant sub-term; lambda = 1e4 makes the triplet the main force
    r = 10.0 ** 0.03
    pos = np.array([[-r, 0, 0], [0.0, 0, 0], [r, 0, 0]])
    ty = np.zeros(3, int)
    a, b = _lambda_parts(pos, ty, lambda lam: n100_table(lam=1e4 * lam))
    assert b["n_triplets"] == 1
    dF = np.abs(b["F"] - a["F"])[:, 0]
    tF = b["A_F"] - a["A_F"]
    ends = [0, 2]   # the centre's two reactions cancel in this symmetric layout
    assert np.all(dF[ends] > 0)
    assert np.all(dF <= tF * (1 + 1e-12)) and np.all(dF[ends] >= 0.99 * tF[ends])
    e3 = abs(b["E3"])
    assert 0.99 * (b["A_E"] - a["A_E"]) <= e3 <= (b["A_E"] - a["A_E"]) * (1 + 1e-12)
    dW = abs(b["W"][0] - a["W"][0])
    assert 0.99 * (b["A_W"] - a["A_W"]) <= dW <= (b["A_W"] - a["A_W"]) * (1 + 1e-12)
    # the centre receives both partners' reactions, so its scale is their sum
    assert tF[1] == pytest.approx(tF[0] + tF[2], rel=1e-12)


# --------------------------------------------------------------------------
# rigid bodies: the Langevin branch thermalises translation and rotation
# --------------------------------------------------------------------------

def test_rigid_langevin_free_body_equipartition():
    B = 3000
    M, I, kT = 2.0, 0.125, 0.8
    bodies = dict(centre=np.arange(B), first=np.zeros(B + 1, np.int64), member=np.zeros(0, np.int64),
                  offset=np.zeros((0, 2)), inertia=np.full(B, I))
    L = (400.0, 400.0, 8.0)
    rng = np.random.default_rng(12)
    pos = np.zeros((B, 3))
    pos[:, :2] = rng.uniform(-190, 190, size=(B, 2))
    vel = np.zeros((B, 3))
    th, w = np.zeros(B), np.zeros(B)
    ty = np.zeros(B, np.int64)
    zero = np.zeros((B, 3))
    kin_t, kin_r = [], []
    for k in range(60):
        pos, vel, th, w = rigid_ref.half_step(pos, vel, zero, th, w, ty, bodies, L, [M], 0.25, kT, 2.0, 77, k, True)
        pos, vel, th, w = rigid_ref.half_step(pos, vel, zero, th, w, ty, bodies, L, [M], 0.25, kT, 2.0, 77, k, False)
        if k >= 20:   # c1^(2k) = exp(-2 gamma dt k) < 1e-8 by then
            kin_t.append(M * np.mean(vel[:, :2] ** 2))
            kin_r.append(I * np.mean(w ** 2))
    assert np.all(vel[:, 2] == 0.0)
    # 2 translational and 1 rotational degree of freedom per body, each kT/2
    assert np.mean(kin_t) == pytest.approx(kT, rel=0.04)
    assert np.mean(kin_r) == pytest.approx(kT, rel=0.05)
