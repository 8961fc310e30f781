"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Every check here is independent of the oracle's own formulas: closed-form
values stated in the paper (well depth, flat barrier, swap barrier, the
scenario descriptions of Fig. 1), finite differences of the energy (forces,
virial via strain), conservation laws, literal triple loops, and published
known-answer vectors for the random number generator.
"""
import json
import math
import os

import numpy as np
import pytest

import workloads as W
from oracle import adjoint_ref, dynamics_ref, literal, philox_ref, rigid_ref, swap_ref

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def paper_values():
    with open(os.path.join(GOLD, "paper_values.json")) as f:
        return json.load(f)


def two_type_table(lam, eps=1.0, sigma=1.0, n=10, rcut=1.5):
    """A-B swap only (types 0 = A, 1 = B); A-A and B-B do not interact."""
    t = W.PairTable.empty(2)
    t.set(0, 1, W.KIND_SWAP, eps, sigma, n, rcut, lam)
    return t


def ev(pos, types, L, table):
    return swap_ref.evaluate(np.asarray(pos, dtype=np.float64), types, L, table)


# --------------------------------------------------------------------------
# closed forms of the pair term and the switching factor (Sec. 2)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("eps,sigma,n", [(1.0, 1.0, 10), (15.0, 0.3, 10), (1.0, 1.0, 100), (2.5, 0.7, 7)])
def test_dimer_at_rmin_has_depth_eps_and_no_force(eps, sigma, n):
    pv = paper_values()["well_depth_at_rmin"]
    rm = sigma * 2.0 ** (1.0 / n)
    tab = W.swap_table_single(eps, sigma, n, rcut=1.5 * sigma, lam=1.0)
    out = ev([[0, 0, 0], [rm, 0, 0]], [0, 0], 50.0, tab)
    assert out["E"] == pytest.approx(pv["value_over_eps"] * eps, rel=1e-13)
    assert np.abs(out["F"]).max() < 1e-9 * eps / sigma
    assert out["E3"] == 0.0


def test_curvature_at_minimum_matches_closed_form():
    # v''(r_min) = 2 n^2 eps / r_min^2 follows from eq. (2b); measured here by
    # a central difference of the oracle's *force*.
    for eps, sigma, n in [(1.0, 1.0, 10), (15.0, 0.3, 10), (1.0, 1.0, 100)]:
        rm = sigma * 2.0 ** (1.0 / n)
        tab = W.swap_table_single(eps, sigma, n, rcut=1.5 * sigma, lam=0.0)
        h = 1e-6 * sigma
        fp = ev([[0, 0, 0], [rm + h, 0, 0]], [0, 0], 50.0, tab)["F"][1, 0]
        fm = ev([[0, 0, 0], [rm - h, 0, 0]], [0, 0], 50.0, tab)["F"][1, 0]
        k = -(fp - fm) / (2 * h)
        assert k == pytest.approx(2 * n * n * eps / rm ** 2, rel=1e-6)


def test_vhat_is_continuous_with_unit_value_at_rmin():
    # eq. (pot): vhat = 1 inside r_min and -v/eps outside; v(r_min) = -eps makes it continuous
    for n in (10, 100):
        rm = 2.0 ** (1.0 / n)
        inside = swap_ref.vhat_scalar(rm * (1 - 1e-12), 1.0, 1.0, n, 1.5)
        outside = swap_ref.vhat_scalar(rm * (1 + 1e-9), 1.0, 1.0, n, 1.5)
        assert inside == 1.0
        assert outside == pytest.approx(1.0, abs=1e-12)
        assert swap_ref.vhat_scalar(1.5, 1.0, 1.0, n, 1.5) == 0.0


def test_cutoff_value_for_n100_is_orders_below_lj():
    pv = paper_values()["cutoff_value_n100"]
    tab = W.swap_table_single(1.0, 1.0, pv["n"], rcut=1.3, lam=0.0)
    e = ev([[0, 0, 0], [pv["r"], 0, 0]], [0, 0], 50.0, tab)["E"]
    # Lennard-Jones 12-6 at 2.5 sigma through the WCA kind minus its shift
    wt = W.PairTable.empty(1).set(0, 0, W.KIND_WCA, 1.0, 1.0, 6, rcut=3.0)
    lj = ev([[0, 0, 0], [pv["lj_r"], 0, 0]], [0, 0], 50.0, wt)["E"] - 1.0
    assert e < 0 and lj < 0
    assert abs(e) / abs(lj) < pv["max_ratio"]


def test_truncation_cutoff_is_strict():
    tab = W.swap_table_single(1.0, 1.0, 10, rcut=1.5, lam=1.0)
    # a pair exactly at r_cut does not interact; just inside it does
    out = ev([[0, 0, 0], [1.5, 0, 0]], [0, 0], 50.0, tab)
    assert out["E"] == 0.0 and out["n_pairs"] == 0
    out = ev([[0, 0, 0], [np.nextafter(np.float32(1.5), np.float32(0)), 0, 0]], [0, 0], 50.0, tab)
    assert out["n_pairs"] == 1 and out["E"] < 0


# --------------------------------------------------------------------------
# the three-body term: scenarios of Fig. 1 and the swap barrier
# --------------------------------------------------------------------------

@pytest.mark.parametrize("lam", [0.0, 0.5, 1.0, 1.5, 3.0])
def test_flat_barrier_and_scenario_b(lam):
    """Collinear A1-B-A2, A1 at r_min, A2 swept from r_min to r_cut.

    Scenario (b) of Fig. 1 / eq. (regb): the three-body term reduces to
    -lambda v(r_BA2), so E = -eps + (1 - lambda) v(r); with lambda = 1 the
    energy is flat and A2 feels no force (Fig. 2).
    """
    rm = 2.0 ** 0.1
    tab = two_type_table(lam)
    tab0 = two_type_table(0.0)
    for r in np.linspace(rm, 1.49, 23)[1:]:
        pos = [[-rm, 0, 0], [0, 0, 0], [r, 0, 0]]
        ty = [0, 1, 0]
        out = ev(pos, ty, 50.0, tab)
        v = ev([[0, 0, 0], [r, 0, 0]], [0, 1], 50.0, tab0)["E"]
        assert out["E"] == pytest.approx(-1.0 + (1.0 - lam) * v, abs=1e-12)
        # only A2 feels the three-body force (scenario b)
        d3 = out["F"] - ev(pos, ty, 50.0, tab0)["F"]
        assert np.abs(d3[0]).max() < 1e-12
        if lam == 1.0:
            assert abs(out["E"] + 1.0) < 1e-12
            assert np.abs(out["F"][2]).max() < 1e-10
    if lam != 0.0:
        # the three-body force on A2 is repulsive (points away from B)
        out = ev([[-rm, 0, 0], [0, 0, 0], [1.2, 0, 0]], [0, 1, 0], 50.0, tab)
        f2 = out["F"][2, 0] - ev([[-rm, 0, 0], [0, 0, 0], [1.2, 0, 0]], [0, 1, 0], 50.0, tab0)["F"][2, 0]
        assert f2 > 0


@pytest.mark.parametrize("lam", [0.5, 1.0, 2.0])
def test_scenario_a_no_three_body_force(lam):
    # both A inside r_min: the three-body term is constant (Fig. 1a)
    rm = 2.0 ** 0.1
    pos = [[-0.99 * rm, 0, 0], [0, 0, 0], [0, 0.995 * rm, 0]]
    ty = [0, 1, 0]
    a = ev(pos, ty, 50.0, two_type_table(lam))
    b = ev(pos, ty, 50.0, two_type_table(0.0))
    assert np.abs(a["F"] - b["F"]).max() < 1e-12
    assert a["E3"] == pytest.approx(lam * 1.0, abs=1e-14)


def three_type_table(lam_ab, lam_bc, eps_ab=1.0, eps_bc=2.5):
    """Swap pairs A-B and B-C with their own lambda and epsilon (types 0 = A, 1 = B, 2 = C); nothing else."""
    t = W.PairTable.empty(3)
    t.set(0, 1, W.KIND_SWAP, eps_ab, 1.0, 10, 1.5, lam_ab)
    t.set(1, 2, W.KIND_SWAP, eps_bc, 1.0, 10, 1.5, lam_bc)
    return t


@pytest.mark.parametrize("lam_ab,lam_bc", [(0.5, 1.5), (1.0, 0.0), (2.0, 0.3)])
def test_unequal_lambdas_at_rmin_give_the_geometric_mean(lam_ab, lam_bc):
    """Reading of the triplet weight for unequal pair coefficients: Lambda_abc = sqrt(Lambda_ab Lambda_bc)
    (Sec. 2 coefficient list), so with both partners of B inside r_min (vhat = 1, Fig. 1a) the three-body
    energy is sqrt(lambda_ab eps_ab lambda_bc eps_bc) and no three-body force acts; lambda_bc = 0 removes
    the term although the A-B pair alone would carry one."""
    rm = 2.0 ** 0.1
    pos = [[-0.99 * rm, 0, 0], [0, 0, 0], [0, 0.995 * rm, 0]]
    ty = [0, 1, 2]
    a = ev(pos, ty, 50.0, three_type_table(lam_ab, lam_bc))
    b = ev(pos, ty, 50.0, three_type_table(0.0, 0.0))
    assert a["E3"] == pytest.approx(math.sqrt(lam_ab * 1.0 * lam_bc * 2.5), rel=1e-13, abs=1e-15)
    assert np.abs(a["F"] - b["F"]).max() < 1e-12
    assert a["E"] - b["E"] == pytest.approx(a["E3"], rel=1e-12, abs=1e-15)


def test_unequal_lambdas_forces_are_minus_energy_gradient():
    """The same triplet with both partners in the attractive tail (vhat < 1): central differences of the
    energy give the forces with unequal pair coefficients too."""
    pos = np.array([[-1.21, 0.05, 0.0], [0.0, 0.0, 0.02], [0.03, 1.27, 0.0]])
    ty = [0, 1, 2]
    tab = three_type_table(0.7, 1.6)
    out = ev(pos, ty, 50.0, tab)
    assert out["E3"] != 0.0
    h = 1e-6
    for i in range(3):
        for d in range(3):
            p1 = pos.copy(); p1[i, d] += h
            p0 = pos.copy(); p0[i, d] -= h
            g = (ev(p1, ty, 50.0, tab)["E"] - ev(p0, ty, 50.0, tab)["E"]) / (2 * h)
            assert out["F"][i, d] == pytest.approx(-g, rel=1e-6, abs=1e-7)


def test_scenario_c_both_partners_feel_force():
    rm = 2.0 ** 0.1
    pos = [[-1.2, 0, 0], [0, 0, 0], [0, 1.25, 0]]
    ty = [0, 1, 0]
    a = ev(pos, ty, 50.0, two_type_table(1.0))
    b = ev(pos, ty, 50.0, two_type_table(0.0))
    d3 = a["F"] - b["F"]
    assert abs(d3[0, 0]) > 1e-3 and abs(d3[2, 1]) > 1e-3
    assert 1.2 > rm and 1.25 > rm


@pytest.mark.parametrize("lam", [0.0, 0.5, 1.0, 1.5])
def test_swap_barrier_symmetric_triplet(lam):
    """Symmetric triplet at r_min: E = (lambda - 2) eps; the barrier over a
    bonded pair plus a free A is eps (lambda - 1) (Sec. 2, after eq. regb)."""
    pv = paper_values()["swap_barrier"]
    rm = 2.0 ** 0.1
    tab = two_type_table(lam, eps=3.0)
    tri = ev([[-rm, 0, 0], [0, 0, 0], [rm, 0, 0]], [0, 1, 0], 50.0, tab)["E"]
    bonded = ev([[-rm, 0, 0], [0, 0, 0], [20.0, 0, 0]], [0, 1, 0], 50.0, tab)["E"]
    assert tri - bonded == pytest.approx(3.0 * (lam + pv["barrier_over_eps_minus_lambda"]), abs=1e-12)


@pytest.mark.parametrize("lam", [0.0, 0.5, 1.0, 1.5])
def test_per_particle_split_of_a_symmetric_triplet(lam):
    """The per-particle split (half of each pair term to each particle, each triplet term to its centre)
    in closed form: A-B-A with both pairs at r_min (v = -eps, vhat = 1) gives the A ends -eps/2 each and
    the centre B 2 (-eps/2) + lambda eps."""
    rm = 2.0 ** 0.1
    out = ev([[-rm, 0, 0], [0, 0, 0], [rm, 0, 0]], [0, 1, 0], 50.0, two_type_table(lam, eps=3.0))
    assert out["pe"] == pytest.approx([-1.5, 3.0 * (lam - 1.0), -1.5], abs=1e-12)


@pytest.mark.parametrize("lam", [0.0, 1.0, 1.7])
def test_equilateral_triangle(lam):
    # one reactive type: three pairs at r_min and three centres with two partners each
    rm = 2.0 ** 0.1
    pos = [[0, 0, 0], [rm, 0, 0], [0.5 * rm, math.sqrt(3) / 2 * rm, 0]]
    out = ev(pos, [0, 0, 0], 50.0, W.swap_table_single(lam=lam))
    assert out["E"] == pytest.approx(3.0 * (lam - 1.0), abs=1e-9)


def test_lambda_zero_is_pure_pair_sum():
    s = W.small_reactive(N=120, density=0.3, seed=5)
    a = ev(s.pos, s.types, s.L, s.table.with_lambda(0.0))
    b = ev(s.pos, s.types, s.L, s.table.with_lambda(1.3))
    assert a["E3"] == 0.0
    assert a["E2"] == pytest.approx(b["E2"], rel=1e-14)
    assert b["E3"] > 0.0


def test_literal_triple_loops_match():
    rng = np.random.default_rng(7)
    tab = W.PairTable.empty(3)
    tab.set(0, 0, W.KIND_SWAP, 1.0, 1.0, 10, 1.5, 0.8)
    tab.set(0, 1, W.KIND_SWAP, 2.0, 0.9, 12, 1.4, 1.3)
    tab.set(1, 1, W.KIND_WCA, 1.0, 0.8, 6)
    tab.set(0, 2, W.KIND_WCA, 1.0, 1.0, 6)
    tab.set(1, 2, W.KIND_NONE)
    tab.set(2, 2, W.KIND_SWAP, 1.0, 1.0, 10, 1.5, 1.0)
    for trial in range(6):
        N = int(rng.integers(4, 16))
        pos = rng.uniform(-1.6, 1.6, size=(N, 3))
        ty = rng.integers(0, 3, size=N)
        e2, e3 = literal.literal_energy(pos, ty, 7.0, tab)
        out = ev(pos, ty, 7.0, tab)
        assert out["E2"] == pytest.approx(e2, rel=1e-12, abs=1e-12)
        assert out["E3"] == pytest.approx(e3, rel=1e-12, abs=1e-12)


# --------------------------------------------------------------------------
# derivatives: forces and virial against finite differences of the energy
# --------------------------------------------------------------------------

def _cluster_away_from_cuts(rng, N, table, L, box=1.9, guard=2e-4, triplets=True):
    """Random cluster with no pair within ``guard`` of any r_cut (E jumps there)
    and, if ``triplets``, at least two three-body terms."""
    while True:
        pos = rng.uniform(-box, box, size=(N, 3))
        ty = rng.integers(0, table.ntypes, size=N)
        d = swap_ref.min_image(pos[:, None, :], pos[None, :, :], np.full(3, L))
        r = np.sqrt(swap_ref.r2_canonical(d))
        rc = table.rcut[ty[:, None], ty[None, :]]
        iu = np.triu_indices(N, 1)
        if np.all(np.abs(r[iu] - rc[iu]) > guard) and np.min(r[iu]) > 0.75:
            if not triplets or swap_ref.evaluate(pos, ty, L, table.with_lambda(1.0),
                                                 scales=False)["n_triplets"] >= 2:
                return pos, ty


@pytest.mark.parametrize("lam", [0.0, 0.6, 1.0, 1.5])
def test_forces_are_minus_energy_gradient(lam):
    rng = np.random.default_rng(11)
    tab = W.PairTable.empty(2)
    tab.set(0, 0, W.KIND_SWAP, 1.0, 1.0, 10, 1.5, lam)
    tab.set(0, 1, W.KIND_WCA, 1.0, 0.9, 6)
    tab.set(1, 1, W.KIND_SWAP, 2.0, 0.8, 8, 1.2, 0.5 * lam)
    L = 12.0
    pos, ty = _cluster_away_from_cuts(rng, 9, tab, L, box=1.5)
    out = ev(pos, ty, L, tab)
    assert out["n_triplets"] > 0 or lam == 0.0
    h = 1e-6
    for m in range(pos.shape[0]):
        for a in range(3):
            p = pos.copy(); p[m, a] += h
            q = pos.copy(); q[m, a] -= h
            fd = -(swap_ref.energy(p, ty, L, tab) - swap_ref.energy(q, ty, L, tab)) / (2 * h)
            assert out["F"][m, a] == pytest.approx(fd, abs=2e-6 * (1 + abs(fd)))


def test_forces_sum_to_zero_and_no_torque():
    rng = np.random.default_rng(3)
    tab = W.swap_table_single(lam=0.7)
    pos, ty = _cluster_away_from_cuts(rng, 12, tab, 30.0, box=1.5)
    out = ev(pos, ty, 30.0, tab)
    assert out["n_triplets"] > 0
    assert np.abs(out["F"].sum(axis=0)).max() < 1e-9 * np.abs(out["F"]).max()
    torque = np.cross(pos, out["F"]).sum(axis=0)
    assert np.abs(torque).max() < 1e-9 * np.abs(out["F"]).max()


def test_virial_is_minus_strain_derivative():
    """W_ab = -dE/d(strain_ab) for an isolated cluster (eq. p3 bracket)."""
    rng = np.random.default_rng(5)
    tab = W.swap_table_single(lam=1.2)
    pos, ty = _cluster_away_from_cuts(rng, 10, tab, 40.0, box=1.6)
    out = ev(pos, ty, 40.0, tab)
    assert out["n_triplets"] > 0
    Wt = out["W_full"]
    h = 1e-7
    for a in range(3):
        for b in range(3):
            e = np.eye(3)
            e[a, b] += h
            ep = swap_ref.energy(pos @ e.T, ty, 40.0, tab)
            e[a, b] -= 2 * h
            em = swap_ref.energy(pos @ e.T, ty, 40.0, tab)
            fd = -(ep - em) / (2 * h)
            # x_a += h x_b  ->  -dE/dh = sum_m F_a x_b = W_ba
            assert Wt[b, a] == pytest.approx(fd, abs=1e-5 * (1 + abs(fd)))
    assert np.abs(Wt - Wt.T).max() < 1e-9 * (1 + np.abs(Wt).max())


def test_periodic_images_match_unwrapped_cluster():
    # a cluster straddling the box faces gives the same result as when centred
    rng = np.random.default_rng(9)
    tab = W.swap_table_single(lam=0.9)
    pos, ty = _cluster_away_from_cuts(rng, 10, tab, 9.0, box=1.6)
    a = ev(pos, ty, 9.0, tab)
    shifted = dynamics_ref.wrap(pos + 4.4, 9.0)[0]
    b = ev(shifted, ty, 9.0, tab)
    assert b["E"] == pytest.approx(a["E"], rel=1e-12)
    assert np.abs(a["F"] - b["F"]).max() < 1e-9 * (1 + np.abs(a["F"]).max())


# --------------------------------------------------------------------------
# bonds
# --------------------------------------------------------------------------

def test_bond_count_threshold_and_pair_kinds():
    rm2 = swap_ref.rmin2_canonical(1.0, 10)
    rm = math.sqrt(rm2)
    tab = two_type_table(1.0)
    # A-B just inside r_min: bonded; A-B just outside: not; A-A inside: not a swap pair
    pos = [[0, 0, 0], [rm * (1 - 1e-7), 0, 0],
           [5, 0, 0], [5 + rm * (1 + 1e-7), 0, 0],
           [-5, 0, 0], [-5 + 0.5 * rm, 0, 0]]
    ty = [0, 1, 0, 1, 0, 0]
    assert swap_ref.bond_count(pos, ty, 30.0, tab) == 1
    assert ev(pos, ty, 30.0, tab)["bonds"] == 1


def test_bond_partners_and_autocorrelation():
    # the bond autocorrelation of the swap test (Sec. 3.1): fraction of the bonds of time 0 whose
    # partner is unchanged at t.  Clusters: a bonded A-B dimer, a B bonded to two A (a triplet at
    # r_min), a free A, and an A-B bond across the periodic face.
    rm = math.sqrt(swap_ref.rmin2_canonical(1.0, 10))
    tab = two_type_table(1.0)
    L = 30.0
    pos = [[0, 0, 0], [0.9 * rm, 0, 0],                          # 0-1 dimer
           [8 - 0.9 * rm, 0, 0], [8, 0, 0], [8 + 0.9 * rm, 0, 0],  # 3 (B) bonded to 2 and 4
           [-8, 8, 8],                                            # free A
           [L / 2 - 0.3, -8, 0], [-L / 2 + 0.3, -8, 0]]           # A-B across the face
    ty = [0, 1, 0, 1, 0, 0, 0, 1]
    p = swap_ref.bond_partners(pos, ty, L, tab)
    assert list(p) == [1, 0, 3, -2, 3, -1, 7, 6]
    assert swap_ref.bond_count(pos, ty, L, tab) == 4
    # a swap: B 1 leaves A 0 for A 5 (moved next to it); the other bonds stay
    pos2 = [list(x) for x in pos]
    pos2[5] = [0.9 * rm + 0.9 * rm, 0, 0]
    pos2[0] = [-5, -5, -5]
    p2 = swap_ref.bond_partners(pos2, ty, L, tab)
    assert p2[1] == 5 and p2[0] == -1 and p2[5] == 1
    is_b = np.array(ty) == 1
    # B particles bonded at time 0: 1 (to 0), 7 (to 6); 3 has two bonds (-2) and is not counted
    assert swap_ref.bond_autocorrelation(p, p2, mask=is_b) == 0.5
    assert swap_ref.bond_autocorrelation(p, p, mask=is_b) == 1.0


def test_dumbbell_mixture_recipe():
    # the swap-test mixture of Sec. 3.1: A:B = 3:2 (600:400 at N = 1000), density 0.125, A-B swap term
    # with n = 100 and the chosen cutoff, A-A and B-B WCA
    s = W.dumbbell_mixture(N=1000, rcut=1.15, seed=3)
    assert np.bincount(s.types).tolist() == [600, 400]
    assert s.N / s.L ** 3 == pytest.approx(0.125, rel=1e-5)
    t = s.table
    assert t.kind[0, 1] == W.KIND_SWAP and t.n[0, 1] == 100 and t.rcut[0, 1] == 1.15
    assert t.kind[0, 0] == W.KIND_WCA and t.kind[1, 1] == W.KIND_WCA
    # v(1.15) for n = 100: about 3e-6 eps, far below the truncation of Lennard-Jones at 2.5 sigma
    v = 4.0 * ((1 / 1.15) ** 200 - (1 / 1.15) ** 100)
    assert -4e-6 < v < -3e-6


def test_generators_invariants():
    s = W.small_reactive(N=500, density=0.2, seed=1)
    assert s.pos.dtype == np.float32
    assert float(np.float32(s.L)) == s.L
    assert np.all(s.pos >= -0.5 * s.L) and np.all(s.pos < 0.5 * s.L)
    d = swap_ref.min_image(s.pos[:, None, :].astype(float), s.pos[None].astype(float), s.box)
    r = np.sqrt(swap_ref.r2_canonical(d))[np.triu_indices(s.N, 1)]
    assert r.min() > 0.8
    m = W.assembly_mixture(N=4000, lam=1.0, seed=2)
    assert m.N == 4000 and np.count_nonzero(m.types == 1) == 2000
    assert m.N / m.L ** 3 == pytest.approx(0.3, rel=1e-5)


# --------------------------------------------------------------------------
# random numbers and the integrator
# --------------------------------------------------------------------------

def test_philox_known_answers():
    rows = []
    with open(os.path.join(GOLD, "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                rows.append([int(x, 16) for x in line.split()])
    for r in rows:
        out = philox_ref.philox4x32_10(np.array([r[0:4]], np.uint64), np.array([r[4:6]], np.uint64))[0]
        assert [int(x) for x in out] == r[6:10]


def test_box_muller_normals_are_standard_normal():
    from scipy import stats
    z = philox_ref.thermostat_normals(1234, np.arange(40000), 17).ravel()
    assert abs(z.mean()) < 0.02 and abs(z.std() - 1) < 0.02
    assert stats.kstest(z, "norm").pvalue > 1e-3
    z2 = philox_ref.thermostat_normals(1234, np.arange(40000), 18).ravel()
    assert abs(np.corrcoef(z, z2)[0, 1]) < 0.02


def _ideal_gas(N=2000):
    tab = W.PairTable.empty(1)
    rng = np.random.default_rng(0)
    L = 20.0
    pos = W.wrap_fp32(rng.uniform(-10, 10, size=(N, 3)), L).astype(float)
    return pos, np.zeros(N, np.int32), L, tab


def test_langevin_equipartition_ideal_gas():
    pos, ty, L, tab = _ideal_gas()
    vel = np.zeros_like(pos)
    mass = np.array([2.0])
    kT = 0.7
    temps = []
    for step in range(60):
        out = dynamics_ref.baoab_step(pos, vel, ty, np.arange(len(ty)), L, tab, mass,
                                      dt=0.05, kT=kT, gamma=2.0, seed=99, step=step)
        pos, vel = out["pos"], out["vel"]
        if step >= 30:
            K = dynamics_ref.kinetic_tensor(vel, ty, mass)
            temps.append(K[:3].sum() / (3 * len(ty)))
    assert np.mean(temps) == pytest.approx(kT, rel=0.03)


def _nve_system():
    # n = 100, r_cut = 1.3: the truncation jump |v(1.3)| ~ 1.6e-11 eps (SI, Performance)
    tab = W.swap_table_single(epsilon=1.0, sigma=1.0, n=100, rcut=1.3, lam=1.0)
    s = W.small_reactive(N=64, density=0.125, seed=21, min_dist=1.0, table=tab, kT=0.03)
    return s


def test_nve_energy_error_is_second_order_and_reversible():
    """Velocity Verlet (gamma = 0): the energy error at a fixed time shrinks by
    4x when dt halves, and reversing the velocities retraces the path."""
    s = _nve_system()
    pos = s.pos.astype(float)
    vel = s.vel.astype(float)
    ty, tags, mass = s.types, s.tags, s.mass

    def total(p, v):
        return swap_ref.energy(p, ty, s.L, s.table) + 0.5 * np.sum(mass[ty][:, None] * v * v)

    def run(p, v, dt, n):
        for step in range(n):
            out = dynamics_ref.baoab_step(p, v, ty, tags, s.L, s.table, mass, dt, 0.0, 0.0, 1, step)
            p, v = out["pos"], out["vel"]
        return p, v

    E0 = total(pos, vel)
    errs = []
    for dt, n in ((4e-4, 25), (2e-4, 50), (1e-4, 100)):
        p, v = run(pos, vel, dt, n)
        errs.append(abs(total(p, v) - E0))
    assert errs[0] / errs[1] == pytest.approx(4.0, rel=0.05)
    assert errs[1] / errs[2] == pytest.approx(4.0, rel=0.05)
    p, v = run(pos, vel, 2e-4, 50)
    p, v = run(p, -v, 2e-4, 50)
    dp = swap_ref.min_image(pos, p, s.box)
    assert np.abs(dp).max() < 1e-9
    assert np.abs(v + vel).max() < 1e-7


def test_baoab_noise_is_keyed_by_tag_not_order():
    s = W.small_reactive(N=50, density=0.05, seed=4)
    pos, vel = s.pos.astype(float), s.vel.astype(float)
    a = dynamics_ref.baoab_step(pos, vel, s.types, s.tags, s.L, s.table, s.mass, 0.002, 0.1, 1.0, 7, 3)
    perm = np.random.default_rng(0).permutation(s.N)
    b = dynamics_ref.baoab_step(pos[perm], vel[perm], s.types[perm], s.tags[perm], s.L, s.table,
                                s.mass, 0.002, 0.1, 1.0, 7, 3)
    assert np.abs(a["pos"][perm] - b["pos"]).max() < 1e-12
    assert np.abs(a["vel"][perm] - b["vel"]).max() < 1e-10


# --------------------------------------------------------------------------
# second derivatives and parameter gradients
# --------------------------------------------------------------------------

@pytest.mark.parametrize("lam", [0.0, 0.7, 1.0, 1.4])
def test_hvp_matches_force_differences(lam):
    rng = np.random.default_rng(17)
    tab = W.PairTable.empty(2)
    tab.set(0, 0, W.KIND_SWAP, 1.0, 1.0, 10, 1.5, lam)
    tab.set(0, 1, W.KIND_WCA, 1.0, 0.9, 6)
    tab.set(1, 1, W.KIND_SWAP, 2.0, 0.8, 8, 1.2, 0.5 * lam)
    L = 12.0
    for _ in range(3):
        pos, ty = _cluster_away_from_cuts(rng, 9, tab, L, guard=1e-3)
        # keep swap pairs away from r_min too (u'' jumps there)
        P = swap_ref.interacting_pairs(pos, ty, L, tab)
        sw = P["kind"] == W.KIND_SWAP
        if np.any(np.abs(np.sqrt(P["r2"][sw]) - np.sqrt(P["rmin2"][sw])) < 1e-3):
            continue
        v = rng.standard_normal(pos.shape)
        Hv = adjoint_ref.hvp(pos, ty, L, tab, v)
        h = 1e-6
        Fp = swap_ref.evaluate(pos + h * v, ty, L, tab, scales=False)["F"]
        Fm = swap_ref.evaluate(pos - h * v, ty, L, tab, scales=False)["F"]
        fd = -(Fp - Fm) / (2 * h)
        assert np.abs(Hv - fd).max() < 1e-5 * (1 + np.abs(fd).max())
        w = rng.standard_normal(pos.shape)
        Hw = adjoint_ref.hvp(pos, ty, L, tab, w)
        assert np.sum(w * Hv) == pytest.approx(np.sum(v * Hw), rel=1e-10, abs=1e-10)
        t = np.tile(rng.standard_normal(3), (pos.shape[0], 1))
        assert np.abs(adjoint_ref.hvp(pos, ty, L, tab, t)).max() < 1e-9 * (1 + np.abs(Hv).max())


def test_param_grad_matches_energy_differences():
    rng = np.random.default_rng(23)
    tab = W.PairTable.empty(2)
    tab.set(0, 0, W.KIND_SWAP, 1.3, 1.0, 10, 1.5, 0.9)
    tab.set(0, 1, W.KIND_WCA, 1.0, 0.9, 6)
    tab.set(1, 1, W.KIND_SWAP, 2.0, 0.8, 8, 1.2, 1.2)
    L = 12.0
    pos, ty = _cluster_away_from_cuts(rng, 10, tab, L, guard=1e-3)
    g = adjoint_ref.param_grad(pos, ty, L, tab)
    for (a, b) in [(0, 0), (0, 1), (1, 1)]:
        for w, name in ((0, "epsilon"), (1, "sigma"), (2, "lam")):
            if w == 2 and tab.kind[a, b] != W.KIND_SWAP:
                continue
            p0 = float(getattr(tab, name)[a, b])
            h = 1e-6
            tp = tab.copy(); getattr(tp, name)[a, b] = getattr(tp, name)[b, a] = p0 + h
            tm = tab.copy(); getattr(tm, name)[a, b] = getattr(tm, name)[b, a] = p0 - h
            fd = (swap_ref.energy(pos, ty, L, tp) - swap_ref.energy(pos, ty, L, tm)) / (2 * h)
            assert g[a, b, w] == pytest.approx(fd, rel=1e-6, abs=1e-7)


def test_param_grad_identities_single_entry():
    s = W.small_reactive(N=150, density=0.3, seed=8, table=W.swap_table_single(epsilon=2.0, lam=1.3))
    out = ev(s.pos, s.types, s.L, s.table)
    g = adjoint_ref.param_grad(s.pos.astype(float), s.types, s.L, s.table)[0, 0]
    assert g[2] == pytest.approx(out["E3"] / 1.3, rel=1e-12)
    assert g[0] == pytest.approx(out["E"] / 2.0, rel=1e-12)
    # dE/dsigma = Tr W / sigma at fixed r_cut (all terms are swap terms here)
    assert g[1] == pytest.approx(out["W"][:3].sum() / 1.0, rel=1e-9)


def test_force_param_vjp_identities_single_entry():
    # one swap entry: F is linear in eps (pair and three-body parts alike) and the
    # three-body force is linear in lambda, so a . dF/deps = a . F / eps and
    # a . dF/dlambda = a . (F(lambda) - F(0)) / lambda
    s = W.small_reactive(N=60, density=0.35, seed=9, table=W.swap_table_single(epsilon=2.0, lam=1.3))
    rng = np.random.default_rng(4)
    adj = rng.standard_normal((s.N, 3))
    x = s.pos.astype(float)
    out = adjoint_ref.force_param_vjp(x, s.types, s.L, s.table, adj)[0, 0]
    F = ev(x, s.types, s.L, s.table)["F"]
    t0 = s.table.copy()
    t0.lam[:] = 0.0
    F0 = ev(x, s.types, s.L, t0)["F"]
    assert out[0] == pytest.approx(np.sum(adj * F) / 2.0, rel=1e-7)
    assert out[2] == pytest.approx(np.sum(adj * (F - F0)) / 1.3, rel=1e-7)
    assert abs(np.sum(adj * (F - F0))) > 1e-3 * abs(np.sum(adj * F))   # the three-body part is present


def test_soft_bonds_gradient_and_bond_limit():
    rng = np.random.default_rng(31)
    tab = W.swap_table_single(lam=0.8)
    L = 12.0
    pos, ty = _cluster_away_from_cuts(rng, 12, tab, L, guard=1e-3)
    B, g = adjoint_ref.soft_bonds(pos, ty, L, tab)
    h = 1e-6
    for m in range(pos.shape[0]):
        for a in range(3):
            xp, xm = pos.copy(), pos.copy()
            xp[m, a] += h
            xm[m, a] -= h
            fd = (adjoint_ref.soft_bonds(xp, ty, L, tab)[0] - adjoint_ref.soft_bonds(xm, ty, L, tab)[0]) / (2 * h)
            assert g[m, a] == pytest.approx(fd, rel=1e-6, abs=1e-8)
    # three particles: one bonded pair (r < r_min), one pair beyond r_cut
    rm = 2.0 ** 0.1
    tri = np.array([[0.0, 0.0, 0.0], [0.9 * rm, 0.0, 0.0], [0.0, 3.0, 0.0]])
    b3, _ = adjoint_ref.soft_bonds(tri, np.zeros(3, np.int32), L, tab)
    assert b3 == 1.0 and swap_ref.bond_count(tri, np.zeros(3, np.int32), L, tab) == 1


# --------------------------------------------------------------------------
# FENE springs
# --------------------------------------------------------------------------

def test_fene_forces_are_minus_energy_gradient_and_closed_form():
    from oracle import fene_ref
    rng = np.random.default_rng(40)
    L = 10.0
    # a chain of 6 beads along x that crosses the boundary between beads 2 and 3
    x = np.zeros((6, 3))
    x[:, 0] = L / 2 - 2.0 + 0.95 * np.arange(6)
    x += rng.uniform(-0.1, 0.1, x.shape)
    x[:, 0] = (x[:, 0] + L / 2) % L - L / 2
    bonds = np.full((6, 2), -1)
    for k in range(5):
        bonds[k, 1], bonds[k + 1, 0] = k + 1, k
    out = fene_ref.evaluate(x, L, bonds, 30.0, 1.5)
    h = 1e-6
    for m in range(6):
        for a in range(3):
            xp, xm = x.copy(), x.copy()
            xp[m, a] += h
            xm[m, a] -= h
            fd = (fene_ref.evaluate(xp, L, bonds, 30.0, 1.5)["E"] - fene_ref.evaluate(xm, L, bonds, 30.0, 1.5)["E"]) / (2 * h)
            assert out["F"][m, a] == pytest.approx(-fd, rel=1e-6, abs=1e-6)
    # one bond at r = 1.2: |F| = K r / (1 - r^2/R0^2) = 30 * 1.2 / 0.36 = 100
    two = fene_ref.evaluate(np.array([[0.0, 0, 0], [1.2, 0, 0]]), L, np.array([[1, -1], [-1, 0]]), 30.0, 1.5)
    assert two["F"][0, 0] == pytest.approx(100.0, rel=1e-12)
    assert two["W"][0] == pytest.approx(-100.0 * 1.2, rel=1e-12)
    assert sum(two["pe"]) == pytest.approx(two["E"], rel=1e-14)


def test_fene_plus_wca_bond_length_is_kremer_grest():
    # K = 30, R0 = 1.5, WCA eps = sigma = 1: the bond potential has its minimum at about
    # 0.96 sigma (Kremer & Grest 1990; the thermal mean bond length at kT = 1 is ~0.97)
    from scipy.optimize import minimize_scalar
    from oracle import fene_ref
    tab = W.PairTable.empty(1)
    tab.set(0, 0, W.KIND_WCA, 1.0, 1.0, 6)
    b = np.array([[1, -1], [-1, 0]])

    def U(r):
        x = np.array([[0.0, 0.0, 0.0], [r, 0.0, 0.0]])
        return fene_ref.evaluate(x, 20.0, b, 30.0, 1.5)["E"] + swap_ref.energy(x, np.zeros(2, np.int32), 20.0, tab)
    res = minimize_scalar(U, bounds=(0.8, 1.12), method="bounded", options={"xatol": 1e-10})
    assert abs(res.x - 0.961) < 0.002


# --------------------------------------------------------------------------
# the C brute force and the numpy evaluator agree
# --------------------------------------------------------------------------

def test_brute_force_matches_numpy(brute_lib):
    s = W.assembly_mixture(N=3000, lam=0.5, seed=12, density=0.3)
    a = ev(s.pos, s.types, s.L, s.table)
    b = brute_lib.evaluate(s.pos, s.types, s.L, s.table)
    assert a["bonds"] == b["bonds"]
    assert a["n_triplets"] == b["n_triplets"]
    assert b["E"] == pytest.approx(a["E"], rel=1e-12)
    assert np.abs(a["F"] - b["F"]).max() < 1e-10 * (1 + np.abs(a["F"]).max())
    assert np.abs(a["W"] - b["W"]).max() < 1e-10 * (1 + np.abs(a["W"]).max())
    idx = np.arange(0, s.N, 37)
    c = brute_lib.forces_subset(s.pos, s.types, s.L, s.table, idx)
    assert np.abs(c["F"] - a["F"][idx]).max() < 1e-10 * (1 + np.abs(a["F"]).max())
    deg = swap_ref.bond_degree(s.pos, s.types, s.L, s.table)
    assert np.array_equal(c["degree"], deg[idx])


def test_per_particle_energies_sum_to_total():
    # the split itself is a reading (pair halves, triplet to its centre); its sum is fixed
    s = W.small_reactive(N=200, density=0.35, seed=13, table=W.swap_table_single(lam=0.6))
    out = ev(s.pos, s.types, s.L, s.table)
    assert out["n_triplets"] > 0
    assert out["pe"].sum() == pytest.approx(out["E"], rel=1e-12)
    # a lone triplet: the three-body energy sits on the centre
    rm = 2.0 ** 0.1
    o = ev([[-rm, 0, 0], [0, 0, 0], [1.2, 0, 0]], [0, 1, 0], 50.0, two_type_table(1.0))
    assert o["pe"][1] - 0.5 * (o["E2"]) == pytest.approx(o["E3"], abs=1e-12)


def test_stress_autocorrelation_pins():
    # G(t) = V/kT < avg over xy, xz, yz of sigma(t0) sigma(t0 + t) > (the autocorrelation method after
    # eq. p3), sigma_ab = -(K_ab + W_ab)/V
    from oracle import observables_ref as O
    V, kT, T = 8.0, 0.5, 12
    lags = np.arange(T)
    # constant shear virial in xy, sigma_xy = -c, the other components zero: V/kT c^2/3 at every lag
    rows = np.zeros((T, 13))
    c = 0.7
    rows[:, 4] = c * V
    assert np.allclose(O.stress_autocorrelation(rows, V, kT, T - 1), V / kT * c * c / 3, rtol=1e-14)
    # alternating kinetic shear term in xz, sigma_xz = -a (-1)^t: V/kT a^2 (-1)^t / 3
    rows = np.zeros((T, 13))
    a = 0.3
    rows[:, 11] = a * V * (-1.0) ** lags
    assert np.allclose(O.stress_autocorrelation(rows, V, kT, T - 1), V / kT * a * a * (-1.0) ** lags / 3,
                       rtol=1e-14)
    rng = np.random.default_rng(5)
    # the energy and the diagonal components do not enter
    rows = rng.standard_normal((T, 13))
    rows[:, [4, 5, 6, 10, 11, 12]] = 0.0
    assert np.all(O.stress_autocorrelation(rows, V, kT, T - 1) == 0.0)
    # kinetic and virial parts add into one stress
    rows = rng.standard_normal((T, 13))
    merged = rows.copy()
    merged[:, 4:7] += merged[:, 10:13]
    merged[:, 10:13] = 0.0
    assert np.allclose(O.stress_autocorrelation(rows, V, kT, 5), O.stress_autocorrelation(merged, V, kT, 5),
                       rtol=1e-12)
    # every origin is averaged: reversing the series in time leaves G unchanged
    G = O.stress_autocorrelation(rows, V, kT, T - 1)
    assert np.allclose(G, O.stress_autocorrelation(rows[::-1], V, kT, T - 1), rtol=1e-12)
    # G(0) is V/kT times the mean square shear stress
    s = -(rows[:, 4:7] + rows[:, 10:13]) / V
    assert np.isclose(G[0], V / kT * np.mean(s * s), rtol=1e-12)
    with pytest.raises(ValueError):
        O.stress_autocorrelation(rows, V, kT, T)


def test_partner_counts_pin():
    # bonded at 0, unchanged (the bond autocorrelation's numerator) and swapped (a bonded site whose
    # single partner is now another particle); a broken bond and a site with several bonds are neither
    from oracle import observables_ref as O
    p0 = [1, 0, 3, -2, 3, -1, 7, 6]
    pt = [5, -1, 3, -2, -2, 1, 7, 6]
    assert O.partner_counts(p0, pt) == (6, 3, 1)
    odd = np.arange(8) % 2 == 1
    assert O.partner_counts(p0, pt, odd) == (2, 1, 0)
    b, u, _ = O.partner_counts(p0, pt, odd)
    assert swap_ref.bond_autocorrelation(p0, pt, mask=odd) == u / b


def test_planar_step_pin():
    # dim 2 drops only the z noise: with every particle at z = 0 and vz = 0 the z force components
    # vanish, so the step keeps z and vz exactly, and the positions in the plane are the 3D step's
    # (whose z noise does move z)
    s = W.planar_reactive(N=60, L=12.0, Lz=6.0, seed=5, min_dist=0.9)
    tags = np.arange(s.N)
    a = dynamics_ref.baoab_step(s.pos, s.vel, s.types, tags, s.box, s.table, s.mass, 0.002, 1.0, 1.0, 7, 3, dim=2)
    b = dynamics_ref.baoab_step(s.pos, s.vel, s.types, tags, s.box, s.table, s.mass, 0.002, 1.0, 1.0, 7, 3, dim=3)
    assert np.all(a["F_old"][:, 2] == 0.0) and np.all(a["F"][:, 2] == 0.0)
    assert np.all(a["pos"][:, 2] == 0.0) and np.all(a["vel"][:, 2] == 0.0)
    assert np.any(b["pos"][:, 2] != 0.0)
    assert np.array_equal(a["pos"][:, :2], b["pos"][:, :2])
    assert np.any(np.abs(a["F_old"][:, :2]) > 0.0)   # the configuration does interact


def _two_bodies(p0, p1, th, v, w, L=(60.0, 60.0, 8.0), eps_patch=10.0):
    # a trifunctional body (3 patches) and a difunctional one (2 patches), tags 0, 1 and 2..6
    off = np.array([[0.5 * np.cos(a), 0.5 * np.sin(a)] for a in (0.0, 2 * np.pi / 3, 4 * np.pi / 3, 0.0, np.pi)])
    bodies = dict(centre=np.array([0, 1]), first=np.array([0, 3, 5]), member=np.arange(2, 7), offset=off,
                  inertia=np.array([0.125, 0.125]))
    pos = np.zeros((7, 3))
    pos[0, :2], pos[1, :2] = p0, p1
    th = np.asarray(th, dtype=np.float64)
    pos = rigid_ref.place(pos, bodies, th, L)
    vel = np.zeros((7, 3))
    vel[0, :2], vel[1, :2] = v[0], v[1]
    types = np.array([0, 1, 2, 2, 2, 2, 2])
    return pos, vel, th, np.asarray(w, dtype=np.float64), types, bodies, W.patchy_table(eps_patch=eps_patch)


def test_rigid_free_body_pin():
    # bodies far apart: no force, so gamma = 0 steps move and turn them uniformly
    L = (60.0, 60.0, 8.0)
    pos, vel, th, w, ty, bodies, tab = _two_bodies((-10.0, 0.0), (10.0, 3.0), (0.3, -2.0), ((0.7, -0.2), (-0.1, 0.4)),
                                                  (1.5, -3.0), L)
    x, v, t, o = pos, vel, th, w
    dt, K = 0.01, 40
    for k in range(K):
        out = rigid_ref.step(x, v, t, o, ty, bodies, L, tab, np.ones(3), dt, 0.0, 0.0, 1, k)
        x, v, t, o = out["pos"], out["vel"], out["theta"], out["omega"]
    want_th = np.mod(th + K * dt * w + np.pi, 2 * np.pi) - np.pi
    assert np.allclose(t, want_th, atol=1e-12) and np.allclose(o, w, atol=0)
    assert np.allclose(x[:2, :2], pos[:2, :2] + K * dt * vel[:2, :2], atol=1e-12)
    assert np.allclose(x, rigid_ref.place(x, bodies, want_th, L), atol=1e-12)


def test_rigid_collision_conserves_energy_and_angular_momentum():
    # two bodies whose facing patches bind, at gamma = 0: energy to O(dt^2), angular momentum about
    # the origin to rounding (every force of the potential is central, so it exerts no net torque)
    L = (60.0, 60.0, 8.0)
    pos, vel, th, w, ty, bodies, tab = _two_bodies((-0.58, 0.0), (0.58, 0.03), (0.0, np.pi),
                                                  ((0.3, 0.1), (-0.3, 0.0)), (0.5, -0.2), L)
    m = np.ones(3)

    def energy(x, v, o):
        kt, kr = rigid_ref.kinetic(v, o, ty, bodies, m)
        return kt + kr + swap_ref.evaluate(x, ty, L, tab, scales=False)["E"]

    e0, l0 = energy(pos, vel, w), rigid_ref.angular_momentum(pos, vel, w, ty, bodies, m)
    assert abs(swap_ref.evaluate(pos, ty, L, tab, scales=False)["E"]) > 0.1   # the patches interact
    x, v, t, o = pos, vel, th, w
    de = 0.0
    for k in range(1000):
        out = rigid_ref.step(x, v, t, o, ty, bodies, L, tab, m, 1e-5, 0.0, 0.0, 1, k)
        x, v, t, o = out["pos"], out["vel"], out["theta"], out["omega"]
        de = max(de, abs(energy(x, v, o) - e0))
    assert de < 2e-3 * abs(e0), (de, e0)
    assert abs(rigid_ref.angular_momentum(x, v, o, ty, bodies, m) - l0) < 1e-10
