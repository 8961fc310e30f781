"""Batches of independent replicas on the GPU, through the batch C ABI.

Every replica of a batch is checked against the FP64 oracle on its own, and
against the same system run alone through the single-system entry points
(bit for bit where the two runs take the same list builds).
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import dynamics_ref, swap_ref
from parity_util import assert_energy, assert_forces, assert_pe, assert_virial

pytestmark = pytest.mark.gpu


def _mixed_replicas():
    """Uneven replicas: sizes below, at and above one wavefront, several tables and boxes."""
    reps = []
    specs = [(40, 0.2, 0.0, 0.0), (64, 0.3, 0.7, 0.3), (65, 0.25, 1.0, 0.0), (1500, 0.3, 1.5, 0.5),
             (777, 0.4, 0.4, 0.2), (3000, 0.2, 1.0, 0.1)]
    rng = np.random.default_rng(77)
    for k, (n, rho, lam, finert) in enumerate(specs):
        L = W.fp32_box(n, rho)
        L = max(L, float(np.float32(8.0)))
        tab = W.PairTable.empty(2)
        tab.set(0, 0, W.KIND_SWAP, 1.0, 1.0, 10, 1.5, lam)
        tab.set(0, 1, W.KIND_WCA, 1.0, 1.0, 6)
        tab.set(1, 1, W.KIND_WCA, 1.0, 1.0, 6)
        n_inert = int(round(n * finert))
        pos, types = W.rsa_positions(rng, L, [n - n_inert, n_inert], np.full((2, 2), 0.95))
        vel = W.maxwell_velocities(rng, types, np.ones(2), 0.1)
        reps.append(W.System(pos=pos, types=types, L=L, table=tab, mass=np.ones(2), vel=vel, name=f"r{k}"))
    return reps


def _batch(reps, **kw):
    from paper_1912_08569_amd import Batch
    return Batch(reps, **kw)


def test_layout_aligns_every_replica_to_a_wavefront():
    reps = _mixed_replicas()
    B = _batch(reps)
    n = np.array([s.N for s in reps])
    assert np.all(B.offsets[:-1] % 64 == 0)
    assert np.array_equal(np.diff(B.offsets), 64 * ((n + 63) // 64))
    assert B.n_slots == B.offsets[-1]


@pytest.mark.parametrize("form", ["walk", "sums"])
def test_batch_forces_match_oracle_per_replica(form):
    reps = _mixed_replicas()
    B = _batch(reps)
    B.set_step_form(form)
    F, ev = B.compute_forces()
    bonds = B.bond_count()
    torch.cuda.synchronize()
    evh = ev.cpu().numpy()
    for r, s in enumerate(reps):
        xyz, _, _, ty = B.state_by_tag(r)
        ref = swap_ref.evaluate(xyz, ty, s.L, s.table)
        Fg = B.by_tag(F, r)
        assert_forces(Fg, ref)
        assert_pe(Fg[:, 3], ref)
        assert_energy(evh[r, 0], ref)
        assert_virial(evh[r, 1:7], ref)
        assert int(bonds[r]) == ref["bonds"], f"replica {r}"


@pytest.mark.parametrize("form", ["walk", "sums"])
def test_batch_replica_equals_single_system_bitwise(form):
    # wide skin: one list build for the whole run in both, so every sum runs in the same order
    reps = _mixed_replicas()
    seeds = [1000 + 17 * r for r in range(len(reps))]
    B = _batch(reps, r_buff=0.9, seeds=seeds)
    B.set_step_form(form)
    cfg = B.integrator(dt=0.002, kT=0.1, gamma=1.0, seed=0)
    rb = B.run(40, cfg, step0=3, log_period=10)
    assert rb.stats.rebuilds == 1 and rb.stats.rollbacks == 0
    from paper_1912_08569_amd import System
    for r, s in enumerate(reps):
        S = System.from_workload(s, r_buff=0.9)
        S.set_step_form(form)
        c1 = S.integrator(dt=0.002, kT=0.1, gamma=1.0, seed=seeds[r])
        rs = S.run(40, c1, step0=3, log_period=10)
        assert rs.stats.rebuilds == 1
        xa, va, ia, _ = S.state_by_tag()
        xb, vb, ib, _ = B.state_by_tag(r)
        assert np.array_equal(xa, xb) and np.array_equal(va, vb) and np.array_equal(ia, ib), f"replica {r}"
        assert np.array_equal(rs.ev, rb.ev[:, r, :]), f"replica {r} logs"
        assert np.array_equal(rs.bonds, rb.bonds[:, r]), f"replica {r} bonds"


def test_batch_graphs_and_direct_launches_agree_bitwise():
    reps = _mixed_replicas()
    A = _batch(reps, seeds=range(6))
    Bb = _batch(reps, seeds=range(6))
    cfg = A.integrator(dt=0.002, kT=0.1, gamma=1.0, seed=0)
    ra = A.run(300, cfg, log_period=50, use_graph=True)
    rb = Bb.run(300, cfg, log_period=50, use_graph=False)
    assert ra.stats.rebuilds == rb.stats.rebuilds and ra.stats.rebuilds > 1
    for r in range(len(reps)):
        xa, va, ia, _ = A.state_by_tag(r)
        xb, vb, ib, _ = Bb.state_by_tag(r)
        assert np.array_equal(xa, xb) and np.array_equal(va, vb) and np.array_equal(ia, ib)
    assert np.array_equal(ra.ev, rb.ev) and np.array_equal(ra.bonds, rb.bonds)


def test_batch_fused_step_matches_oracle_step():
    reps = _mixed_replicas()
    seeds = [5 + r for r in range(len(reps))]
    B = _batch(reps, seeds=seeds)
    B.build()
    before = [B.state_by_tag(r) for r in range(len(reps))]
    cfg = B.integrator(dt=0.002, kT=0.1, gamma=1.0, seed=0)
    B.run(1, cfg, step0=41, use_graph=False)
    for r, s in enumerate(reps):
        x0, v0, _, ty = before[r]
        x1, v1, img, _ = B.state_by_tag(r)
        ref = dynamics_ref.baoab_step(x0, v0, ty, np.arange(s.N), s.L, s.table, s.mass, 0.002, 0.1, 1.0,
                                      seeds[r], 41)
        e0 = swap_ref.evaluate(x0, ty, s.L, s.table)
        e1 = swap_ref.evaluate(ref["pos"], ty, s.L, s.table)
        m = s.mass[ty][:, None]
        c2 = np.sqrt((1 - np.exp(-2 * 0.002)) * 0.1 / m)
        vscale = np.abs(v0) + 4.0 * c2 + 0.002 * (e0["A_F"] + e1["A_F"])[:, None] / m + np.abs(ref["vel"])
        assert np.all(np.abs(v1 - ref["vel"]) <= 2e-5 * vscale + 1e-7), f"replica {r} velocities"
        dx = np.abs(swap_ref.min_image(ref["pos"], x1.astype(np.float64), s.box))
        ulp = np.abs(np.nextafter(np.abs(ref["pos"]).astype(np.float32), np.float32(np.inf))
                     - np.abs(ref["pos"]).astype(np.float32)).astype(np.float64)
        assert np.all(dx <= 4 * ulp + 0.002 * 2e-5 * vscale), f"replica {r} positions"
        assert np.array_equal(img, ref["image"])


def test_batch_long_run_ends_on_oracle_values():
    reps = _mixed_replicas()
    B = _batch(reps, seeds=range(10, 16))
    cfg = B.integrator(dt=0.002, kT=0.1, gamma=1.0, seed=0)
    rb = B.run(800, cfg, log_period=200)
    assert rb.stats.steps_done == 800 and rb.stats.rebuilds > 1
    for r, s in enumerate(reps):
        x, _, _, ty = B.state_by_tag(r)
        ref = swap_ref.evaluate(x, ty, s.L, s.table)
        assert int(rb.bonds[-1, r]) == ref["bonds"]
        assert abs(rb.ev[-1, r, 0] - ref["E"]) <= 1e-5 * ref["A_E"]


def test_single_replica_batch_is_the_system():
    s = W.small_reactive(N=1000, density=0.2, seed=1001, table=W.swap_table_single(lam=1.0), kT=0.1)
    from paper_1912_08569_amd import System
    B = _batch([s], seeds=[9], r_buff=0.6)
    S = System.from_workload(s, r_buff=0.6, step_form="walk")   # the batch's default form
    cfg = B.integrator(dt=0.002, kT=0.1, gamma=1.0, seed=9)
    rb = B.run(40, cfg, log_period=10)
    rs = S.run(40, cfg, log_period=10)
    # one replica: the batch rebuilds exactly when the system alone does
    assert rb.stats.rebuilds == rs.stats.rebuilds and rb.stats.rollbacks == rs.stats.rollbacks
    assert np.array_equal(S.state_by_tag()[0], B.state_by_tag(0)[0])
    assert np.array_equal(S.state_by_tag()[1], B.state_by_tag(0)[1])
    assert np.array_equal(rs.ev, rb.ev[:, 0, :]) and np.array_equal(rs.bonds, rb.bonds[:, 0])


def test_full_replica_set_parity_on_samples():
    # the 256-replica workload (N ~ logU[500, 20000]): per-replica energies and bonds of
    # a sample of replicas against the oracle, every replica's bond count against its list
    reps = W.replica_set()
    B = _batch(reps, seeds=range(256))
    F, ev = B.compute_forces()
    bonds = B.bond_count()
    evh = ev.cpu().numpy()
    rng = np.random.default_rng(3)
    for r in sorted(rng.choice(len(reps), 6, replace=False).tolist()) + [int(np.argmin([s.N for s in reps]))]:
        s = reps[r]
        xyz, _, _, ty = B.state_by_tag(r)
        ref = swap_ref.evaluate(xyz, ty, s.L, s.table)
        assert_forces(B.by_tag(F, r), ref)
        assert_energy(evh[r, 0], ref)
        assert_virial(evh[r, 1:7], ref)
        assert int(bonds[r]) == ref["bonds"]


def test_batch_list_overflow_mid_run_resumes_exactly():
    # lists sized to the first build's longest list overflow during the run; the driver returns the
    # state at the failed build with the steps done, the batch grows its lists and resumes (the last
    # half kick owed): with the rebuild threshold at the stale threshold the result equals a batch with
    # room to spare, bit for bit
    # (an even start, every pair 1.1 sigma apart, has short lists that bonding then lengthens)
    reps = [W.small_reactive(N=4000, density=0.35, seed=sd, kT=0.5, min_dist=1.1) for sd in (47, 48)]
    probe = _batch(reps, k_max=64)
    probe.build()
    kmax0 = int(((probe.nn & 0xFFFF) + (probe.nn >> 16)).max().item())
    A = _batch(reps, k_max=kmax0, seeds=[1, 2])
    B = _batch(reps, k_max=64, seeds=[1, 2])
    for X in (A, B):
        X.set_step_form("walk")
    cfg = A.integrator(dt=0.002, kT=0.5, gamma=1.0, seed=0)
    A.run(800, cfg, soft_frac=1.0)
    B.run(800, cfg, soft_frac=1.0)
    assert A.k_max > kmax0
    for r in range(len(reps)):
        assert all(np.array_equal(x, y) for x, y in zip(A.state_by_tag(r), B.state_by_tag(r))), f"replica {r}"


def test_partial_rebuilds_keep_valid_lists_and_match_oracle():
    # per-replica rebuilds: a build re-lists only the replicas that crossed (or neared) the rebuild
    # threshold; the others keep their order, lists and path lengths.  After a long run every replica's
    # current list must still hold every pair inside the cutoff: forces from the lists in place (no
    # rebuild) against the oracle, bonds exact, and every path length below the stale threshold.
    # (margin 1: only the replicas that crossed are rebuilt, the most partial builds)
    reps = _mixed_replicas()
    B = _batch(reps, seeds=range(20, 26), r_buff=0.3, rebuild_margin=1.0)
    cfg = B.integrator(dt=0.002, kT=0.1, gamma=1.0, seed=0)
    rb = B.run(1200, cfg, log_period=300)
    n_all = int(sum(s.N for s in reps))
    st = rb.stats
    assert st.steps_done == 1200 and st.rebuilds > 2
    assert 0 < st.particles_rebuilt < st.rebuilds * n_all, "every build re-listed every replica"
    assert B.vel[:, 3].max().item() <= 0.5 * 0.3 + 1e-6
    F, ev = B.compute_forces()
    bonds = B.bond_count()
    evh = ev.cpu().numpy()
    for r, s in enumerate(reps):
        xyz, _, _, ty = B.state_by_tag(r)
        ref = swap_ref.evaluate(xyz, ty, s.L, s.table)
        assert_forces(B.by_tag(F, r), ref)
        assert_energy(evh[r, 0], ref)
        assert int(bonds[r]) == ref["bonds"], f"replica {r}"


def test_zero_margin_rebuilds_every_replica():
    reps = _mixed_replicas()
    B = _batch(reps, seeds=range(6), rebuild_margin=0.0)
    cfg = B.integrator(dt=0.002, kT=0.1, gamma=1.0, seed=0)
    rb = B.run(300, cfg, log_period=100)
    n_all = int(sum(s.N for s in reps))
    assert rb.stats.rebuilds > 1 and rb.stats.particles_rebuilt == rb.stats.rebuilds * n_all
