"""Dynamics on the GPU: the fused step against the oracle's BAOAB step, the
chunked driver (graphs, rollbacks, rebuilds), energy conservation and the
Langevin temperature.  All calls go through the C ABI."""
import numpy as np
import pytest
import torch

import workloads as W
from paper_1912_08569_amd import _lib as rcl
from oracle import dynamics_ref, swap_ref

pytestmark = pytest.mark.gpu


def _system(s, **kw):
    from paper_1912_08569_amd import System
    return System.from_workload(s, **kw)


def _ulp32(x):
    x = np.abs(np.asarray(x, dtype=np.float32))
    return (np.nextafter(x, np.float32(np.inf)) - x).astype(np.float64)


def _one_step_check(s, kind, dt, kT, gamma, seed, step, form="walk", dim=3):
    S = _system(s)
    S.set_step_form(form)
    S.build()
    x0, v0, _, ty = S.state_by_tag()
    cfg = S.integrator(kind=kind, dt=dt, kT=kT, gamma=gamma, seed=seed, dim=dim)
    S.run(1, cfg, step0=step, use_graph=False)
    x1, v1, img, _ = S.state_by_tag()
    ref = dynamics_ref.baoab_step(x0, v0, ty, np.arange(s.N), s.L, s.table, s.mass, dt, kT,
                                  gamma if kind == "langevin" else 0.0, seed, step, dim=dim)
    if dim == 2:   # the plane is kept exactly
        assert np.all(x1[:, 2] == x0[:, 2]) and np.all(v1[:, 2] == 0.0)
    e0 = swap_ref.evaluate(x0, ty, s.L, s.table)
    e1 = swap_ref.evaluate(ref["pos"], ty, s.L, s.table)
    m = s.mass[ty][:, None]
    c2 = np.sqrt((1 - np.exp(-2 * gamma * dt)) * kT / m) if kind == "langevin" else 0.0 * m
    vscale = (np.abs(v0) + 4.0 * c2 + dt * (e0["A_F"] + e1["A_F"])[:, None] / m
              + np.abs(ref["vel"]))
    dv = np.abs(v1 - ref["vel"])
    assert np.all(dv <= 2e-5 * vscale + 1e-7), f"velocity error {np.max(dv / (vscale + 1e-30)):.3e}"
    dx = np.abs(swap_ref.min_image(ref["pos"], x1.astype(np.float64), s.box))
    xtol = 4 * _ulp32(ref["pos"]) + dt * 2e-5 * vscale
    assert np.all(dx <= xtol), f"position error {np.max(dx - xtol):.3e} over tolerance"
    assert np.array_equal(img, ref["image"])
    return float(dx.max())


@pytest.mark.parametrize("kind", ["langevin", "nve"])
def test_fused_step_matches_oracle_small(kind):
    s = W.small_reactive(N=1000, density=0.2, seed=1001, table=W.swap_table_single(lam=0.7))
    _one_step_check(s, kind, 0.002, 0.1, 1.0, 2001, 17)


@pytest.mark.parametrize("kind", ["langevin", "nve"])
def test_planar_step_matches_oracle(kind):
    # the paper's 2d box (side 39.63, 1000 particles, kT 1): integrator dim 2
    s = W.planar_reactive(N=1000, seed=1012)
    _one_step_check(s, kind, 0.001, 1.0, 1.0, 2012, 31, dim=2)


def test_planar_run_stays_in_the_plane():
    from paper_1912_08569_amd import RcError, api
    s = W.planar_reactive(N=1000, seed=1013)
    S = _system(s)
    with pytest.raises(RcError):
        S.run(1, api.integrator(dt=0.001, kT=1.0, gamma=1.0, seed=5, mass=list(S.mass), dim=4))
    cfg = S.integrator(dt=0.001, kT=1.0, gamma=1.0, seed=5, dim=2)
    res = S.run(3000, cfg, log_period=0)
    assert res.stats.rebuilds >= 1
    x, v, img, ty = S.state_by_tag()
    assert np.all(x[:, 2] == 0.0) and np.all(v[:, 2] == 0.0) and np.all(img[:, 2] == 0)
    # equipartition in the plane: <m (vx^2 + vy^2)> = 2 kT (2000 degrees of freedom: ~3 % scatter)
    ke2 = float(np.mean(s.mass[ty] * (v[:, 0].astype(np.float64) ** 2 + v[:, 1].astype(np.float64) ** 2)))
    assert abs(ke2 / 2.0 - 1.0) < 0.12, ke2


@pytest.mark.parametrize("form", ["walk", "sums"])
def test_fused_step_unequal_pair_lambdas(form):
    _one_step_check(W.unequal_lambda_mixture(N=3000, seed=62), "langevin", 0.002, 0.1, 1.0, 5, 7, form=form)


def test_fused_step_matches_oracle_mixture():
    s = W.assembly_mixture(N=20000, lam=1.0, seed=1003, kT=0.05)
    _one_step_check(s, "langevin", 0.001, 0.05, 1.0, 2003, 123456789)


@pytest.mark.parametrize("lam", [0.3, 1.0])
def test_fused_step_sums_form_matches_oracle(lam):
    # dense reactive system (many partners per centre): the two-pass form of the step
    s = W.small_reactive(N=3000, density=0.5, seed=1010, min_dist=0.85, table=W.swap_table_single(lam=lam))
    _one_step_check(s, "langevin", 0.002, 0.1, 1.0, 2010, 77, form="sums")
    _one_step_check(s, "nve", 0.002, 0.0, 0.0, 2010, 78, form="walk")


def test_sums_form_graph_and_direct_launches_agree_bitwise():
    s = W.small_reactive(N=4000, density=0.4, seed=52, table=W.swap_table_single(lam=0.5), kT=0.1)
    A, B = _system(s), _system(s)
    A.set_step_form("sums")
    B.set_step_form("sums")
    cfg = A.integrator(dt=0.002, kT=0.1, gamma=1.0, seed=9)
    ra = A.run(300, cfg, step0=5, use_graph=True, log_period=50)
    rb = B.run(300, cfg, step0=5, use_graph=False, log_period=50)
    assert ra.stats.rebuilds == rb.stats.rebuilds
    xa, va, ia, _ = A.state_by_tag()
    xb, vb, ib, _ = B.state_by_tag()
    assert np.array_equal(xa, xb) and np.array_equal(va, vb) and np.array_equal(ia, ib)
    assert np.array_equal(ra.ev, rb.ev) and np.array_equal(ra.bonds, rb.bonds)
    # the logged state of the last row against the oracle
    x, _, _, ty = A.state_by_tag()
    ref = swap_ref.evaluate(x, ty, s.L, s.table)
    assert int(ra.bonds[-1]) == ref["bonds"]
    assert abs(ra.ev[-1, 0] - ref["E"]) <= 1e-5 * ref["A_E"]


def test_gather_widths_give_identical_trajectories():
    s = W.small_reactive(N=3000, density=0.35, seed=53, table=W.swap_table_single(lam=0.8), kT=0.1)
    out = []
    for w in (1, 2, 4):
        S = _system(s)
        S.set_gather_width(w)
        cfg = S.integrator(dt=0.002, kT=0.1, gamma=1.0, seed=4)
        r = S.run(200, cfg, log_period=50)
        out.append((S.state_by_tag(), r.ev))
    for (st, ev) in out[1:]:
        assert all(np.array_equal(a, b) for a, b in zip(out[0][0], st))
        assert np.array_equal(out[0][1], ev)


def test_fused_step_crossing_the_box():
    # particles placed on the faces move across them in one step: image counters
    rng = np.random.default_rng(4)
    L = float(np.float32(12.0))
    pts = rng.uniform(-6, 6, (200, 3))
    pts[:40, 0] = np.float32(L / 2) - np.float32(1e-4)
    pts[40:80, 1] = -np.float32(L / 2)
    s = W.cluster(pts, L=L, table=W.swap_table_single(lam=1.0))
    s.table = W.PairTable.empty(1)            # ideal gas: only the integrator acts
    s.vel = np.where(np.arange(200)[:, None] < 80, 3.0, 0.1).astype(np.float32) * np.sign(
        rng.standard_normal((200, 3))).astype(np.float32)
    s.vel[:40, 0] = 3.0
    s.vel[40:80, 1] = -3.0
    _one_step_check(s, "nve", 0.01, 0.0, 0.0, 1, 0)


def test_driver_graph_and_direct_launches_agree_bitwise():
    s = W.small_reactive(N=4000, density=0.3, seed=44, table=W.swap_table_single(lam=1.0), kT=0.1)
    A, B = _system(s), _system(s)
    cfg = A.integrator(dt=0.002, kT=0.1, gamma=1.0, seed=9)
    ra = A.run(400, cfg, step0=5, use_graph=True, log_period=50)
    rb = B.run(400, cfg, step0=5, use_graph=False, log_period=50)
    xa, va, ia, _ = A.state_by_tag()
    xb, vb, ib, _ = B.state_by_tag()
    assert ra.stats.rebuilds == rb.stats.rebuilds
    assert np.array_equal(xa, xb) and np.array_equal(va, vb) and np.array_equal(ia, ib)
    assert np.array_equal(ra.ev, rb.ev) and np.array_equal(ra.bonds, rb.bonds)


def test_driver_rollbacks_repair_stale_chunks():
    # fixed long chunks with a thin skin: chunks go stale and are replayed
    s = W.small_reactive(N=3000, density=0.25, seed=45, table=W.swap_table_single(lam=1.0), kT=0.5)
    A = _system(s, r_buff=0.06)
    B = _system(s, r_buff=0.06)
    cfg = A.integrator(dt=0.002, kT=0.5, gamma=1.0, seed=10)
    ra = A.run(300, cfg, max_chunk=64, adapt=False, log_period=100)
    rb = B.run(300, cfg, max_chunk=1, adapt=True, log_period=100)
    assert ra.stats.rollbacks > 0
    assert ra.stats.steps_done == 300 and rb.stats.steps_done == 300
    # both trajectories are valid: compare the final state with the oracle
    for S in (A, B):
        x, _, _, ty = S.state_by_tag()
        ref = swap_ref.evaluate(x, ty, s.L, s.table)
        F, ev = S.compute_forces()
        torch.cuda.synchronize()
        Fg = S.by_tag(F)
        err = np.abs(Fg[:, :3] - ref["F"]).max(axis=1) / np.maximum(ref["A_F"], 1e-30)
        assert err.max() < 1e-5
        assert S.bond_count() == ref["bonds"]
    # the list was never stale in the evaluated forces: the logged energies of the
    # first row agree exactly (same start), later rows agree to rounding
    assert ra.ev[0, 0] == rb.ev[0, 0]


@pytest.mark.parametrize("n", [3000, 1000])
def test_rollback_replays_are_exact(n):
    # With the rebuild threshold at the stale threshold (soft_frac 1), long fixed chunks rebuild right
    # after the first crossing, either at a chunk's end or by a rollback to the epoch's start and a
    # replay up to that step: the same schedule as one-step chunks.  The restore (state and zero path
    # lengths) and the replay are exact, so both runs agree bit for bit.  1000 particles replay in one
    # workgroup.
    s = W.small_reactive(N=n, density=0.25, seed=46, table=W.swap_table_single(lam=1.0), kT=0.5)
    A = _system(s, r_buff=0.06)
    B = _system(s, r_buff=0.06)
    for S in (A, B):
        S.set_step_form("walk")
    cfg = A.integrator(dt=0.002, kT=0.5, gamma=1.0, seed=11)
    ra = A.run(300, cfg, max_chunk=64, adapt=False, log_period=100, soft_frac=1.0)
    rb = B.run(300, cfg, max_chunk=1, adapt=False, log_period=100, soft_frac=1.0)
    assert ra.stats.rollbacks > 0 and rb.stats.rollbacks == 0
    assert ra.stats.rebuilds == rb.stats.rebuilds
    sa, sb = A.state_by_tag(), B.state_by_tag()
    assert all(np.array_equal(x, y) for x, y in zip(sa, sb))
    assert np.array_equal(ra.ev, rb.ev) and np.array_equal(ra.bonds, rb.bonds)


@pytest.mark.parametrize("n,steps,short", [(4000, 400, 0), (1000, 300, 2)])
def test_list_overflow_mid_run_resumes_exactly(n, steps, short):
    # A list sized to the first build's longest list overflows during the run.  The driver returns the
    # state at the failed build (its last half kick still owed) with the steps done; the engine grows the
    # list and resumes.  With the rebuild threshold at the stale threshold the rebuild schedule does not
    # depend on chunking, so the result equals a run with room to spare, bit for bit.  short > 0: the
    # list is too short for the first build already (found at the end of the first chunk, zero steps done).
    s = W.small_reactive(N=n, density=0.35, seed=47, kT=0.5)
    probe = _system(s, k_max=64)
    probe.build()
    kmax0 = int(((probe.nn & 0xFFFF) + (probe.nn >> 16)).max().item())
    A = _system(s, k_max=kmax0 - short)
    B = _system(s, k_max=64)
    for S in (A, B):
        S.set_step_form("walk")
    cfg = A.integrator(dt=0.002, kT=0.5, gamma=1.0, seed=12)
    ra = A.run(steps, cfg, soft_frac=1.0)
    rb = B.run(steps, cfg, soft_frac=1.0)
    assert A.k_max > kmax0                      # the list overflowed and grew
    sa, sb = A.state_by_tag(), B.state_by_tag()
    assert all(np.array_equal(x, y) for x, y in zip(sa, sb))


def test_nve_energy_is_conserved():
    # n = 100, r_cut = 1.3: the truncation jump is 1.6e-11 eps (SI, Performance)
    tab = W.swap_table_single(epsilon=1.0, sigma=1.0, n=100, rcut=1.3, lam=1.0)
    s = W.small_reactive(N=4000, density=0.125, seed=46, min_dist=1.0, table=tab, kT=0.03)
    S = _system(s, r_buff=0.2)
    cfg = S.integrator(kind="nve", dt=2e-4)
    r = S.run(5000, cfg, log_period=100)
    E = r.ev[:, 0] + 0.5 * r.ev[:, 7:10].sum(axis=1)
    K = 0.5 * r.ev[:, 7:10].sum(axis=1)
    # scale: kinetic energy plus the binding energy released by the bonds formed
    scale = K.max() + abs(r.ev[:, 0]).max()
    drift = abs(E[-10:].mean() - E[:10].mean())
    assert drift < 1e-3 * scale, (drift, scale)
    assert np.abs(E - E[0]).max() < 5e-3 * scale


def test_langevin_temperature():
    s = W.small_reactive(N=2000, density=0.2, seed=47, table=W.swap_table_single(lam=1.0), kT=0.1)
    S = _system(s)
    cfg = S.integrator(dt=0.002, kT=0.1, gamma=1.0, seed=11)
    S.run(3000, cfg)                      # relax the random start
    r = S.run(5000, cfg, step0=3000, log_period=50)
    T = r.ev[:, 7:10].sum(axis=1) / (3 * s.N)
    assert np.mean(T[10:]) == pytest.approx(0.1, rel=0.03)


def test_integrator_halves_match_fused_step():
    from paper_1912_08569_amd import _lib as L
    from paper_1912_08569_amd import api
    s = W.small_reactive(N=1500, density=0.25, seed=48, table=W.swap_table_single(lam=0.8), kT=0.1)
    A, B = _system(s), _system(s)
    A.build()
    B.build()
    cfg = A.integrator(dt=0.002, kT=0.1, gamma=1.0, seed=12)
    # separate kernels: F(x0), B A O A, F(x1), B
    A.compute_forces()
    api.rc_integrate_step(A.ctx, A.pos, A.vel, A.force, A.image, A.box, cfg, 7, L.RC_HALF_FIRST, None, A.status)
    A.compute_forces()
    api.rc_integrate_step(A.ctx, A.pos, A.vel, A.force, A.image, A.box, cfg, 7, L.RC_HALF_SECOND, None, A.status)
    # fused: START then FINISH
    api.rc_step_fused(B.ctx, B.pos, B.pos_alt, B.vel, B.image, B.nlist, B.nn, B.box, cfg, 7, L.RC_STEP_START,
                      0.8, None, B.status)
    api.rc_step_fused(B.ctx, B.pos_alt, B.pos, B.vel, B.image, B.nlist, B.nn, B.box, cfg, 8, L.RC_STEP_FINISH,
                      0.8, None, B.status)
    torch.cuda.synchronize()
    xa, va, _, _ = A.state_by_tag()
    _, _, tags = api.unpack_positions(B.pos_alt)
    xb = np.empty_like(xa)
    xb[tags] = api.unpack_positions(B.pos_alt)[0]
    vb = B.by_tag(B.vel)[:, :3]
    assert np.abs(xa - xb).max() < 1e-5
    assert np.abs(va - vb).max() < 1e-4 * (1 + np.abs(va).max())


def test_bonds_log_matches_oracle_at_the_end():
    s = W.assembly_mixture(N=30000, lam=0.5, seed=49, kT=0.05)
    S = _system(s)
    cfg = S.integrator(dt=0.001, kT=0.05, gamma=1.0, seed=13)
    r = S.run(1000, cfg, log_period=250)
    x, _, _, ty = S.state_by_tag()
    ref = swap_ref.evaluate(x, ty, s.L, s.table)
    assert int(r.bonds[-1]) == ref["bonds"]
    assert r.bonds[-1] > r.bonds[0]                # bonds form during assembly
    assert abs(r.ev[-1, 0] - ref["E"]) <= 1e-5 * ref["A_E"]


@pytest.mark.parametrize("form", ["walk", "sums"])
def test_fused_bond_counts_equal_the_list_walk(form):
    """Log rows with both logs take each bond count from the energy/virial step's gather; a run with the
    bond log alone counts by a walk of the swap lists (k_bonds).  Same trajectory, same counts."""
    from paper_1912_08569_amd import api
    s = W.assembly_mixture(N=20000, lam=1.0, seed=52, kT=0.05)
    rows = 1000 // 100 + 2
    out = []
    for both in (True, False):
        S = _system(s)
        S.set_step_form(form)
        cfg = S.integrator(dt=0.001, kT=0.05, gamma=1.0, seed=17)
        S.build()
        ev = torch.zeros(rows * 13, dtype=torch.float64, device=S.device)
        bonds = torch.zeros(rows, dtype=torch.int64, device=S.device)
        opts = rcl.MdOptions(1, 16, 256, 100, 0.8, 1, 1, 0, 0, 0)
        st = api.rc_md_run(S.ctx, S.md_buffers(ev if both else None, bonds), S.N, S.box, cfg, 0, 1000, opts)
        out.append((bonds[:int(st.log_rows)].cpu().numpy(), S.state_by_tag()[0], S.bond_count()))
        del S
    (ba, xa, ca), (bb, xb, cb) = out
    assert len(ba) == 11 and np.array_equal(ba, bb)   # steps 0, 100, ..., 900 and the end
    assert np.array_equal(xa, xb)
    assert int(ba[-1]) == ca == cb
    assert ba[-1] > ba[0]


def test_rebuild_graph_replays_equal_direct_rebuilds():
    """With a caller-owned workspace the driver replays its rebuilds as recorded graphs (from the second
    rebuild of a position buffer on); without one it launches them directly.  Same states, logs and
    schedules, bit for bit, over a run with many rebuilds."""
    s = W.small_reactive(N=6000, density=0.3, seed=57, table=W.swap_table_single(lam=1.0), kT=0.3)
    out = []
    for attached in (True, False):
        S = _system(s)
        if not attached:
            S.ctx.set_workspace(None)    # the context allocates its own buffers: rebuilds run directly
        cfg = S.integrator(dt=0.002, kT=0.3, gamma=1.0, seed=23)
        r = S.run(600, cfg, log_period=100)
        out.append((S.state_by_tag(), r))
        del S
    (sa, ra), (sb, rb) = out
    assert ra.stats.rebuilds >= 6 and ra.stats.rebuilds == rb.stats.rebuilds
    assert all(np.array_equal(x, y) for x, y in zip(sa, sb))
    assert np.array_equal(ra.ev, rb.ev) and np.array_equal(ra.bonds, rb.bonds)
    assert ra.stats.chunks == rb.stats.chunks and ra.stats.rollbacks == rb.stats.rollbacks


def test_auto_form_follows_the_swap_range_length():
    # "auto" picks the two-pass form for an all-reactive system and the walk form for the site/colloid
    # mixture, before the first run's steps (speed only: both forms are checked against the oracle)
    s = W.small_reactive(N=2000, seed=54, kT=0.1)
    S = _system(s)
    S.run(20, S.integrator(dt=0.001, kT=0.1, gamma=1.0, seed=1))
    assert S.mean_swap_length() >= S.AUTO_SUMS_KSWAP and S.ctx.step_form == "sums"
    m = W.assembly_mixture(N=20000, lam=1.0, seed=24, kT=0.05)
    M = _system(m)
    M.run(20, M.integrator(dt=0.001, kT=0.05, gamma=1.0, seed=1))
    assert M.mean_swap_length() < M.AUTO_SUMS_KSWAP and M.ctx.step_form == "walk"
    # an explicit form is kept by later runs
    S.set_step_form("walk")
    S.run(20, S.integrator(dt=0.001, kT=0.1, gamma=1.0, seed=1), step0=20)
    assert S.ctx.step_form == "walk"


def _one_block_case(case):
    if case == "dumbbells":
        return W.dumbbell_mixture(N=512, rcut=1.3, seed=41), None, dict(dt=0.001, kT=0.03)
    if case == "reactive_walk":
        return W.small_reactive(N=1000, density=0.3, seed=42, kT=0.1), "walk", dict(dt=0.002, kT=0.1)
    if case == "reactive_sums":
        return W.small_reactive(N=1000, density=0.3, seed=43, kT=0.1), "sums", dict(dt=0.002, kT=0.1)
    if case == "tiny":
        return W.small_reactive(N=100, density=0.2, seed=44, kT=0.1), "walk", dict(dt=0.002, kT=0.1)
    return W.vitrimer_network(n_chains=60, n_dimers=30, seed=12), None, dict(dt=2e-4, kT=1.0)


@pytest.mark.parametrize("case", ["dumbbells", "reactive_walk", "reactive_sums", "tiny", "network"])
def test_one_block_replays_equal_graph_replays(case):
    # systems of at most 1024 particles replay graph_steps steps in one workgroup with the positions
    # in LDS: the trajectory, the logs and the driver's decisions equal the hipGraph replays bit for bit
    # (ragged last wavefronts: 1000, 100 and 1020 particles; FENE springs in the network)
    s, form, kw = _one_block_case(case)
    out = []
    for one_block in (True, False):
        S = _system(s)
        if form:
            S.set_step_form(form)
        cfg = S.integrator(gamma=1.0, seed=17, **kw)
        r = S.run(400, cfg, step0=3, log_period=50, one_block=one_block)
        out.append((S.state_by_tag(), r, S.ctx.step_form))
    (sa, ra, fa), (sb, rb, fb) = out
    assert fa == fb
    assert all(np.array_equal(x, y) for x, y in zip(sa, sb))
    assert np.array_equal(ra.ev, rb.ev) and np.array_equal(ra.bonds, rb.bonds)
    assert (ra.stats.rebuilds, ra.stats.rollbacks, ra.stats.chunks) == (rb.stats.rebuilds, rb.stats.rollbacks,
                                                                       rb.stats.chunks)
    assert ra.stats.steps_done == 400


# --------------------------------------------------------------------------
# consecutive runs: the second continues on the first's list
# --------------------------------------------------------------------------

def _same_state(A, B):
    return all(np.array_equal(x, y) for x, y in zip(A.state_by_tag(), B.state_by_tag()))


@pytest.mark.parametrize("n", [4000, 1000])
def test_split_runs_equal_one_run_bitwise(n):
    # a wide skin: no list build after the first, so run(10); run(10) and run(20) take the same steps
    # (the finishing kick of the first run and the second run's first half kick are the one step's
    # kicks), and the continued run builds nothing at entry.  Rows at multiples of the log period
    # and at the end; the continued run does not repeat the first run's last row.
    # (a start at least 1.0 apart: no pair deep in the core, so nothing moves far in 20 steps)
    s = W.small_reactive(N=n, density=0.25, seed=61, table=W.swap_table_single(lam=0.8), kT=0.1, min_dist=1.0)
    A, B = _system(s, r_buff=0.8), _system(s, r_buff=0.8)
    for S in (A, B):
        S.set_step_form("walk")
    cfg = A.integrator(dt=0.002, kT=0.1, gamma=1.0, seed=3)
    ra1 = A.run(10, cfg, step0=0, log_period=5)
    ra2 = A.run(10, cfg, step0=10, log_period=5)
    rb = B.run(20, cfg, step0=0, log_period=5)
    assert ra2.stats.list_kept == 1 and ra2.stats.rebuilds == 0 and rb.stats.rebuilds == 1
    assert _same_state(A, B)
    assert np.array_equal(np.concatenate([ra1.ev, ra2.ev]), rb.ev)
    assert np.array_equal(np.concatenate([ra1.bonds, ra2.bonds]), rb.bonds)
    # a list build between runs, or a new step index, starts the next run with a build
    A.build()
    assert A.run(5, cfg, step0=20).stats.list_kept == 0
    assert A.run(5, cfg, step0=40).stats.list_kept == 0
    assert A.run(5, cfg, step0=45).stats.list_kept == 1


@pytest.mark.parametrize("n", [3000, 1000])
def test_continued_run_rolls_back_into_the_previous_runs_epoch(n):
    # a thin skin and long fixed chunks: the continued run's first chunk goes stale inside the epoch the
    # first run began, and is replayed from that epoch's snapshot (the first run's last steps again),
    # exactly as one run with one-step chunks takes them (the rollback test above, across two calls)
    s = W.small_reactive(N=n, density=0.25, seed=46, table=W.swap_table_single(lam=1.0), kT=0.5)
    A, B = _system(s, r_buff=0.06), _system(s, r_buff=0.06)
    for S in (A, B):
        S.set_step_form("walk")
    cfg = A.integrator(dt=0.002, kT=0.5, gamma=1.0, seed=11)
    kw = dict(max_chunk=64, adapt=False, soft_frac=1.0, log_period=100)
    ra1 = A.run(150, cfg, step0=0, **kw)
    ra2 = A.run(150, cfg, step0=150, **kw)
    rb = B.run(300, cfg, step0=0, max_chunk=1, adapt=False, soft_frac=1.0, log_period=100)
    assert ra2.stats.list_kept == 1 and ra2.stats.rollbacks > 0 and rb.stats.rollbacks == 0
    assert ra1.stats.rebuilds + ra2.stats.rebuilds == rb.stats.rebuilds
    assert _same_state(A, B)
    # rows: 0, 100, end 150 | 200, end 300   against 0, 100, 200, end 300
    assert np.array_equal(ra1.ev[:2], rb.ev[:2]) and np.array_equal(ra2.ev, rb.ev[2:])
    assert np.array_equal(ra1.bonds[:2], rb.bonds[:2]) and np.array_equal(ra2.bonds, rb.bonds[2:])


def test_timed_kernels_take_the_same_steps():
    # time_kernels launches every step directly between events: the same trajectory as graph replays
    s = W.assembly_mixture(N=20000, lam=1.0, seed=62, kT=0.05)
    A, B = _system(s), _system(s)
    cfg = A.integrator(dt=0.001, kT=0.05, gamma=1.0, seed=4)
    ra = A.run(200, cfg, log_period=50, time_kernels=True)
    rb = B.run(200, cfg, log_period=50)
    assert _same_state(A, B)
    assert np.array_equal(ra.ev, rb.ev) and np.array_equal(ra.bonds, rb.bonds)
    # every plain step launch is timed: all steps but the log steps (0, 50, 100, 150)
    assert ra.stats.kernel_launches >= 196 and ra.stats.kernel_ms > 0.0
    assert rb.stats.kernel_launches == 0
