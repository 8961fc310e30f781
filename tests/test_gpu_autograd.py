"""The torch.autograd bindings and the trajectory fit of lambda, on the GPU.

Values and derivatives come from the HIP library through the C ABI; they are
compared with the FP64 oracle (forces, analytic Hessian-vector products,
energy gradients, finite-difference force-parameter VJPs) and, for the
trajectory, with finite differences of the trajectory loss itself.
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import adjoint_ref, swap_ref
from parity_util import assert_forces, vjp_scale

pytestmark = pytest.mark.gpu


def _mixture(n0=250, n1=150, lam=0.8, seed=70, L=9.0, dmin=0.9):
    tab = W.PairTable.empty(2)
    tab.set(0, 0, W.KIND_SWAP, 1.3, 1.0, 10, 1.5, lam)
    tab.set(0, 1, W.KIND_WCA, 1.0, 0.9, 6)
    tab.set(1, 1, W.KIND_SWAP, 2.0, 0.8, 8, 1.2, 0.7 * lam)
    rng = np.random.default_rng(seed)
    Lf = float(np.float32(L))
    pos, types = W.rsa_positions(rng, Lf, [n0, n1], np.full((2, 2), dmin))
    vel = W.maxwell_velocities(rng, types, np.ones(2), 0.1)
    return W.System(pos=pos, types=types, L=Lf, table=tab, mass=np.ones(2), vel=vel)


def _model(s, **kw):
    from paper_1912_08569_amd import System
    from paper_1912_08569_amd.autograd import SwapModel
    return SwapModel(System.from_workload(s, **kw))


def test_energy_gradients_match_oracle():
    from paper_1912_08569_amd.autograd import swap_energy
    s = _mixture()
    M = _model(s)
    x = torch.from_numpy(s.pos).cuda().requires_grad_(True)
    theta = M.theta().requires_grad_(True)
    E = swap_energy(M, x, theta)
    gx, gt = torch.autograd.grad(E, (x, theta))
    ref = swap_ref.evaluate(s.pos.astype(np.float64), s.types, s.L, s.table)
    assert abs(float(E.detach()) - ref["E"]) <= 1e-5 * ref["A_E"]
    assert_forces(-gx.cpu().numpy(), ref)
    g = adjoint_ref.param_grad(s.pos.astype(np.float64), s.types, s.L, s.table)
    iu = np.triu_indices(2)
    assert np.abs(gt.numpy()[iu] - g[iu]).max() <= 1e-5 * np.abs(g).max()
    assert np.all(gt.numpy()[1, 0] == 0.0)


def test_forces_vjp_matches_oracle():
    from paper_1912_08569_amd.autograd import swap_forces
    s = _mixture(seed=71)
    M = _model(s)
    x = torch.from_numpy(s.pos).cuda().requires_grad_(True)
    theta = M.theta().requires_grad_(True)
    F = swap_forces(M, x, theta)
    rng = np.random.default_rng(2)
    a = rng.standard_normal((s.N, 3)).astype(np.float32)
    gx, gt = torch.autograd.grad(F, (x, theta), torch.from_numpy(a).cuda())
    xd = s.pos.astype(np.float64)
    hv, scale = adjoint_ref.hvp(xd, s.types, s.L, s.table, a.astype(np.float64), with_scale=True)
    err = np.abs(-gx.cpu().numpy() - hv).max(axis=1)
    assert np.all(err <= 2e-5 * scale + 1e-30)
    ref = adjoint_ref.force_param_vjp(xd, s.types, s.L, s.table, a.astype(np.float64))
    sc = vjp_scale(swap_ref.evaluate(xd, s.types, s.L, s.table)["A_F"], a, s.table)
    iu = np.triu_indices(2)
    for w in range(3):
        d = np.abs(gt.numpy()[..., w][iu] - ref[..., w][iu])
        act = sc[..., w][iu] > 0
        assert np.all(d[act] <= 1e-5 * sc[..., w][iu][act]) and np.all(d[~act] == 0.0)


def test_model_rebuilds_and_keeps_tag_order():
    from paper_1912_08569_amd.autograd import swap_forces
    s = _mixture(seed=72)
    M = _model(s, r_buff=0.2)
    theta = M.theta()
    rng = np.random.default_rng(3)
    x = s.pos.astype(np.float64)
    for k in range(3):
        x = x + rng.normal(scale=0.08, size=x.shape)          # beyond half the skin: rebuilds
        x = (x + s.L / 2) % s.L - s.L / 2
        xf = x.astype(np.float32)
        F = swap_forces(M, torch.from_numpy(xf).cuda(), theta)
        ref = swap_ref.evaluate(xf.astype(np.float64), s.types, s.L, s.table)
        assert_forces(F.cpu().numpy(), ref)
    assert M.rebuilds >= 2


def _traj_fit(N=400, steps=30, segment=10, lam=0.8, seed=73, table=None, dt=0.002, density=0.35, min_dist=0.95):
    from paper_1912_08569_amd.fit import TrajectoryFit
    tab = table if table is not None else W.swap_table_single(lam=lam)
    s = W.small_reactive(N=N, density=density, seed=seed, min_dist=min_dist, table=tab, kT=0.1)
    M = _model(s)
    x0 = torch.from_numpy(s.pos).cuda()
    v0 = torch.from_numpy(s.vel).cuda()
    m = torch.ones(s.N, device="cuda")
    return M, TrajectoryFit(M, x0, v0, m, dt=dt, kT=0.1, gamma=1.0, steps=steps, segment=segment, n_swap=s.N,
                            seed=5)


def test_trajectory_gradient_matches_finite_differences():
    # n = 100, r_cut = 1.3: the force jump at the cutoff is ~1e-10 eps/sigma, so the
    # trajectory is smooth in lambda and its derivative is what backpropagation gives
    # (with a visible jump, pairs crossing r_cut add impulses that only differences see)
    tab = W.swap_table_single(epsilon=1.0, sigma=1.0, n=100, rcut=1.3, lam=0.8)
    # (start at 1.02 sigma: the n = 100 wall is far too stiff for closer starts)
    M, fit = _traj_fit(N=1000, steps=40, segment=10, table=tab, dt=5e-4, density=0.3, min_dist=1.02)
    theta0 = M.theta()
    lam = torch.tensor(0.8, dtype=torch.float64, requires_grad=True)

    def loss_at(l, ckpt=True):
        mask = torch.zeros_like(theta0)
        mask[0, 0, 2] = 1.0
        th = theta0 * (1 - mask) + mask * l
        return fit.observable(th, checkpointed=ckpt)

    (g_ck,) = torch.autograd.grad(loss_at(lam), lam)
    (g_full,) = torch.autograd.grad(loss_at(lam, ckpt=False), lam)
    assert float(g_ck) == pytest.approx(float(g_full), rel=1e-4, abs=1e-9)
    # differences of the engine's own FP32 trajectories: the two losses differ by ~1e-6 of their size,
    # about the FP32 rounding of the trajectory, so this difference quotient carries a few per cent of
    # noise (the FP64 oracle's differences below pin the derivative itself)
    h = 2e-3
    with torch.no_grad():
        fd = (float(loss_at(torch.tensor(0.8 + h, dtype=torch.float64)))
              - float(loss_at(torch.tensor(0.8 - h, dtype=torch.float64)))) / (2 * h)
    assert float(g_ck) == pytest.approx(fd, rel=0.06), (float(g_ck), fd)
    assert abs(fd) > 0.0


def test_fit_moves_lambda_toward_the_target():
    from paper_1912_08569_amd.fit import fit_lambda
    M, fit = _traj_fit(N=2000, steps=40, segment=10, lam=0.5, seed=74)
    theta0 = M.theta()
    with torch.no_grad():
        b0 = float(fit.observable(theta0))
    target = 0.9 * b0          # fewer bonds: lambda has to grow (the three-body term penalises sharing)
    hist = fit_lambda(fit, (0, 0), 0.5, target, iters=4, step=0.3)
    assert min(h["loss"] for h in hist[1:]) < hist[0]["loss"]
    assert hist[0]["grad"] < 0.0          # more lambda, fewer bonds, smaller loss


def test_engine_noise_is_the_oracles_philox():
    from oracle import philox_ref
    from paper_1912_08569_amd import api
    xi = api.rc_thermostat_normals(77, 1000, 3, 5000).cpu().numpy()
    for k in range(3):
        ref = np.asarray(philox_ref.thermostat_normals(77, np.arange(5000), 1000 + k), dtype=np.float64)
        assert np.abs(xi[k, :, :3] - ref).max() <= 1e-5 * max(1.0, np.abs(ref).max())
    assert np.all(xi[..., 3] == 0.0)
    xi2 = api.rc_thermostat_normals(77, 1000, 1, 100, dim=2).cpu().numpy()
    assert np.all(xi2[0, :, 2] == 0.0) and np.array_equal(xi2[0, :, :2], xi[0, :100, :2])


def test_fit_trajectory_follows_the_engine():
    # the fit's torch BAOAB with the engine's noise takes the steps rc_md_run takes (to FP32 rounding)
    from paper_1912_08569_amd import System
    from paper_1912_08569_amd.autograd import swap_forces
    s = W.small_reactive(N=1000, density=0.3, seed=75, min_dist=1.0, table=W.swap_table_single(lam=0.8), kT=0.1)
    M, fit = _fit_for(s, steps=20, segment=10, dt=0.002)
    with torch.no_grad():
        theta = M.theta()
        x, v = fit.x0, fit.v0
        F = swap_forces(M, x, theta)
        for k in range(20):
            x, v, F, _ = fit._segment(k, k + 1, theta, x, v, F)
    S = System.from_workload(s)
    S.run(20, S.integrator(dt=0.002, kT=0.1, gamma=1.0, seed=5), step0=0)
    xe, ve, _, _ = S.state_by_tag()
    d = swap_ref.min_image(x.cpu().numpy().astype(np.float64), xe.astype(np.float64), s.box)
    assert np.abs(d).max() < 1e-4
    assert np.abs(v.cpu().numpy() - ve).max() < 1e-3


def _fit_for(s, steps, segment, dt):
    from paper_1912_08569_amd.fit import TrajectoryFit
    M = _model(s)
    return M, TrajectoryFit(M, torch.from_numpy(s.pos).cuda(), torch.from_numpy(s.vel).cuda(),
                            torch.ones(s.N, device="cuda"), dt=dt, kT=0.1, gamma=1.0, steps=steps,
                            segment=segment, n_swap=s.N, seed=5)


def test_trajectory_gradient_matches_oracle_finite_differences():
    # the lambda derivative of the trajectory observable: backpropagation through the engine's
    # forces against central differences of the FP64 oracle's trajectory (swap_ref forces,
    # dynamics_ref BAOAB, adjoint_ref soft bonds) with the same Philox noise (common random numbers)
    from oracle import dynamics_ref
    tab = W.swap_table_single(epsilon=1.0, sigma=1.0, n=100, rcut=1.3, lam=0.8)
    s = W.small_reactive(N=1000, density=0.3, seed=73, min_dist=1.02, table=tab, kT=0.1)
    steps, dt = 40, 5e-4
    M, fit = _fit_for(s, steps=steps, segment=10, dt=dt)
    theta0 = M.theta()
    mask = torch.zeros_like(theta0)
    mask[0, 0, 2] = 1.0
    lam = torch.tensor(0.8, dtype=torch.float64, requires_grad=True)
    (g,) = torch.autograd.grad(fit.observable(theta0 * (1 - mask) + mask * lam), lam)

    def oracle_observable(l):
        t = tab.with_lambda(l)
        x, v = s.pos.astype(np.float64), s.vel.astype(np.float64)
        F = swap_ref.evaluate(x, s.types, s.L, t, scales=False)["F"]
        tot = 0.0
        for k in range(steps):
            out = dynamics_ref.baoab_step(x, v, s.types, np.arange(s.N), s.L, t, s.mass, dt, 0.1, 1.0, 5, k, force=F)
            x, v, F = out["pos"], out["vel"], out["F"]
            tot += adjoint_ref.soft_bonds(x, s.types, s.L, t)[0]
        return tot / (steps * s.N)

    h = 2e-3
    fd = (oracle_observable(0.8 + h) - oracle_observable(0.8 - h)) / (2 * h)
    assert abs(fd) > 0.0
    assert float(g) == pytest.approx(fd, rel=0.03), (float(g), fd)
