"""Differentiation on the GPU: Hessian-vector products and parameter
gradients against the oracle's analytic second derivatives (themselves
pinned by finite differences in the CPU tests)."""
import numpy as np
import pytest
import torch

import workloads as W
from parity_util import vjp_scale
from oracle import adjoint_ref, swap_ref

pytestmark = pytest.mark.gpu

HVP_TOL = 2e-5   # of the per-particle term scale (second derivatives of (sigma/r)^(2n) in FP32)


def _system(s, **kw):
    from paper_1912_08569_amd import System
    return System.from_workload(s, **kw)


def _hvp_check(s, seed=0):
    S = _system(s)
    S.build()
    x, _, _, ty = S.state_by_tag()
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((s.N, 3))
    v /= np.linalg.norm(v)
    v4 = np.zeros((s.N, 4), np.float32)
    v4[:, :3] = v
    hv = S.by_tag(S.hvp(S.to_engine_order(v4)))[:, :3]
    torch.cuda.synchronize()
    ref, scale = adjoint_ref.hvp(x, ty, s.L, s.table, v4[:, :3].astype(np.float64), with_scale=True)
    err = np.abs(hv - ref).max(axis=1)
    bad = err > HVP_TOL * scale + 1e-30
    assert not bad.any(), f"HVP error {np.max(err / np.maximum(scale, 1e-30)):.3e} x scale"
    return S, v4


@pytest.mark.parametrize("lam", [0.0, 0.6, 1.0, 1.5])
def test_hvp_small(lam):
    s = W.small_reactive(N=2000, density=0.3, seed=61, table=W.swap_table_single(lam=lam))
    _hvp_check(s)


def test_hvp_dense_triplets():
    s = W.small_reactive(N=3000, density=0.55, seed=31, min_dist=0.85, table=W.swap_table_single(lam=0.4))
    _hvp_check(s, seed=3)


def test_hvp_differentiation_workload():
    # 32768 reactive particles at density 0.25, eps 10, sigma 1, n 10, lambda 1
    s = W.small_reactive(N=32768, density=0.25, seed=1005, table=W.swap_table_single(epsilon=10.0, lam=1.0))
    _hvp_check(s, seed=3005)


@pytest.mark.parametrize("n,nvec", [(32768, 64), (1000, 3)])
def test_hvp_batch_equals_single_products(n, nvec):
    # several tangent vectors in one launch per pass (64 at the differentiation workload's size; a
    # ragged 1000-particle case): every product equals the single-vector product bit for bit
    s = W.small_reactive(N=n, density=0.25, seed=1005, table=W.swap_table_single(epsilon=10.0, lam=1.0))
    S = _system(s)
    S.build()
    gen = torch.Generator().manual_seed(8)
    V = torch.randn((nvec, n, 4), generator=gen, dtype=torch.float32)
    V[:, :, 3] = 0.0
    V = V.to(S.device)
    H = S.hvp_batch(V)
    for k in range(nvec):
        assert torch.equal(H[k], S.hvp(V[k])), f"vector {k}"
    # the first product also against the oracle
    x, _, _, ty = S.state_by_tag()
    v0 = S.by_tag(V[0])[:, :3].astype(np.float64)
    ref, scale = adjoint_ref.hvp(x, ty, s.L, s.table, v0, with_scale=True)
    err = np.abs(S.by_tag(H[0])[:, :3] - ref).max(axis=1)
    assert np.all(err <= HVP_TOL * scale + 1e-30)


def test_hvp_mixture():
    s = W.assembly_mixture(N=20000, lam=1.0, seed=62)
    _hvp_check(s, seed=5)


def test_hvp_symmetry_and_translation():
    s = W.small_reactive(N=2000, density=0.3, seed=63, table=W.swap_table_single(lam=0.8))
    S = _system(s)
    S.build()
    rng = np.random.default_rng(1)
    v = torch.from_numpy(np.concatenate([rng.standard_normal((s.N, 3)), np.zeros((s.N, 1))], 1)
                         .astype(np.float32)).cuda()
    w = torch.from_numpy(np.concatenate([rng.standard_normal((s.N, 3)), np.zeros((s.N, 1))], 1)
                         .astype(np.float32)).cuda()
    Hv, Hw = S.hvp(v), S.hvp(w)
    a = float((w.double() * Hv.double()).sum())
    b = float((v.double() * Hw.double()).sum())
    assert a == pytest.approx(b, rel=1e-4)
    t = torch.zeros_like(v)
    t[:, :3] = torch.tensor([0.3, -1.0, 0.7])
    Ht = S.hvp(t)
    assert float(Ht.abs().max()) < 1e-4 * float(Hv.abs().max())


@pytest.mark.parametrize("lam", [0.0, 0.7, 1.3])
def test_param_grad(lam):
    s = W.assembly_mixture(N=20000, lam=lam, seed=64)
    S = _system(s)
    S.build()
    g = S.param_grad()
    x, _, _, ty = S.state_by_tag()
    ref = adjoint_ref.param_grad(x, ty, s.L, s.table)
    scale = np.abs(ref).max() + 1e-30
    assert np.abs(g - ref).max() <= 1e-5 * scale, (g, ref)


def test_param_grad_identities_on_gpu():
    from oracle import swap_ref
    s = W.small_reactive(N=4000, density=0.35, seed=65, table=W.swap_table_single(epsilon=2.0, lam=1.3))
    S = _system(s)
    S.build()
    g = S.param_grad()[0, 0]
    x, _, _, ty = S.state_by_tag()
    ref = swap_ref.evaluate(x, ty, s.L, s.table)
    assert g[2] == pytest.approx(ref["E3"] / 1.3, rel=1e-5)
    assert g[0] == pytest.approx(ref["E"] / 2.0, rel=1e-5, abs=1e-5 * ref["A_E"])


@pytest.mark.parametrize("lam", [0.4, 1.0, 1.5])
def test_param_vjp_mixture_matches_force_differences(lam):
    # two swap entries and a WCA entry, dense enough for many triplets
    tab = W.PairTable.empty(2)
    tab.set(0, 0, W.KIND_SWAP, 1.3, 1.0, 10, 1.5, lam)
    tab.set(0, 1, W.KIND_WCA, 1.0, 0.9, 6)
    tab.set(1, 1, W.KIND_SWAP, 2.0, 0.8, 8, 1.2, 0.7 * lam)
    rng = np.random.default_rng(66)
    L = float(np.float32(9.0))
    pos, types = W.rsa_positions(rng, L, [250, 150], np.full((2, 2), 0.9))
    s = W.System(pos=pos, types=types, L=L, table=tab, mass=np.ones(2), vel=np.zeros((400, 3), np.float32))
    S = _system(s)
    S.build()
    x, _, _, ty = S.state_by_tag()
    adj = rng.standard_normal((s.N, 3))
    a4 = np.zeros((s.N, 4), np.float32)
    a4[:, :3] = adj
    got = S.param_vjp(S.to_engine_order(a4))
    ref = adjoint_ref.force_param_vjp(x, ty, s.L, tab, a4[:, :3].astype(np.float64))
    # FP32 terms summed with random-sign adjoints: 1e-5 of the size of the summed terms
    sc = vjp_scale(swap_ref.evaluate(x, ty, s.L, tab)["A_F"], a4, tab)
    act = sc > 0
    err = np.abs(got - ref)
    assert np.all(err[act] <= 1e-5 * sc[act]), (err / np.where(act, sc, 1.0)).max()
    assert np.all(err[~act] == 0.0)
    assert np.abs(ref[:, :, 2]).max() > 0.0   # three-body part present


def test_param_vjp_lambda_zero_single_entry():
    # at lambda = 0 the three-body force is linear in lambda: a . dF/dlambda = a . (F(1) - F(0))
    from oracle import swap_ref
    s = W.small_reactive(N=1500, density=0.4, seed=67, table=W.swap_table_single(lam=0.0))
    S = _system(s)
    S.build()
    x, _, _, ty = S.state_by_tag()
    rng = np.random.default_rng(5)
    a4 = np.zeros((s.N, 4), np.float32)
    a4[:, :3] = rng.standard_normal((s.N, 3))
    got = S.param_vjp(S.to_engine_order(a4))[0, 0]
    t1 = s.table.copy()
    t1.lam[:] = 1.0
    F0 = swap_ref.evaluate(x, ty, s.L, s.table, scales=False)["F"]
    F1 = swap_ref.evaluate(x, ty, s.L, t1, scales=False)["F"]
    adj = a4[:, :3].astype(np.float64)
    r3, r0 = np.sum(adj * (F1 - F0)), np.sum(adj * F0) / 1.0
    # scales: the three-body terms' sizes at lambda = 1 (dF/dlambda at 0 is F3(1)), all terms / eps
    e0 = swap_ref.evaluate(x, ty, s.L, s.table)
    e1 = swap_ref.evaluate(x, ty, s.L, t1)
    na = np.linalg.norm(adj, axis=1)
    assert abs(got[2] - r3) <= 1e-5 * float(np.sum(na * (e1["A_F"] - e0["A_F"])))
    assert abs(got[0] - r0) <= 1e-5 * float(np.sum(na * e0["A_F"]))


def test_param_vjp_differentiation_workload_eps_identity():
    # 32768 reactive particles, eps 10: a . dF/deps = a . F / eps for one entry
    s = W.small_reactive(N=32768, density=0.25, seed=1005, table=W.swap_table_single(epsilon=10.0, lam=1.0))
    S = _system(s)
    S.build()
    rng = np.random.default_rng(6)
    a4 = np.zeros((s.N, 4), np.float32)
    a4[:, :3] = rng.standard_normal((s.N, 3))
    ae = S.to_engine_order(a4)
    got = S.param_vjp(ae)[0, 0]
    F, _ = S.compute_forces(gather=True)
    torch.cuda.synchronize()
    aF = float((ae[:, :3].double() * F[:, :3].double()).sum())
    x, _, _, ty = S.state_by_tag()
    sc = vjp_scale(swap_ref.evaluate(x, ty, s.L, s.table)["A_F"], a4, s.table)
    assert abs(got[0] - aF / 10.0) <= 1e-5 * sc[0, 0, 0]
