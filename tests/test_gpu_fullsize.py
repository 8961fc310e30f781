"""Parity at the full 1,048,576-particle size, in the launch configuration
the benchmark times (fused step kernel, graph-captured driver)."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import swap_ref
from parity_util import assert_energy, assert_forces, assert_virial

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def big():
    from paper_1912_08569_amd import System
    s = W.assembly_mixture(N=1048576, lam=0.5, seed=1003, kT=0.05)
    S = System.from_workload(s)
    S.build()
    return s, S


def _parity(s, S):
    F, ev = S.compute_forces(gather=True)
    torch.cuda.synchronize()
    x, _, _, ty = S.state_by_tag()
    ref = swap_ref.evaluate(x, ty, s.L, s.table)
    Fg = S.by_tag(F)
    assert_forces(Fg, ref)
    evh = ev.cpu().numpy()
    assert_energy(evh[0], ref)
    assert_virial(evh[1:7], ref)
    assert S.bond_count() == ref["bonds"]
    # the triplet kernel agrees too
    F2, ev2 = S.compute_forces(gather=False)
    torch.cuda.synchronize()
    assert_forces(S.by_tag(F2), ref)
    assert_energy(ev2.cpu().numpy()[0], ref)
    return ref


def test_fullsize_start(big):
    s, S = big
    _parity(s, S)


def test_fullsize_after_assembly(big):
    s, S = big
    cfg = S.integrator(dt=0.001, kT=0.05, gamma=1.0, seed=2003)
    r = S.run(1000, cfg, log_period=500)
    ref = _parity(s, S)
    assert ref["n_triplets"] > 0
    assert int(r.bonds[-1]) == ref["bonds"]


def test_fullsize_sampled_forces_vs_brute_force(big, brute_lib):
    s, S = big
    F, _ = S.compute_forces(gather=True)
    torch.cuda.synchronize()
    x, _, _, ty = S.state_by_tag()
    idx = np.random.default_rng(7).choice(s.N, 128, replace=False)
    b = brute_lib.forces_subset(x, ty, s.L, s.table, idx)
    Fg = S.by_tag(F)[idx, :3]
    ref = swap_ref.evaluate(x, ty, s.L, s.table)
    err = np.abs(Fg - b["F"]).max(axis=1) / np.maximum(ref["A_F"][idx], 1e-30)
    assert err.max() < 1e-5
    assert np.array_equal(b["degree"], swap_ref.bond_degree(x, ty, s.L, s.table)[idx])
