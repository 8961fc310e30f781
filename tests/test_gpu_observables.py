"""The paper's bond-swap test system (Sec. 3.1: A:B = 3:2 dumbbell mixture, n = 100,
density 0.125, kT 0.03) and the bond-partner observable behind its bond
autocorrelation, on the GPU through the C ABI, against the FP64 oracle."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import observables_ref, swap_ref
from parity_util import assert_energy, assert_forces, assert_virial

pytestmark = pytest.mark.gpu


def _system(s, **kw):
    from paper_1912_08569_amd import System
    return System.from_workload(s, **kw)


def _partners_ref(S, s):
    """Oracle bond partners of the engine's current state, as tags."""
    x, _, _, ty = S.state_by_tag()
    return swap_ref.bond_partners(x.astype(np.float64), ty, s.L, s.table)


@pytest.mark.parametrize("rcut", [1.3, 1.15])
def test_dumbbell_mixture_matches_oracle(rcut):
    s = W.dumbbell_mixture(N=1000, rcut=rcut, seed=21)
    S = _system(s)
    F, ev = S.compute_forces(gather=True)
    torch.cuda.synchronize()
    x, _, _, ty = S.state_by_tag()
    ref = swap_ref.evaluate(x.astype(np.float64), ty, s.L, s.table)
    assert_forces(S.by_tag(F), ref)
    assert_energy(ev[0].item(), ref)
    assert_virial(ev[1:7].cpu().numpy(), ref)
    assert S.bond_count() == ref["bonds"]
    assert np.array_equal(S.bond_partners(), _partners_ref(S, s))


def test_dumbbell_dynamics_bonds_and_partners():
    # at kT 0.03 the minority B bind A partners; partners on the GPU equal the oracle's on the
    # engine's own state at every check, and the bond autocorrelation is a fraction in [0, 1]
    s = W.dumbbell_mixture(N=2000, rcut=1.3, seed=22)
    S = _system(s)
    cfg = S.integrator(dt=0.001, kT=0.03, gamma=1.0, seed=31)
    S.build()
    is_b = s.types == 1                    # the workload lists particles in tag order
    p0 = S.bond_partners()
    assert np.array_equal(p0, _partners_ref(S, s))
    bonded0 = np.mean(p0[is_b] >= 0)
    S.run(3000, cfg, step0=0)
    S.build()
    p1 = S.bond_partners()
    assert np.array_equal(p1, _partners_ref(S, s))
    bonded1 = np.mean(p1[is_b] >= 0)
    assert bonded1 > bonded0               # B particles bind during the run
    c = swap_ref.bond_autocorrelation(p0, p1, mask=is_b)
    assert np.isnan(c) or 0.0 <= c <= 1.0


def test_bond_partners_of_the_assembly_mixture():
    # reactive sites of the self-assembly mixture after bonds formed: partners (single, none or
    # several bonds) equal the oracle's, and every bond is reported at both ends
    s = W.assembly_mixture(N=20000, lam=1.0, seed=23, kT=0.05)
    S = _system(s)
    S.run(2000, S.integrator(dt=0.001, kT=0.05, gamma=1.0, seed=32))
    S.build()
    p = S.bond_partners()
    ref = _partners_ref(S, s)
    assert np.array_equal(p, ref)
    single = np.flatnonzero(p >= 0)
    both = single[p[p[single]] >= 0]
    assert np.all(p[p[both]] == both)        # symmetric where both ends have one bond
    assert np.count_nonzero(p != -1) > 0


def test_partner_counts_and_stress_autocorrelation_match_oracle():
    # on-device statistics of two partner snapshots (exact) and G(t) of the logged stress rows (FP64,
    # reduction order) against the oracle, for the dumbbell mixture
    s = W.dumbbell_mixture(N=2000, rcut=1.3, seed=24)
    S = _system(s)
    cfg = S.integrator(dt=0.001, kT=0.03, gamma=1.0, seed=34)
    S.build()
    p0 = S.bond_partners()
    r = S.run(2000, cfg, log_period=10)
    S.build()
    p1 = S.bond_partners()
    for sel in (None, s.types == 1):
        assert S.partner_counts(p0, p1, sel) == observables_ref.partner_counts(p0, p1, sel)
    rows = r.ev
    assert rows.shape[0] > 100
    G = S.stress_autocorrelation(rows, 0.03, 60)
    ref = observables_ref.stress_autocorrelation(rows, float(s.L) ** 3, 0.03, 60)
    assert np.allclose(G, ref, rtol=1e-11, atol=1e-11 * abs(ref[0]))


def test_partner_counts_hand_example():
    # a broken bond, a site with several bonds, a swap, unchanged bonds; with and without a selection
    s = W.dumbbell_mixture(N=512, rcut=1.3, seed=25)
    S = _system(s)
    p0 = np.array([1, 0, 3, -2, 3, -1, 7, 6])
    pt = np.array([5, -1, 3, -2, -2, 1, 7, 6])
    assert S.partner_counts(p0, pt) == (6, 3, 1)
    assert S.partner_counts(p0, pt, np.arange(8) % 2 == 1) == (2, 1, 0)
