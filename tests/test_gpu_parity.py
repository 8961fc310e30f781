"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Inputs are the seeded synthetic systems of ``workloads``; the library
re-orders particles, so every comparison is made in tag order.  Tolerances
are explained in ``parity_util``.
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import swap_ref
from parity_util import assert_energy, assert_forces, assert_pe, assert_virial

pytestmark = pytest.mark.gpu


def _system(s, **kw):
    from paper_1912_08569_amd import System
    return System.from_workload(s, **kw)


def _check_all(sysg, s, gather):
    F, ev = sysg.compute_forces(gather=gather)
    torch.cuda.synchronize()
    xyz, _, _, ty = sysg.state_by_tag()
    ref = swap_ref.evaluate(xyz, ty, s.L, s.table)
    Fg = sysg.by_tag(F)
    evh = ev.cpu().numpy()
    ef = assert_forces(Fg, ref)
    assert_pe(Fg[:, 3], ref)
    assert_energy(evh[0], ref)
    assert_virial(evh[1:7], ref)
    assert sysg.bond_count() == ref["bonds"]
    return ref, ef


@pytest.mark.parametrize("gather", [False, True, "sums"])
@pytest.mark.parametrize("lam", [0.0, 0.5, 1.0, 1.5])
def test_small_reactive_one_call(lam, gather):
    # N=1000, density 0.2, eps 1, sigma 1, n 10, r_cut 1.5 (the small plain system)
    s = W.small_reactive(N=1000, density=0.2, seed=1001, table=W.swap_table_single(lam=lam))
    ref, _ = _check_all(_system(s), s, gather)
    assert ref["n_pairs"] > 0


@pytest.mark.parametrize("gather", [False, True, "sums"])
def test_dense_clusters_many_triplets(gather):
    # a dense lambda < 1 configuration: many centres with 3+ partners
    s = W.small_reactive(N=3000, density=0.55, seed=31, min_dist=0.85, table=W.swap_table_single(lam=0.4))
    ref, _ = _check_all(_system(s), s, gather)
    assert ref["n_triplets"] > 500


@pytest.mark.parametrize("gather", [False, True, "sums"])
@pytest.mark.parametrize("lam", [0.0, 1.0, 1.5])
def test_assembly_mixture_small(lam, gather):
    s = W.assembly_mixture(N=20000, lam=lam, seed=1003)
    _check_all(_system(s), s, gather)


@pytest.mark.parametrize("gather", [False, True, "sums"])
def test_unequal_pair_lambdas(gather):
    # every swap pair with its own lambda and epsilon: triplet weights from unequal entries (reading 4)
    s = W.unequal_lambda_mixture()
    ref, _ = _check_all(_system(s), s, gather)
    assert ref["n_triplets"] > 100


def test_boundary_straddling_pairs():
    # triplets across every face and edge of the box
    L = 9.0
    rm = 2.0 ** 0.1
    h = float(np.float32(L)) / 2
    pts = []
    for ax in range(3):
        for sgn in (-1, 1):
            c = np.zeros(3)
            c[ax] = sgn * (h - 0.3)
            a = c.copy(); a[ax] += sgn * 1.1 * rm
            b = c.copy(); b[(ax + 1) % 3] += 1.2
            pts += [c, a, b]
    pts.append([h - 0.2, h - 0.2, h - 0.2])
    pts.append([-h + 0.5, -h + 0.6, -h + 0.4])
    s = W.cluster(np.array(pts), L=L, table=W.swap_table_single(lam=0.7))
    sysg = _system(s, r_buff=0.3)
    ref, _ = _check_all(sysg, s, gather=False)
    _check_all(sysg, s, gather=True)
    _check_all(sysg, s, gather="sums")
    assert ref["n_triplets"] >= 6


def idx_sorted_types(sysg, idx):
    """Tags of engine indices idx (so that types in tag order can be looked up)."""
    _, _, tags = __import__("paper_1912_08569_amd").unpack_positions(sysg.pos)
    return tags[np.asarray(idx)]


def test_nlist_contains_every_interacting_pair():
    s = W.assembly_mixture(N=20000, lam=1.0, seed=5)
    sysg = _system(s)
    sysg.build()
    xyz, _, _, ty = sysg.state_by_tag()
    P = swap_ref.interacting_pairs(xyz, ty, s.L, s.table)
    _, _, tags = __import__("paper_1912_08569_amd").unpack_positions(sysg.pos)
    idx_of_tag = np.empty(s.N, np.int64)
    idx_of_tag[tags] = np.arange(s.N)
    nl = sysg.nlist.cpu().numpy().reshape(sysg.k_max, s.N)
    packed = sysg.nn.cpu().numpy()
    ns, no = packed & 0xFFFF, packed >> 16          # swap range at the front, the rest at the back
    have = set()
    for slot in range(ns.max()):
        m = ns > slot
        have.update(zip(np.nonzero(m)[0].tolist(), nl[slot][m].tolist()))
    for slot in range(no.max()):
        m = no > slot
        have.update(zip(np.nonzero(m)[0].tolist(), nl[sysg.k_max - 1 - slot][m].tolist()))
    # the front range holds exactly the swap-kind neighbours
    kinds = s.table.kind
    for slot in range(ns.max()):
        m = np.nonzero(ns > slot)[0]
        assert np.all(kinds[ty[idx_sorted_types(sysg, m)], ty[idx_sorted_types(sysg, nl[slot][m])]] == W.KIND_SWAP)
    for a, b in zip(P["i"], P["j"]):
        ia, ib = int(idx_of_tag[a]), int(idx_of_tag[b])
        assert (ia, ib) in have and (ib, ia) in have
    # the list is sorted by cell key: tags travel, rtag maps tag -> index
    rtag = sysg.rtag.cpu().numpy()
    assert np.array_equal(rtag[tags], np.arange(s.N))


def test_nlist_overflow_is_reported_and_recovered():
    from paper_1912_08569_amd import _lib as L
    from paper_1912_08569_amd import api
    s = W.small_reactive(N=2000, density=0.5, seed=9, min_dist=0.8)
    sysg = _system(s, k_max=2)
    api.rc_build_cells(sysg.ctx, sysg.pos, sysg.vel, sysg.image, sysg.rtag, sysg.box, sysg.ws)
    api.rc_clear_status(sysg.status)
    api.rc_build_nlist(sysg.ctx, sysg.pos, sysg.vel, sysg.box, sysg.ws, 2, sysg.nlist, sysg.nn, sysg.status)
    code, st = api.rc_read_status(sysg.status)
    assert code == L.RC_ERR_NLIST_OVERFLOW and st[L.RC_ST_KMAX] > 2
    k = sysg.build()
    assert sysg.k_max >= k
    _check_all(sysg, s, gather=True)


def test_argument_errors_are_synchronous():
    from paper_1912_08569_amd import RcError, api
    s = W.small_reactive(N=200, density=0.2, seed=3)
    sysg = _system(s)
    with pytest.raises(RcError):
        api.rc_build_cells(sysg.ctx, sysg.pos, sysg.vel, None, None, api.box(s.L + 0.1), sysg.ws)
    with pytest.raises(RcError):
        api.rc_compute_forces(sysg.ctx, sysg.pos, sysg.nlist, sysg.nn, sysg.box, sysg.force, None, 64)
    bad = W.swap_table_single(lam=-1.0)
    with pytest.raises(RcError):
        api.Context(bad)


def test_argument_errors_of_the_newer_entry_points():
    # rejected before any launch, with RC_ERR_ARG and a message
    import ctypes

    import torch
    from paper_1912_08569_amd import RcError, api
    from paper_1912_08569_amd import _lib as L
    s = W.small_reactive(N=300, density=0.2, seed=4)
    S = _system(s)
    S.build()

    def rejected(fn):
        with pytest.raises(RcError) as e:
            fn()
        assert e.value.code == L.RC_ERR_ARG and len(str(e.value)) > 20
    V = torch.zeros((2, s.N, 4), dtype=torch.float32, device=S.device)
    flat = torch.zeros(2 * s.N * 4 + 1, dtype=torch.float32, device=S.device)
    rejected(lambda: L.check(L.load().rc_force_hvp_batch(S.ctx.handle, api._ptr(S.pos), api._ptr(S.nlist),
                                                         api._ptr(S.nn), S.k_max, s.N, S.box, 0, api._ptr(V),
                                                         api._ptr(V), None), S.ctx.handle))
    mis = ctypes.c_void_p(flat.data_ptr() + 4)          # 4 bytes off 16-byte alignment
    rejected(lambda: L.check(L.load().rc_force_hvp_batch(S.ctx.handle, api._ptr(S.pos), api._ptr(S.nlist),
                                                         api._ptr(S.nn), S.k_max, s.N, S.box, 2, mis,
                                                         api._ptr(V), None), S.ctx.handle))
    rows = torch.zeros((10, 13), dtype=torch.float64, device=S.device)
    G = torch.zeros(20, dtype=torch.float64, device=S.device)
    rejected(lambda: api.rc_stress_autocorrelation(S.ctx, rows, 8.0, 1.0, 10, G))      # max_lag == T
    rejected(lambda: api.rc_stress_autocorrelation(S.ctx, rows, 0.0, 1.0, 3, G))       # volume 0
    rejected(lambda: api.rc_stress_autocorrelation(S.ctx, rows, 8.0, -1.0, 3, G))      # kT < 0
    p = torch.zeros(4, dtype=torch.int32, device=S.device)
    c = torch.zeros(3, dtype=torch.int64, device=S.device)
    rejected(lambda: L.check(L.load().rc_partner_counts(S.ctx.handle, api._ptr(p), None, None, 4, api._ptr(c),
                                                        None), S.ctx.handle))
    rejected(lambda: S.ctx.set_gather_width(3))
    rejected(lambda: L.check(L.load().rc_set_step_form(S.ctx.handle, 7), S.ctx.handle))
    # the driver: k_max outside [1, 512]
    cfg = S.integrator(dt=0.001, kT=0.1, gamma=1.0, seed=1)
    buf = S.md_buffers(torch.zeros((2, 13), dtype=torch.float64, device=S.device),
                       torch.zeros(2, dtype=torch.int64, device=S.device))
    buf.k_max = 0
    rejected(lambda: api.rc_md_run(S.ctx, buf, s.N, S.box, cfg, 0, 10, None))
