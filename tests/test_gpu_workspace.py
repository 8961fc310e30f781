"""Caller-owned scratch: the context's large buffers live in a torch-owned workspace.

With a workspace attached (System and Batch attach one), the packed list, the
switching sums and the HVP sums come from it: the context itself holds only
the coefficient table, the FP64 reduction rows and the per-block status slots,
O(ntypes^2 + N/64), and a call that needs more than the workspace holds fails
with RC_ERR_WORKSPACE instead of allocating.  All calls through the C ABI."""
import numpy as np
import pytest
import torch

import workloads as W
from paper_1912_08569_amd import RcError, System, api
from paper_1912_08569_amd import _lib as rcl

pytestmark = pytest.mark.gpu


def _small_bound(N):
    # reduction rows (at least 1 MiB), 13 doubles, a bond count and 3 status ints per 64-particle block,
    # 256 x 14 words of reduction slices, table, counters
    return (1 << 20) + (13 * 8 + 4 + 3 * 4) * (N // 64 + 1024) + 8 * 256 * 14 + 4096


def test_context_holds_only_small_buffers():
    s = W.small_reactive(N=20000, density=0.3, seed=81, table=W.swap_table_single(lam=0.8), kT=0.1)
    S = System.from_workload(s)
    S.run(50, S.integrator(dt=0.002, kT=0.1, gamma=1.0, seed=1), log_period=10)
    for form in ("sums", "walk"):
        S.set_step_form(form)
        S.run(20, S.integrator(dt=0.002, kT=0.1, gamma=1.0, seed=1), step0=50 if form == "sums" else 70)
    S.compute_forces(gather="sums")
    V = torch.randn((3, s.N, 4), device="cuda")
    S.hvp_batch(V)                       # grows the caller's workspace, not the context's
    torch.cuda.synchronize()
    own = S.ctx.device_bytes()
    assert own <= _small_bound(s.N), own
    assert S.work.numel() >= api.rc_workspace_bytes(S.ctx, s.N, S.k_max, 3)
    # detached, the context allocates the same buffers itself again
    S.ctx.set_workspace(None)
    S.compute_forces(gather="sums")
    S.run(10, S.integrator(dt=0.002, kT=0.1, gamma=1.0, seed=1), step0=90)
    torch.cuda.synchronize()
    assert S.ctx.device_bytes() > own + 4 * s.N


def test_too_small_a_workspace_is_an_error_not_an_allocation():
    s = W.small_reactive(N=5000, density=0.3, seed=82, table=W.swap_table_single(lam=0.8), kT=0.1)
    S = System.from_workload(s)
    S.build()
    V = torch.randn((2, s.N, 4), device="cuda")
    HV = torch.empty_like(V)
    before = S.ctx.device_bytes()
    with pytest.raises(RcError) as e:     # the workspace holds the sums of one vector
        api.rc_force_hvp_batch(S.ctx, S.pos, S.nlist, S.nn, S.box, V, HV)
    assert e.value.code == rcl.RC_ERR_WORKSPACE
    assert S.ctx.device_bytes() == before
    # the same call through the System grows its workspace and agrees with single products
    out = S.hvp_batch(V)
    one = S.hvp(V[1])
    torch.cuda.synchronize()
    assert torch.equal(out[1], one)
    with pytest.raises(RcError):
        S.ctx.set_workspace(torch.empty(16, dtype=torch.uint8, device="cuda"), s.N, S.k_max, 1)


def test_batch_runs_on_its_workspace():
    from paper_1912_08569_amd import Batch
    reps = [W.small_reactive(N=n, density=0.3, seed=83 + n, table=W.swap_table_single(lam=0.6), kT=0.1)
            for n in (700, 1500, 300)]
    B = Batch(reps, seeds=[1, 2, 3])
    B.set_step_form("sums")
    B.run(30, B.integrator(dt=0.002, kT=0.1, gamma=1.0, seed=0), log_period=10)
    torch.cuda.synchronize()
    assert B.work.numel() >= api.rc_batch_workspace_bytes(B.bc, B.k_max)
