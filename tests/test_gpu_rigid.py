"""Rigid planar bodies (the patchy colloids of Sec. 3.2) on the GPU: one body step
against the oracle, and a Langevin run that keeps the bodies rigid, the plane
and equipartition.  All calls go through the C ABI (rc_compute_forces,
rc_rigid_step)."""
import numpy as np
import pytest

import workloads as W
from oracle import rigid_ref, swap_ref

pytestmark = pytest.mark.gpu


_FRESH = r"""
import sys
sys.path.insert(0, {root!r})
import numpy as np
import workloads as W
s = W.patchy_mixture()                        # host-side set-up first, torch not imported yet
from paper_1912_08569_amd import System       # then the engine (it brings torch's HIP runtime first)
S = System.from_workload(s)
F, ev = S.compute_forces()
print("ok", s.N, bool(np.isfinite(F.cpu().numpy()).all()))
"""


def test_fresh_process_sets_up_the_workload_before_the_device():
    # a process that generates the patchy mixture before its first device use, with torch imported only by
    # the engine package (the order that once mapped two HIP runtimes and failed to bring up the device)
    import os
    import subprocess
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    print("fresh process: patchy_mixture, then System and compute_forces", flush=True)
    out = subprocess.run(["python", "-c", _FRESH.format(root=root)], capture_output=True, text=True, timeout=240)
    assert out.returncode == 0, out.stderr[-3000:]
    assert out.stdout.split()[0] == "ok" and out.stdout.split()[-1] == "True", out.stdout


def _bodies(s):
    from paper_1912_08569_amd import RigidBodies, System
    S = System.from_workload(s)
    return S, RigidBodies(S, s.meta["bodies"], s.meta["theta"], s.meta["omega"])


def _owner(b):
    return np.repeat(np.arange(len(b["centre"])), np.diff(b["first"]))


@pytest.mark.parametrize("kind", ["langevin", "nve"])
def test_rigid_step_matches_oracle(kind):
    s = W.patchy_mixture(seed=1014)
    S, R = _bodies(s)
    gamma = 1.0 if kind == "langevin" else 0.0
    cfg = S.integrator(kind=kind, dt=0.001, kT=1.0, gamma=gamma, seed=21, dim=2)
    S.build()
    x0, v0, _, ty = S.state_by_tag()
    th0, w0 = R.theta.cpu().numpy().copy(), R.omega.cpu().numpy().copy()
    R.run(1, cfg, step0=7)
    x1, v1, _, _ = S.state_by_tag()
    th1, w1 = R.theta.cpu().numpy(), R.omega.cpu().numpy()
    ref = rigid_ref.step(x0, v0, th0, w0, ty, s.meta["bodies"], s.box, s.table, s.mass, 0.001, 1.0, gamma, 21, 7)
    dx = np.abs(swap_ref.min_image(ref["pos"], x1.astype(np.float64), s.box))
    kx = int(np.argmax(np.max(dx, axis=1)))
    b = s.meta["bodies"]
    ob = int(np.searchsorted(b["first"], kx - len(b["centre"]), side="right") - 1) if kx >= len(b["centre"]) else kx
    assert dx.max() < 1e-5, (f"tag {kx} body {ob}: gpu {x1[kx]} oracle {ref['pos'][kx]} start {x0[kx]}; "
                             f"centre gpu {x1[ob]} oracle {ref['pos'][ob]} start {x0[ob]}; "
                             f"theta gpu {th1[ob]} oracle {ref['theta'][ob]} start {th0[ob]}; "
                             f"{int(np.sum(np.max(dx, axis=1) > 1e-5))} particles off")
    dv = np.abs(v1 - ref["vel"])
    k = int(np.argmax(np.max(dv / (1.0 + np.abs(ref["vel"])), axis=1)))
    nb = len(s.meta["bodies"]["centre"])
    assert np.all(dv <= 1e-4 * (1.0 + np.abs(ref["vel"]))), (
        f"tag {k} ({'centre' if k < nb else 'member'}): gpu {v1[k]} oracle {ref['vel'][k]} start {v0[k]}; "
        f"{int(np.sum(np.any(dv > 1e-4 * (1.0 + np.abs(ref['vel'])), axis=1)))} particles off")
    dth = np.abs(np.mod(th1 - ref["theta"] + np.pi, 2 * np.pi) - np.pi)
    assert dth.max() < 1e-5, dth.max()
    assert np.all(np.abs(w1 - ref["omega"]) <= 1e-4 * (1.0 + np.abs(ref["omega"])))
    assert np.all(x1[:, 2] == 0.0) and np.all(v1[:, 2] == 0.0)


def test_rigid_run_keeps_bodies_plane_and_temperature():
    # weak patches (eps 1) so that bonding heats little: equipartition of translation and rotation
    s = W.patchy_mixture(seed=1015, table=W.patchy_table(eps_patch=1.0))
    S, R = _bodies(s)
    cfg = S.integrator(dt=0.001, kT=1.0, gamma=1.0, seed=5, dim=2)
    out = R.run(3000, cfg)
    print(f"rigid patchy mixture: {3000 / out['seconds']:.0f} steps/s, {out['rebuilds']} rebuilds")
    assert out["rebuilds"] >= 1
    x, v, img, ty = S.state_by_tag()
    b = s.meta["bodies"]
    d = swap_ref.min_image(x[b["centre"][_owner(b)]].astype(np.float64), x[b["member"]].astype(np.float64),
                           s.box)
    assert np.allclose(np.linalg.norm(d[:, :2], axis=1), 0.5, atol=2e-5)
    assert np.all(x[:, 2] == 0.0) and np.all(v[:, 2] == 0.0)
    vc = v[b["centre"]].astype(np.float64)
    w = R.omega.cpu().numpy().astype(np.float64)
    kt_trans = float(np.mean(np.sum(vc[:, :2] ** 2, axis=1)) / 2.0)   # unit masses, two degrees of freedom
    kt_rot = float(np.mean(b["inertia"] * w ** 2))
    assert abs(kt_trans - 1.0) < 0.15 and abs(kt_rot - 1.0) < 0.2, (kt_trans, kt_rot)


def test_rigid_argument_errors():
    from paper_1912_08569_amd import RcError
    s = W.patchy_mixture(n_tri=40, n_di=60, L=12.5, seed=1016)
    S, R = _bodies(s)
    with pytest.raises(RcError):   # rigid planar bodies need dim 2
        R.run(1, S.integrator(dt=0.001, kT=1.0, gamma=1.0, seed=5, dim=3))
