"""Throughput of the swap-potential MD step on one MI355X.

Workload: the 1,048,576-particle self-assembly mixture (50 % inert WCA
colloids, 50 % reactive swap sites: eps 15, sigma 0.3, n 10, r_cut 0.45,
lambda 1; colloid-site WCA sigma 0.65), cubic periodic box at density 0.3,
seeded non-overlapping start, BAOAB Langevin kT 0.05, dt 0.001, gamma 1.
A step is one pass of the whole hot path: the fused force+integrate kernel,
the skin test, the cell/neighbour-list rebuilds when the skin is used up, and
the chunk bookkeeping of the driver; energy, virial, kinetic tensor and bond
count are logged every 100 steps.  Inputs are resident on the GPU before the
timed region starts.

Prints one JSON line (metric, value, roofline of the dominant kernel,
CPU-oracle baseline).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0     # MI355X HBM3E, 8 TB/s


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=2000)
    p.add_argument("--warmup", type=int, default=200)
    p.add_argument("--N", type=int, default=1048576)
    p.add_argument("--lam", type=float, default=1.0)
    p.add_argument("--log-period", type=int, default=100)
    p.add_argument("--r-buff", type=float, default=0.3, help="neighbour-list skin")
    p.add_argument("--no-graph", action="store_true")
    p.add_argument("--kernel-steps", type=int, default=400,
                   help="steps of the driver run whose step launches are timed one by one")
    p.add_argument("--cpu-seconds", type=float, default=12.0)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--traffic", type=str, default=os.path.join(ROOT, "profiles", "traffic.json"))
    p.add_argument("--copy-calibration", action="store_true",
                   help="also run a plain 256 MiB device copy (to scale FETCH/WRITE counters)")
    p.add_argument("--no-batch", action="store_true", help="skip the batched-replica comparison")
    p.add_argument("--no-rigid", action="store_true", help="skip the rigid patchy-body run")
    p.add_argument("--rigid-steps", type=int, default=2000)
    p.add_argument("--batch-steps", type=int, default=1000)
    p.add_argument("--seq-steps", type=int, default=200, help="steps of each replica run alone")
    p.add_argument("--no-tune", action="store_true", help="batched run with the default launch settings")
    p.add_argument("--tune-walk", action="store_true",
                   help="let the batch autotuner try the walk form too (2-4x slower on the replica set)")
    p.add_argument("--no-adjoint", action="store_true", help="skip the forward/adjoint timings")
    p.add_argument("--only-extras", action="store_true", help="skip the 1M-particle run (debugging)")
    p.add_argument("--no-dumbbells", action="store_true", help="skip the dumbbell-mixture size sweep")
    p.add_argument("--dumbbell-steps", type=int, default=4000)
    p.add_argument("--dumbbell-warmup", type=int, default=1000)
    p.add_argument("--dumbbell-n", type=str, default="", help="comma-separated sizes (default 2^9 ... 2^17)")
    p.add_argument("--dumbbell-rcut", type=str, default="1.3,1.15", help="comma-separated cutoffs")
    p.add_argument("--no-sweep", action="store_true", help="skip the lambda sweep of the 1M mixture")
    p.add_argument("--sweep-steps", type=int, default=2000)
    p.add_argument("--sweep-warmup", type=int, default=200)
    p.add_argument("--no-vitrimer", action="store_true", help="skip the vitrimer-network run")
    p.add_argument("--vit-steps", type=int, default=2000)
    p.add_argument("--vit-warmup", type=int, default=500)
    p.add_argument("--profile-kernel", action="store_true",
                   help="only the 1M system: build, warm up, then the timed-launch run (for counter runs)")
    return p.parse_args()


def step_kernel_source_hash():
    """Hash of the sources the fused step kernel is built from (counter validity)."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1912_08569_amd", "csrc")
    for name in ("k_forces.hip", "rc_internal.h", "rc_gather.h", "rc_step.h"):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(sysw, seconds):
    """The FP64 oracle on the host cores, as it stands (a baseline, not a target: O(N^2) brute force is
    not a fair CPU MD engine).

    value: the C brute force (plain O(N^2) FP64, OpenMP, every core) on sampled particles of the
    benchmark system: per sampled particle every pair and triplet term acting on it against all N
    particles, which is what one step costs it per particle (the integration is negligible next to it),
    so sampled particles per second = particle-timesteps/s of the oracle.  Beside it: the same at one
    thread, the 1000-particle system's 1000-step BAOAB run (C brute-force forces, numpy integrator) at
    every core and a bounded sample at one thread, and one forward evaluation (C) and one Hessian-vector
    product (numpy) of the 32,768-particle differentiation system."""
    import workloads as W
    from oracle import adjoint_ref, brute, dynamics_ref
    brute.build(force=False)
    cores = len(os.sched_getaffinity(0))
    rng = np.random.default_rng(99)

    def c3_rate(threads, budget):
        m = 2 * threads
        t0 = time.perf_counter()
        brute.forces_subset(sysw.pos, sysw.types, sysw.L, sysw.table, rng.choice(sysw.N, m, replace=False), threads)
        dt = time.perf_counter() - t0
        M = int(max(m, min(200000, m * budget / max(dt, 1e-3))))
        idx = rng.choice(sysw.N, M, replace=False)
        t0 = time.perf_counter()
        brute.forces_subset(sysw.pos, sysw.types, sysw.L, sysw.table, idx, threads)
        return M, time.perf_counter() - t0

    M, dt = c3_rate(cores, seconds)
    M1, dt1 = c3_rate(1, 0.3 * seconds)

    # the plain small system: 1000 reactive particles, density 0.2, BAOAB kT 0.1 dt 0.002 gamma 1
    s1 = W.small_reactive(N=1000, density=0.2, seed=1001, kT=0.1)

    def c1_run(threads, steps):
        x, v = s1.pos.astype(np.float64), s1.vel.astype(np.float64)
        force = lambda y: brute.evaluate(y, s1.types, s1.L, s1.table, threads)["F"]  # noqa: E731
        tags = np.arange(s1.N)
        t0 = time.perf_counter()
        F = None
        for k in range(steps):
            out = dynamics_ref.baoab_step(x, v, s1.types, tags, s1.L, s1.table, s1.mass, 0.002, 0.1, 1.0, 2001, k,
                                          force=F, force_fn=force)
            x, v, F = out["pos"], out["vel"], out["F"]
        return time.perf_counter() - t0

    t_c1 = c1_run(cores, 1000)
    t_c1_1 = c1_run(1, 200)

    # the differentiation system: 32,768 reactive particles, density 0.25, eps 10
    s5 = W.small_reactive(N=32768, density=0.25, seed=1005, table=W.swap_table_single(epsilon=10.0, lam=1.0))
    x5 = s5.pos.astype(np.float64)
    t0 = time.perf_counter()
    brute.evaluate(x5, s5.types, s5.L, s5.table, cores)
    t_fwd = time.perf_counter() - t0
    vec = np.random.default_rng(3005).standard_normal(x5.shape)
    t0 = time.perf_counter()
    adjoint_ref.hvp(x5, s5.types, s5.L, s5.table, vec)
    t_hvp = time.perf_counter() - t0
    return {"value": M / dt, "unit": "particle-timesteps/s", "cores": cores, "kind": "oracle",
            "cpu_model": _cpu_model(),
            "sample": f"forces on {M} random particles of the {sysw.N}-particle system, each against all "
                      f"{sysw.N} particles (FP64 brute force, {dt:.1f} s at {cores} threads)",
            "single_thread": {"value": M1 / dt1, "unit": "particle-timesteps/s", "cores": 1,
                              "sample": f"{M1} particles, {dt1:.1f} s"},
            "small_system_run": {"workload": "1000 reactive particles, density 0.2, 1000 BAOAB steps kT 0.1 dt 0.002",
                                 "value": 1000 * 1000 / t_c1, "unit": "particle-timesteps/s", "cores": cores,
                                 "seconds": round(t_c1, 2),
                                 "single_thread_value": 1000 * 200 / t_c1_1,
                                 "single_thread_sample": f"200 steps, {t_c1_1:.1f} s"},
            "differentiation_system": {"workload": "32768 reactive particles, density 0.25, eps 10 (random start)",
                                       "forward_s": round(t_fwd, 3), "forward_cores": cores,
                                       "forward_kind": "C brute force, O(N^2)",
                                       "hvp_s": round(t_hvp, 3), "hvp_kind": "numpy, candidate pairs by k-d tree",
                                       "hvp_cores": 1},
            "note": "baseline only: the oracle is an O(N^2) brute force written for checking, not a CPU MD engine"}


def _log_steps(step0, n, lp, skip_first):
    """Step indices of the rows a run logs (multiples of the period, then the end)."""
    s = [k for k in range(step0, step0 + n) if lp > 0 and k % lp == 0 and not (skip_first and k == step0)]
    return s + [step0 + n]


def lambda_sweep(a, sysw):
    """The self-assembly mixture at lambda 0, 0.5, 1 and 1.5 (the swap-barrier knob of Sec. 2) from the
    same start: particle-timesteps/s of `sweep_steps` steps after `sweep_warmup`, and the bond-count
    trajectory of the whole run (a row every log period)."""
    import torch

    from paper_1912_08569_amd import System
    rows = []
    for lam in (0.0, 0.5, 1.0, 1.5):
        S = System(sysw.pos, sysw.types, sysw.L, sysw.table.with_lambda(lam), vel=sysw.vel, mass=sysw.mass,
                   r_buff=a.r_buff, k_max=32)
        cfg = S.integrator(dt=0.001, kT=0.05, gamma=1.0, seed=2003)
        S.build()
        r0 = S.run(a.sweep_warmup, cfg, step0=0, log_period=a.log_period)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = S.run(a.sweep_steps, cfg, step0=a.sweep_warmup, log_period=a.log_period)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        steps = _log_steps(0, a.sweep_warmup, a.log_period, False) + \
            _log_steps(a.sweep_warmup, a.sweep_steps, a.log_period, bool(r.stats.list_kept))
        bonds = [int(b) for b in np.concatenate([r0.bonds, r.bonds])]
        assert len(steps) == len(bonds)
        rows.append({"lambda": lam, "particle_timesteps_per_s": a.N * a.sweep_steps / dt,
                     "us_per_step": round(dt / a.sweep_steps * 1e6, 3), "rebuilds": int(r.stats.rebuilds),
                     "rollbacks": int(r.stats.rollbacks), "chunks": int(r.stats.chunks),
                     "bond_trajectory": {"steps": steps, "bonds": bonds}})
        print(f"# lambda {lam}: {rows[-1]['us_per_step']:.2f} us/step, bonds {bonds[0]} -> {bonds[-1]}, "
              f"rebuilds {rows[-1]['rebuilds']}, rollbacks {rows[-1]['rollbacks']}, chunks {rows[-1]['chunks']}",
              file=sys.stderr, flush=True)
        del S
        torch.cuda.empty_cache()
    return {"workload": f"self-assembly mixture N={a.N}, density 0.3, Langevin kT 0.05 dt 0.001, one start",
            "unit": "particle-timesteps/s", "warmup": a.sweep_warmup, "steps": a.sweep_steps,
            "log_period": a.log_period, "rows": rows}


def vitrimer_bench(a):
    """The vitrimer-like network: 4000 chains of 16 beads and 1600 crosslinker dimers (67,200 beads,
    FENE K 30 R0 1.5, WCA, 10 % reactive sites with the swap potential eps 20 sigma 0.3 n 10, lambda 1)
    at density 0.85, Langevin kT 1 dt 0.002: particle-timesteps/s after a gentle push-off (dt 2e-4)
    of the grown start's 0.8 sigma contacts and a relaxation."""
    import torch

    import workloads as W
    from paper_1912_08569_amd import System
    t_gen = time.perf_counter()
    s = W.vitrimer_network()
    print(f"# vitrimer network: {s.N} beads generated in {time.perf_counter() - t_gen:.1f}s", file=sys.stderr,
          flush=True)
    S = System.from_workload(s)
    S.run(3000, S.integrator(dt=2e-4, kT=1.0, gamma=1.0, seed=23))
    cfg = S.integrator(dt=0.002, kT=1.0, gamma=1.0, seed=23)
    S.run(a.vit_warmup, cfg, step0=3000, log_period=a.log_period)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = S.run(a.vit_steps, cfg, step0=3000 + a.vit_warmup, log_period=a.log_period)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    out = {"workload": "vitrimer-like network: 4000 chains x 16 beads + 1600 crosslinker dimers (67,200 beads), "
                       "density 0.85, FENE K 30 R0 1.5, WCA, swap sites eps 20 sigma 0.3 n 10 lambda 1, "
                       "Langevin kT 1 dt 0.002, log every 100 steps",
           "unit": "particle-timesteps/s", "value": s.N * a.vit_steps / dt, "steps": a.vit_steps,
           "us_per_step": round(dt / a.vit_steps * 1e6, 3), "rebuilds": int(r.stats.rebuilds),
           "step_form": S.ctx.step_form, "mean_list_length": round(S.mean_list_length(), 3),
           "bonds_final": int(r.bonds[-1]), "energy_final": float(r.ev[-1, 0])}
    print(f"# vitrimer: {out['us_per_step']:.2f} us/step", file=sys.stderr, flush=True)
    del S
    torch.cuda.empty_cache()
    return out


def batch_bench(a):
    """256 replicas (N ~ logU[500, 20000], lambda ~ U[0, 1.5], density 0.2-0.4, 0-50 % inert WCA) advanced
    by one launch per step, against the same replicas run one after the other with the single-system
    engine.  Both log energies, virials and bonds every 100 steps."""
    import torch

    import workloads as W
    from paper_1912_08569_amd import Batch, System, tune

    t_gen = time.perf_counter()
    reps = W.replica_set()
    R = len(reps)
    ntot = int(sum(s.N for s in reps))
    print(f"# replicas: R={R}, {ntot} particles, generated in {time.perf_counter() - t_gen:.1f}s", file=sys.stderr,
          flush=True)
    mk_cfg = lambda S, seed=0: S.integrator(dt=0.002, kT=0.1, gamma=1.0, seed=seed)  # noqa: E731
    tuned = None
    r_buff, form, width, G = 0.3, "sums", 4, 32   # the tuned settings of the replica set
    if not a.no_tune:
        factory = lambda rb: Batch(reps, r_buff=rb, seeds=range(R))  # noqa: E731
        probe = factory(0.3)
        cfg = mk_cfg(probe)
        del probe
        # every candidate from the same start, timed over the benchmark's own window
        tuned = tune.autotune(factory, cfg, signature=f"replica_set R={R} N={ntot} seed=1004",
                              r_buffs=(0.2, 0.3, 0.45), forms=("sums", "walk") if a.tune_walk else ("sums",),
                              steps=a.batch_steps, warmup=200, cache=None,
                              log=lambda m: print("# " + m, file=sys.stderr, flush=True))
        r_buff, form, width, G = tuned["r_buff"], tuned["form"], tuned["width"], tuned["graph_steps"]
    B = Batch(reps, r_buff=r_buff, seeds=range(R))
    B.set_step_form(form)
    B.set_gather_width(width)
    cfg = mk_cfg(B)
    B.run(200, cfg, step0=0, log_period=a.log_period, graph_steps=G)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rb = B.run(a.batch_steps, cfg, step0=200, log_period=a.log_period, graph_steps=G)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    batched = ntot * a.batch_steps / tb
    print(f"# batched: {a.batch_steps} steps in {tb * 1e3:.1f} ms ({tb / a.batch_steps * 1e6:.2f} us/step), "
          f"rebuilds {rb.stats.rebuilds}", file=sys.stderr, flush=True)
    del B
    torch.cuda.empty_cache()
    # the same replicas alone, one after the other (default settings of the single-system engine)
    systems = [System.from_workload(s, r_buff=0.3) for s in reps]
    cfgs = [mk_cfg(S, seed=r) for r, S in enumerate(systems)]
    for S, c in zip(systems, cfgs):
        S.run(20, c, step0=0, log_period=a.log_period)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for S, c in zip(systems, cfgs):
        S.run(a.seq_steps, c, step0=20, log_period=a.log_period)
    torch.cuda.synchronize()
    ts = time.perf_counter() - t0
    seq = ntot * a.seq_steps / ts
    print(f"# sequential: {R} x {a.seq_steps} steps in {ts * 1e3:.1f} ms", file=sys.stderr, flush=True)
    out = {"workload": f"{R} replicas, N ~ logU[500, 20000] ({ntot} particles), lambda ~ U[0, 1.5], "
                       "density 0.2-0.4, inert fraction 0-0.5, Langevin kT 0.1 dt 0.002, log every 100 steps",
           "unit": "particle-timesteps/s", "batched": batched, "batched_ms_per_step": tb / a.batch_steps * 1e3,
           "batched_steps": a.batch_steps, "sequential_plain": seq,
           "sequential_ms_per_replica_step": ts / (R * a.seq_steps) * 1e3, "sequential_steps": a.seq_steps,
           "speedup": batched / seq, "settings": {"r_buff": r_buff, "step_form": form, "gather_width": width, "graph_steps": G}}
    if tuned is not None:
        out["autotune"] = [{k: c[k] for k in ("r_buff", "form", "width", "graph_steps", "us_per_step")}
                           for c in tuned["candidates"]]
    del systems
    torch.cuda.empty_cache()
    return out


def adjoint_bench(a):
    """Forward vs adjoint on 32768 reactive particles (density 0.25, eps 10, sigma 1, n 10, lambda 1):
    forces + energy/virial, dE/d(eps, sigma, lambda), and H v for 64 random unit vectors."""
    import torch

    import workloads as W
    from paper_1912_08569_amd import System

    s = W.small_reactive(N=32768, density=0.25, seed=1005, table=W.swap_table_single(epsilon=10.0, lam=1.0))
    S = System.from_workload(s)
    # equilibration of the random start (contacts at 0.8 sigma): a gentle push-off, then 1000 BAOAB
    # steps at kT = 1; timings and the fit start from the equilibrated state
    S.run(1000, S.integrator(dt=2e-4, kT=1.0, gamma=1.0, seed=5), step0=0)
    S.run(1000, S.integrator(dt=0.002, kT=1.0, gamma=1.0, seed=5), step0=1000)
    S.build()
    x_eq, v_eq, _, ty_eq = S.state_by_tag()
    rng = np.random.default_rng(7)
    V = rng.standard_normal((64, s.N, 3))
    V /= np.linalg.norm(V.reshape(64, -1), axis=1)[:, None, None]
    vs = []
    for k in range(64):
        v = np.zeros((s.N, 4), np.float32)
        v[:, :3] = V[k]
        vs.append(S.to_engine_order(v))

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps * 1e3   # us

    from paper_1912_08569_amd import api
    from paper_1912_08569_amd import _lib as rcl
    nt = S.ctx.ntypes
    g = torch.zeros(nt * nt * 3, dtype=torch.float64, device=S.device)
    hv = torch.empty_like(S.pos)
    fwd = timed(lambda: api.rc_compute_forces(S.ctx, S.pos, S.nlist, S.nn, S.box, S.force, S.ev,
                                              rcl.RC_FORCE_GATHER, S.status), 200)
    fwd_tri = timed(lambda: api.rc_compute_forces(S.ctx, S.pos, S.nlist, S.nn, S.box, S.force, S.ev, 0,
                                                  S.status), 200)
    grad = timed(lambda: api.rc_param_grad(S.ctx, S.pos, S.nlist, S.nn, S.box, g), 200)
    it = iter(range(10 ** 9))
    hvp = timed(lambda: api.rc_force_hvp(S.ctx, S.pos, S.nlist, S.nn, S.box, vs[next(it) % 64], hv), 640)
    V64 = torch.stack(list(vs[:64])).contiguous()       # the 64 tangent vectors of the workload
    HV64 = torch.empty_like(V64)
    S.reserve_hvp_vectors(64)
    hvp64 = timed(lambda: api.rc_force_hvp_batch(S.ctx, S.pos, S.nlist, S.nn, S.box, V64, HV64), 50)
    adj = vs[0]
    vjp = timed(lambda: api.rc_param_vjp(S.ctx, S.pos, S.nlist, S.nn, S.box, adj, g), 200)
    fwd_sums = timed(lambda: api.rc_compute_forces(S.ctx, S.pos, S.nlist, S.nn, S.box, S.force, S.ev,
                                                   rcl.RC_FORCE_SUMS, S.status), 200)
    best = min(fwd, fwd_sums, fwd_tri)
    out = {"workload": "32768 reactive particles, density 0.25, eps 10, sigma 1, n 10, lambda 1, equilibrated at kT 1",
           "forward_us": best, "forward_walk_form_us": fwd, "forward_sums_form_us": fwd_sums,
           "forward_triplet_kernel_us": fwd_tri,
           "param_grad_us": grad, "param_vjp_us": vjp, "hvp_us_per_vector": hvp,
           "fwd_plus_param_grad_over_fwd": (best + grad) / best, "hvp_over_fwd": hvp / best,
           "hvp_64_vectors_ms": hvp * 64 / 1e3, "hvp_64_batched_ms": hvp64 / 1e3,
           "hvp_batched_us_per_vector": hvp64 / 64, "hvp_batched_over_fwd": hvp64 / 64 / best}
    # HVP roofline: per particle and vector the forward's bytes (pos 16, nn 4, list 4k, force out 16)
    # plus the tangent vector in and the product out (16 + 16), i.e. 68 + 4k
    kbar = S.mean_list_length()
    hb = 68.0 + 4.0 * kbar
    ach = s.N * hb / (hvp * 1e-6) / 1e9
    ach64 = s.N * hb / (hvp64 / 64 * 1e-6) / 1e9
    out["hvp_roofline"] = {"bound": "hbm", "unit": "GB/s", "peak": HBM_PEAK_GBS,
                           "algorithmic_bytes_per_particle": round(hb, 2), "mean_list_length": round(kbar, 3),
                           "achieved": round(ach, 1), "frac": round(ach / HBM_PEAK_GBS, 4),
                           "achieved_batched_per_vector": round(ach64, 1),
                           "frac_batched": round(ach64 / HBM_PEAK_GBS, 4)}
    # one iteration of the lambda fit: 200 BAOAB steps forward, checkpointed backward (segments of 20)
    from paper_1912_08569_amd.autograd import SwapModel
    from paper_1912_08569_amd.fit import TrajectoryFit
    M = SwapModel(System(x_eq, ty_eq, s.L, s.table, vel=v_eq, mass=s.mass))
    fit = TrajectoryFit(M, torch.from_numpy(np.ascontiguousarray(x_eq)).cuda(),
                        torch.from_numpy(np.ascontiguousarray(v_eq)).cuda(),
                        torch.ones(s.N, device="cuda"), dt=0.002, kT=0.1, gamma=1.0, steps=200, segment=20,
                        n_swap=s.N, seed=1)
    theta0 = M.theta()
    with torch.no_grad():
        target = 1.05 * float(fit.observable(theta0))
    mask = torch.zeros_like(theta0)
    mask[0, 0, 2] = 1.0

    def iteration():
        lam = torch.tensor(1.0, dtype=torch.float64, requires_grad=True)
        L = fit.loss(theta0 * (1 - mask) + mask * lam, target)
        (gl,) = torch.autograd.grad(L, lam)
        return float(gl)

    iteration()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    gl = iteration()
    torch.cuda.synchronize()
    t_it = time.perf_counter() - t0
    with torch.no_grad():
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fit.observable(theta0)
        torch.cuda.synchronize()
        t_fwd = time.perf_counter() - t0
    out.update({"fit_iteration_ms": t_it * 1e3, "fit_forward_only_ms": t_fwd * 1e3,
                "fit_backward_over_forward": (t_it - t_fwd) / t_fwd, "fit_steps": 200, "fit_segment": 20,
                "fit_dloss_dlambda": gl, "fit_list_rebuilds": M.rebuilds})
    return out


def rigid_bench(a):
    """The 2d patchy mixture of Sec. 3.2 as rigid bodies: steps/s of the body step (forces, body kernel,
    list rebuilds when due; one host check of the path lengths per step)."""
    import workloads as W
    from paper_1912_08569_amd import RigidBodies, System
    s = W.patchy_mixture()
    S = System.from_workload(s)
    R = RigidBodies(S, s.meta["bodies"], s.meta["theta"], s.meta["omega"])
    cfg = S.integrator(dt=0.001, kT=1.0, gamma=1.0, seed=9, dim=2)
    R.run(200, cfg)
    out = R.run(a.rigid_steps, cfg, step0=200)
    print(f"# rigid patchy mixture: {a.rigid_steps / out['seconds']:.0f} steps/s", file=sys.stderr, flush=True)
    return {"workload": "2d patchy mixture: 400 trifunctional + 600 difunctional rigid disks (3400 particles), "
                        "box 39.63, patch swap eps 10 sigma 0.1 n 6 r_cut 0.2, Langevin kT 1 dt 0.001",
            "unit": "timesteps/s", "steps": a.rigid_steps, "steps_per_s": round(a.rigid_steps / out["seconds"], 1),
            "rebuilds": out["rebuilds"], "particles": int(s.N), "bodies": int(len(s.meta["bodies"]["centre"]))}


def dumbbell_bench(a):
    """The paper's performance workload: the A:B = 3:2 dumbbell mixture (n = 100, WCA AA/BB, density
    0.125, kT 0.03) at N = 2^9 ... 2^17 particles and cutoffs 1.3 and 1.15, as timesteps per second.
    Langevin dt 0.001, neighbour-list skin 0.3, log every 100 steps; each size is relaxed for
    `dumbbell_warmup` steps from its random start before `dumbbell_steps` timed steps."""
    import torch

    import workloads as W
    from paper_1912_08569_amd import System

    rows = []
    sizes = [int(v) for v in a.dumbbell_n.split(",")] if a.dumbbell_n else [1 << x for x in range(9, 18)]
    for rcut in [float(v) for v in a.dumbbell_rcut.split(",")]:
        for N in sizes:
            x = N.bit_length() - 1
            s = W.dumbbell_mixture(N=N, rcut=rcut, seed=1100 + x)
            S = System.from_workload(s, r_buff=0.3)
            cfg = S.integrator(dt=0.001, kT=0.03, gamma=1.0, seed=2100 + x)
            S.run(a.dumbbell_warmup, cfg, step0=0, log_period=a.log_period)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            res = S.run(a.dumbbell_steps, cfg, step0=a.dumbbell_warmup, log_period=a.log_period)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            nn = S.nn
            kbar = float(((nn & 0xFFFF) + (nn >> 16)).float().mean().item())
            bonds = int(res.bonds[-1]) if res.bonds is not None and len(res.bonds) else None
            form = S.ctx.step_form
            rows.append({"N": N, "r_cut": rcut, "steps_per_s": round(a.dumbbell_steps / dt, 1),
                         "us_per_step": round(dt / a.dumbbell_steps * 1e6, 3),
                         "particle_steps_per_s": N * a.dumbbell_steps / dt, "mean_list_length": round(kbar, 3),
                         "step_form": form, "rebuilds": int(res.stats.rebuilds), "bonds": bonds,
                         "n_b": int(np.count_nonzero(s.types == 1))})
            print(f"# dumbbells N={N} r_cut={rcut}: {rows[-1]['steps_per_s']:.0f} steps/s "
                  f"({rows[-1]['us_per_step']:.2f} us/step), k={kbar:.2f}, form {form}, bonds {bonds}",
                  file=sys.stderr, flush=True)
            del S
    torch.cuda.empty_cache()
    return {"workload": "dumbbell mixture A:B = 3:2, n 100, WCA AA/BB, density 0.125, Langevin kT 0.03 dt 0.001, "
                        "skin 0.3, log every 100 steps", "unit": "timesteps/s",
            "warmup": a.dumbbell_warmup, "steps": a.dumbbell_steps, "rows": rows}


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this engine runs on one GPU; --gpus must be 1",
                          "n_gpus_requested": a.gpus}))
        sys.exit(2)
    import torch

    import workloads as W
    from paper_1912_08569_amd import System, api
    from paper_1912_08569_amd import _lib as rcl

    torch.cuda.set_device(0)
    if a.only_extras:
        out = {}
        if not a.no_adjoint:
            out["adjoint"] = adjoint_bench(a)
        if not a.no_batch:
            out["batch"] = batch_bench(a)
        if not a.no_dumbbells:
            out["dumbbells"] = dumbbell_bench(a)
        if not a.no_rigid:
            out["rigid"] = rigid_bench(a)
        print(json.dumps(out), flush=True)
        return
    t_gen = time.perf_counter()
    sysw = W.assembly_mixture(N=a.N, lam=a.lam, seed=1003, kT=0.05)
    print(f"# generated {sysw.name} in {time.perf_counter() - t_gen:.1f}s, L={sysw.L}", file=sys.stderr,
          flush=True)
    S = System.from_workload(sysw, r_buff=a.r_buff, k_max=32)
    cfg = S.integrator(dt=0.001, kT=0.05, gamma=1.0, seed=2003)
    S.build()
    use_graph = not a.no_graph
    # warm-up (also relaxes the random start)
    S.run(a.warmup, cfg, step0=0, log_period=a.log_period, use_graph=use_graph)
    torch.cuda.synchronize()
    if a.profile_kernel:
        # counter runs: nothing but the step launches of a driver run, each launched directly
        rk = S.run(a.kernel_steps, cfg, step0=a.warmup, log_period=a.log_period, time_kernels=True)
        out = {"kernel": "k_step", "N": a.N, "launches": int(rk.stats.kernel_launches),
               "kernel_us": rk.stats.kernel_ms / max(1, rk.stats.kernel_launches) * 1e3,
               "mean_list_length": S.mean_list_length(), "step_kernel_source_hash": step_kernel_source_hash()}
        if a.copy_calibration:   # a plain 256 MiB device copy: the scale of the byte counters
            src = torch.empty(64 << 20, dtype=torch.float32, device="cuda")
            dst = torch.empty_like(src)
            for _ in range(3):
                dst.copy_(src)
            torch.cuda.synchronize()
            out["copy_calibration_bytes"] = int(src.numel() * 4)
        print(json.dumps(out), flush=True)
        return
    # ---- timed region: exactly `steps` steps ------------------------------------------
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = S.run(a.steps, cfg, step0=a.warmup, log_period=a.log_period, use_graph=use_graph)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_events = e0.elapsed_time(e1)
    sec = wall
    value = a.N * a.steps / sec
    st = res.stats
    print(f"# {a.steps} steps in {sec * 1e3:.1f} ms ({sec / a.steps * 1e6:.2f} us/step; events "
          f"{ms_events:.1f} ms); rebuilds {st.rebuilds} rollbacks {st.rollbacks} chunks {st.chunks}",
          file=sys.stderr, flush=True)
    # ---- dominant kernel: the fused step, every launch of a driver run timed by its own events ----
    # The kernel slows as its list ages (about 25 us on a fresh list, 27 us a hundred steps later at
    # 1M particles), so it is timed over whole list lives: a further run of the driver continues the
    # state with every plain step launched directly between events (the same trajectory, bit for
    # bit, as graph replays), and the average is taken over all of its step launches.
    nn = S.nn
    k_before = float(((nn & 0xFFFF) + (nn >> 16)).float().mean().item())  # n_swap | n_other << 16
    rk = S.run(a.kernel_steps, cfg, step0=a.warmup + a.steps, log_period=a.log_period, use_graph=use_graph,
               time_kernels=True)
    nn = S.nn
    k_after = float(((nn & 0xFFFF) + (nn >> 16)).float().mean().item())
    kbar = 0.5 * (k_before + k_after)
    t_kernel = rk.stats.kernel_ms / max(1, rk.stats.kernel_launches) * 1e-3
    # Algorithmic bytes of one particle-step of the method (force pass: pos 16 + nn 4 + list 4k
    # + force out 16; integrate pass: pos, vel, force, reference position in 64, pos, vel out 32),
    # i.e. 132 + 4k.  The fused kernel does the whole step but never stores a force array or a
    # reference position, so it moves only 68 + 4k of them; both are reported.
    bytes_per_particle = 132.0 + 4.0 * kbar
    fused_bytes_per_particle = 68.0 + 4.0 * kbar
    achieved = a.N * bytes_per_particle / t_kernel / 1e9
    achieved_fused = a.N * fused_bytes_per_particle / t_kernel / 1e9
    traffic = None
    if os.path.exists(a.traffic):
        try:
            with open(a.traffic) as f:
                tr = json.load(f)
            if (tr.get("kernel") == "k_step" and int(tr.get("N", 0)) == a.N
                    and tr.get("source_hash") == step_kernel_source_hash()):
                traffic = tr.get("bytes_per_launch")
        except Exception:
            traffic = None
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "kernel": "k_step (fused force + BAOAB)", "kernel_us": round(t_kernel * 1e6, 3),
            "timed_launches": int(rk.stats.kernel_launches), "timed_run_steps": a.kernel_steps,
            "timed_run_rebuilds": int(rk.stats.rebuilds),
            "algorithmic_bytes_per_particle": round(bytes_per_particle, 2),
            "fused_kernel_bytes_per_particle": round(fused_bytes_per_particle, 2),
            "achieved_fused_bytes": round(achieved_fused, 1), "frac_fused_bytes": round(achieved_fused / HBM_PEAK_GBS, 4),
            "mean_list_length": round(kbar, 3)}
    out = {
        "metric": "particle-timesteps/s", "value": value, "unit": "particle-timesteps/s",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup, "ms_per_step": sec / a.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"swap/WCA self-assembly mixture, N={a.N}, density 0.3, lambda {a.lam}, "
                               "Langevin kT 0.05 dt 0.001, log every 100 steps",
                   "N": a.N, "lambda": a.lam, "graph": use_graph, "r_buff": a.r_buff, "rebuilds": int(st.rebuilds),
                   "rollbacks": int(st.rollbacks), "chunks": int(st.chunks), "list_kept": int(st.list_kept),
                   "bonds_final": int(res.bonds[-1]) if res.bonds is not None and len(res.bonds) else None},
        "roofline": roof,
    }
    if a.copy_calibration:
        src = torch.empty(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = int(src.numel() * 4)
    out["step_kernel_source_hash"] = step_kernel_source_hash()
    del S
    torch.cuda.empty_cache()
    if not a.no_sweep:
        out["lambda_sweep"] = lambda_sweep(a, sysw)
    if not a.no_vitrimer:
        out["vitrimer"] = vitrimer_bench(a)
    if not a.no_adjoint:
        out["adjoint"] = adjoint_bench(a)
    if not a.no_batch:
        out["batch"] = batch_bench(a)
    if not a.no_dumbbells:
        out["dumbbells"] = dumbbell_bench(a)
    if not a.no_rigid:
        out["rigid"] = rigid_bench(a)
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(sysw, a.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
