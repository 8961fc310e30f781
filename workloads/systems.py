"""Input generators: positions, types, velocities, boxes and coefficient tables.

Conventions shared by every generated system
--------------------------------------------
* Cubic periodic box, origin centred.  The edge ``L`` is rounded to the
  nearest FP32 value (so that the engine's FP32 positions and the FP64 oracle
  see the same box).
* Positions are FP32 values in ``[-L/2, L/2)`` (shape ``(N, 3)``).
* ``types`` is int32 in ``[0, ntypes)``; ``tags`` are ``0..N-1``.
* Coefficient tables are symmetric ``ntypes x ntypes`` arrays of
  (kind, epsilon, sigma, n, r_cut, lambda), one entry per unordered type pair,
  following the per-type-pair coefficient set of the paper's potential
  (Sec. 2, the revcross coefficient list: sigma, n, epsilon, lambda3, plus a
  cutoff).  ``kind`` selects the pair function: 0 = no interaction,
  1 = swap (generalized LJ + three-body), 2 = WCA (purely repulsive LJ).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np
from scipy.spatial import cKDTree

KIND_NONE = 0
KIND_SWAP = 1
KIND_WCA = 2
# WCA is the 12-6 LJ cut at its minimum, 2^(1/6) sigma (Weeks-Chandler-Andersen).
WCA_CUT_FACTOR = 2.0 ** (1.0 / 6.0)


@dataclasses.dataclass
class PairTable:
    """Symmetric per-type-pair coefficient table (float64 / int arrays)."""
    kind: np.ndarray      # int32 [nt, nt]
    epsilon: np.ndarray   # float64 [nt, nt]
    sigma: np.ndarray     # float64 [nt, nt]
    n: np.ndarray         # int32 [nt, nt]   (exponent of the swap pair; 6 for WCA)
    rcut: np.ndarray      # float64 [nt, nt]
    lam: np.ndarray       # float64 [nt, nt] (three-body lambda; 0 unless swap)

    @property
    def ntypes(self) -> int:
        return int(self.kind.shape[0])

    @staticmethod
    def empty(nt: int) -> "PairTable":
        return PairTable(kind=np.zeros((nt, nt), np.int32),
                         epsilon=np.zeros((nt, nt)), sigma=np.ones((nt, nt)),
                         n=np.full((nt, nt), 6, np.int32), rcut=np.zeros((nt, nt)),
                         lam=np.zeros((nt, nt)))

    def set(self, a: int, b: int, kind: int, epsilon: float = 1.0, sigma: float = 1.0,
            n: int = 6, rcut: Optional[float] = None, lam: float = 0.0) -> "PairTable":
        if rcut is None:
            rcut = WCA_CUT_FACTOR * sigma if kind == KIND_WCA else 0.0
        for (p, q) in ((a, b), (b, a)):
            self.kind[p, q] = kind
            self.epsilon[p, q] = epsilon
            self.sigma[p, q] = sigma
            self.n[p, q] = n
            self.rcut[p, q] = rcut
            self.lam[p, q] = lam
        return self

    def copy(self) -> "PairTable":
        return PairTable(*(np.array(getattr(self, f.name)) for f in dataclasses.fields(self)))

    def with_lambda(self, lam: float) -> "PairTable":
        t = self.copy()
        t.lam = np.where(t.kind == KIND_SWAP, float(lam), 0.0)
        return t

    def max_rcut(self) -> float:
        m = np.where(self.kind != KIND_NONE, self.rcut, 0.0)
        return float(m.max())


@dataclasses.dataclass
class System:
    """One periodic system: FP32 positions and the data the engine needs."""
    pos: np.ndarray            # float32 [N, 3] in [-L/2, L/2)
    types: np.ndarray          # int32 [N]
    L: float                   # FP32-exact box edge (as a Python float)
    table: PairTable
    mass: np.ndarray           # float64 [ntypes]
    vel: Optional[np.ndarray] = None   # float32 [N, 3]
    name: str = ""
    meta: dict = dataclasses.field(default_factory=dict)
    bonds: Optional[np.ndarray] = None  # int32 [N, 2] spring partner tags per tag (-1 none)
    fene: Optional[tuple] = None        # (K, R0) of the springs

    @property
    def N(self) -> int:
        return int(self.pos.shape[0])

    @property
    def tags(self) -> np.ndarray:
        return np.arange(self.N, dtype=np.int32)

    @property
    def box(self) -> np.ndarray:
        return np.broadcast_to(np.asarray(self.L, dtype=np.float64), (3,)).copy()


def fp32_box(N: int, density: float) -> float:
    """Cubic box edge for N particles at number density ``density``, rounded to FP32."""
    return float(np.float32((N / density) ** (1.0 / 3.0)))


def wrap_fp32(x: np.ndarray, L: float) -> np.ndarray:
    """Round float64 coordinates to FP32 and fold them into [-L/2, L/2)."""
    h = np.float32(0.5 * L)
    xf = np.asarray(x, dtype=np.float64)
    xf = xf - L * np.floor(xf / L + 0.5)
    out = xf.astype(np.float32)
    out = np.where(out >= h, out - np.float32(L), out)
    out = np.where(out < -h, out + np.float32(L), out)
    return out.astype(np.float32)


def rsa_positions(rng: np.random.Generator, L: float, counts: Sequence[int],
                  min_dist: np.ndarray, max_rounds: int = 200) -> tuple:
    """Random sequential addition of ``counts[t]`` particles of each type.

    A candidate is rejected when its periodic distance to any accepted
    particle of type u is <= ``min_dist[t, u]``.  Types are placed in the order
    given; candidates are drawn in batches and conflicts inside a batch are
    resolved by dropping the later candidate.  Returns (pos float32, types).
    """
    nt = len(counts)
    placed: List[np.ndarray] = [np.zeros((0, 3), np.float32) for _ in range(nt)]
    half = 0.5 * L
    for t in range(nt):
        need = int(counts[t])
        rounds = 0
        while need > 0:
            rounds += 1
            if rounds > max_rounds:
                raise RuntimeError("random sequential addition did not converge")
            m = max(16, int(need * 1.15) + 16)
            cand = wrap_fp32(rng.uniform(-half, half, size=(m, 3)), L)
            c64 = cand.astype(np.float64) + half
            c64 = np.minimum(c64, np.nextafter(L, 0.0))
            keep = np.ones(m, dtype=bool)
            for u in range(nt):
                if placed[u].shape[0] == 0:
                    continue
                thr = float(min_dist[t, u])
                if thr <= 0:
                    continue
                p64 = np.minimum(placed[u].astype(np.float64) + half, np.nextafter(L, 0.0))
                tree = cKDTree(p64, boxsize=L)
                d, _ = tree.query(c64, k=1, distance_upper_bound=thr * 1.000001 + 1e-12)
                keep &= ~(d <= thr * 1.000001)
            idx = np.nonzero(keep)[0]
            sub = c64[idx]
            thr = float(min_dist[t, t])
            if thr > 0 and sub.shape[0] > 1:
                tree = cKDTree(sub, boxsize=L)
                pairs = tree.query_pairs(thr * 1.000001, output_type="ndarray")
                if pairs.size:
                    drop = np.zeros(sub.shape[0], dtype=bool)
                    # greedy: walk pairs in order, drop the later index if both still kept
                    for a, b in pairs[np.lexsort((pairs[:, 1], pairs[:, 0]))]:
                        if not drop[a] and not drop[b]:
                            drop[b] = True
                    idx = idx[~drop]
            idx = idx[:need]
            placed[t] = np.concatenate([placed[t], cand[idx]], axis=0)
            need -= idx.size
    pos = np.concatenate(placed, axis=0).astype(np.float32)
    types = np.concatenate([np.full(int(c), t, np.int32) for t, c in enumerate(counts)])
    return pos, types


def maxwell_velocities(rng: np.random.Generator, types: np.ndarray, mass: np.ndarray,
                       kT: float) -> np.ndarray:
    """Maxwell-Boltzmann velocities at temperature kT with zero net momentum."""
    m = mass[types][:, None]
    v = rng.standard_normal((types.shape[0], 3)) * np.sqrt(kT / m)
    p = (m * v).sum(axis=0) / m.sum()
    v = v - p[None, :]
    return v.astype(np.float32)


def swap_table_single(epsilon=1.0, sigma=1.0, n=10, rcut=1.5, lam=1.0) -> PairTable:
    """One reactive type interacting through the swap potential."""
    return PairTable.empty(1).set(0, 0, KIND_SWAP, epsilon, sigma, n, rcut, lam)


def assembly_table(lam: float, eps_site=15.0, sigma_site=0.3, n=10, rcut_site=0.45,
                   sigma_colloid=1.0, sigma_cross=0.65) -> PairTable:
    """Type 0 = inert WCA colloid, type 1 = reactive site.

    colloid-colloid WCA (sigma 1), colloid-site WCA (sigma 0.65),
    site-site swap (eps 15, sigma 0.3, n 10, r_cut 0.45, lambda).
    """
    t = PairTable.empty(2)
    t.set(0, 0, KIND_WCA, 1.0, sigma_colloid, 6)
    t.set(0, 1, KIND_WCA, 1.0, sigma_cross, 6)
    t.set(1, 1, KIND_SWAP, eps_site, sigma_site, n, rcut_site, lam)
    return t


def planar_reactive(N=1000, L=39.63, Lz=8.0, seed=1012, min_dist=0.9, kT=1.0,
                    table: Optional[PairTable] = None) -> System:
    """N reactive particles in the plane z = 0 of a (L, L, Lz) box with vz = 0: the paper's 2d square
    box (Sec. 3.2: side 39.63 sigma, 1000 particles, kT/eps = 1) filled with point particles of the
    single-entry swap table (eps 1, sigma 1, n 10, r_cut 1.5, lambda 1).  Run it with an integrator of
    dim 2.  Lz only has to hold three list radii.  Uniform random sequential addition in the plane,
    rejecting distances <= min_dist."""
    rng = np.random.default_rng(seed)
    Lf = float(np.float32(L))
    Lzf = float(np.float32(Lz))
    acc = []
    while len(acc) < N:
        for c in wrap_fp32(rng.uniform(-0.5 * Lf, 0.5 * Lf, size=(4 * N, 3)), Lf)[:, :2].astype(np.float64):
            if len(acc) >= N:
                break
            if acc:
                d = c - np.asarray(acc)
                d -= Lf * np.round(d / Lf)
                if np.min(np.einsum("ij,ij->i", d, d)) <= min_dist * min_dist:
                    continue
            acc.append(c)
    pos = np.zeros((N, 3), np.float32)
    pos[:, :2] = np.asarray(acc, dtype=np.float32)
    types = np.zeros(N, np.int32)
    tab = table if table is not None else swap_table_single(lam=1.0)
    mass = np.ones(tab.ntypes)
    vel = maxwell_velocities(rng, types, mass, kT)
    vel[:, 2] = 0.0
    return System(pos=pos, types=types, L=(Lf, Lf, Lzf), table=tab, mass=mass, vel=vel,
                  name=f"planar reactive N={N} L={Lf}")


def patchy_table(eps_patch=10.0, sigma_patch=0.1, n=6, rcut_patch=0.2, lam=1.0) -> PairTable:
    """Sec. 3.2's swapping patchy mixture: type 0 = trifunctional disk, 1 = difunctional disk (WCA,
    eps 1, sigma 1, among all disks), 2 = patch (the swap potential among patches: eps 10 kT at kT 1,
    sigma 0.1 so that r_min ~ the paper's patch length 0.1, r_cut 0.2 = its bond distance, n 6 so that
    the bond vibration, ~440 per unit time, is resolved at dt 1e-3 like the paper's strongest Gaussian
    patches; lambda 1); disks and patches do not interact."""
    t = PairTable.empty(3)
    for a in (0, 1):
        for b in (0, 1):
            t.set(a, b, KIND_WCA, 1.0, 1.0, 6)
    t.set(2, 2, KIND_SWAP, eps_patch, sigma_patch, n, rcut_patch, lam)
    return t


def patchy_mixture(n_tri=400, n_di=600, L=39.63, Lz=8.0, seed=1014, kT=1.0, min_dist=0.95, radius=0.5,
                   patch_gap=0.15, table: Optional[PairTable] = None) -> System:
    """The 2d mixture of Sec. 3.2: n_tri trifunctional and n_di difunctional disks (sigma 1) with patches
    on the rim (radius 0.5; three at 120 degrees, two at 180) in a square box of side 39.63, kT 1.
    Tags 0 .. B-1 are the disk centres (type 0 / 1), then the patches (type 2), body by body.  Random
    sequential addition of the centres in the plane z = 0, uniform angles (redrawn for bodies with a
    patch closer than patch_gap to another body's patch), Maxwell velocities in the
    plane (vz = 0) and angular velocities of variance kT/I with I = radius^2 / 2 (unit-mass disks).
    meta["bodies"] holds centre [B], first [B+1], member [M], offset [M, 2] (body frame), inertia [B];
    meta["theta"], meta["omega"] the initial angles and angular velocities."""
    base = planar_reactive(N=n_tri + n_di, L=L, Lz=Lz, seed=seed, min_dist=min_dist, kT=kT)
    rng = np.random.default_rng(seed + 1)
    B = n_tri + n_di
    Lf = float(base.L[0])
    ctype = np.array([0] * n_tri + [1] * n_di, np.int32)
    rng.shuffle(ctype)
    npatch = np.where(ctype == 0, 3, 2)
    first = np.concatenate([[0], np.cumsum(npatch)]).astype(np.int32)
    M = int(first[-1])
    ang = np.concatenate([np.arange(k) * (2.0 * np.pi / k) for k in npatch])
    offset = np.stack([radius * np.cos(ang), radius * np.sin(ang)], axis=1).astype(np.float32)
    owner = np.repeat(np.arange(B), npatch)
    theta = rng.uniform(-np.pi, np.pi, B).astype(np.float32)
    inertia = np.full(B, 0.5 * radius * radius, np.float32)
    omega = (rng.standard_normal(B) * np.sqrt(kT / inertia)).astype(np.float32)
    cen = base.pos[:, :2].astype(np.float64)

    def rim(th_b):
        th = th_b.astype(np.float64)[owner]
        return np.stack([np.cos(th) * offset[:, 0] - np.sin(th) * offset[:, 1],
                         np.sin(th) * offset[:, 0] + np.cos(th) * offset[:, 1]], axis=1)

    # no two patches of different bodies start closer than patch_gap (the stiff swap term's core):
    # redraw the angles of the bodies involved
    from scipy.spatial import cKDTree
    for _ in range(200):
        p = cen[owner] + rim(theta)
        p = np.mod(p + 0.5 * Lf, Lf)
        pairs = cKDTree(np.minimum(p, np.nextafter(Lf, 0.0)), boxsize=Lf).query_pairs(patch_gap, output_type="ndarray")
        pairs = pairs[owner[pairs[:, 0]] != owner[pairs[:, 1]]] if len(pairs) else pairs
        if len(pairs) == 0:
            break
        bad = np.unique(owner[pairs[:, 0]])
        theta[bad] = rng.uniform(-np.pi, np.pi, len(bad)).astype(np.float32)
    else:
        raise RuntimeError("patchy_mixture: could not separate the patches")
    d = rim(theta)
    pos = np.zeros((B + M, 3), np.float32)
    pos[:B] = base.pos
    pos[B:, :2] = wrap_fp32(np.concatenate([base.pos[owner, :2].astype(np.float64) + d,
                                            np.zeros((M, 1))], axis=1), Lf)[:, :2]
    vel = np.zeros((B + M, 3), np.float32)
    vel[:B, :2] = base.vel[:, :2]
    vel[B:, 0] = vel[owner, 0] - omega[owner] * d[:, 1]
    vel[B:, 1] = vel[owner, 1] + omega[owner] * d[:, 0]
    types = np.concatenate([ctype, np.full(M, 2, np.int32)])
    bodies = dict(centre=np.arange(B, dtype=np.int32), first=first,
                  member=(B + np.arange(M)).astype(np.int32), offset=offset, inertia=inertia)
    tab = table if table is not None else patchy_table()
    return System(pos=pos, types=types, L=base.L, table=tab, mass=np.ones(tab.ntypes), vel=vel,
                  name=f"patchy mixture {n_tri}+{n_di} L={Lf}",
                  meta={"bodies": bodies, "theta": theta, "omega": omega})


def small_reactive(N=1000, density=0.2, seed=1001, min_dist=0.8, kT=0.1,
                   table: Optional[PairTable] = None) -> System:
    """N identical reactive particles (eps 1, sigma 1, n 10, r_cut 1.5, lambda 1)."""
    rng = np.random.default_rng(seed)
    L = fp32_box(N, density)
    tab = table if table is not None else swap_table_single()
    pos, types = rsa_positions(rng, L, [N], np.array([[min_dist]]))
    mass = np.ones(tab.ntypes)
    vel = maxwell_velocities(rng, types, mass, kT)
    return System(pos=pos, types=types, L=L, table=tab, mass=mass, vel=vel,
                  name=f"reactive N={N} rho={density}")


def unequal_lambda_mixture(N=6000, density=0.3, seed=61, kT=0.1, min_dist=0.85) -> System:
    """Three reactive types whose swap pairs each carry their own lambda, epsilon, sigma and cutoff, so a
    triplet's weight combines unequal entries; type 1 - type 1 is WCA.  Uniform random sequential
    addition."""
    tab = PairTable.empty(3)
    tab.set(0, 0, KIND_SWAP, 1.0, 1.0, 10, 1.5, 1.0)
    tab.set(0, 1, KIND_SWAP, 1.5, 0.9, 10, 1.4, 0.4)
    tab.set(0, 2, KIND_SWAP, 0.8, 1.1, 10, 1.6, 1.7)
    tab.set(1, 2, KIND_SWAP, 2.0, 1.0, 10, 1.5, 0.9)
    tab.set(1, 1, KIND_WCA, 1.0, 0.9, 6)
    rng = np.random.default_rng(seed)
    L = fp32_box(N, density)
    pos, types = rsa_positions(rng, L, [N // 3, N // 3, N - 2 * (N // 3)], np.full((3, 3), min_dist))
    mass = np.ones(3)
    vel = maxwell_velocities(rng, types, mass, kT)
    return System(pos=pos, types=types, L=L, table=tab, mass=mass, vel=vel,
                  name=f"unequal-lambda mixture N={N}")


def assembly_mixture(N=1048576, lam=1.0, density=0.3, seed=1003, kT=0.05,
                     frac_sites=0.5, min_frac=1.0) -> System:
    """Inert WCA colloids + reactive sites at total density ``density``.

    Non-overlapping start: every pair at least ``min_frac * sigma_ab`` apart
    (closer starts put site pairs deep in the repulsive core of the stiff
    eps 15, n 10 pair term, where dt 0.001 is unstable).
    """
    rng = np.random.default_rng(seed)
    L = fp32_box(N, density)
    tab = assembly_table(lam)
    n_sites = int(round(N * frac_sites))
    counts = [N - n_sites, n_sites]
    md = min_frac * tab.sigma
    pos, types = rsa_positions(rng, L, counts, md)
    # interleave the two species in memory order (the engine re-orders anyway)
    perm = rng.permutation(N)
    pos, types = pos[perm], types[perm]
    mass = np.ones(tab.ntypes)
    vel = maxwell_velocities(rng, types, mass, kT)
    return System(pos=pos, types=types, L=L, table=tab, mass=mass, vel=vel,
                  name=f"assembly N={N} lambda={lam}", meta={"lam": lam})


def dumbbell_table(rcut=1.3, n=100, lam=1.0) -> PairTable:
    """The bond-swap test mixture of the paper's Sec. 3.1: type 0 = A, type 1 = B.

    A-B swap term (eps 1, sigma 1, exponent n = 100, cutoff r_cut, lambda);
    A-A and B-B WCA (eps 1, sigma 1)."""
    t = PairTable.empty(2)
    t.set(0, 0, KIND_WCA, 1.0, 1.0, 6)
    t.set(1, 1, KIND_WCA, 1.0, 1.0, 6)
    t.set(0, 1, KIND_SWAP, 1.0, 1.0, n, rcut, lam)
    return t


def dumbbell_mixture(N=1000, rcut=1.3, density=0.125, seed=1006, kT=0.03, frac_b=0.4,
                     min_dist=1.05) -> System:
    """N particles, A:B = 3:2 at number density 0.125 (the paper's Sec. 3.1 and its performance
    figure, N = 2^9 ... 2^17): at kT 0.03 every B binds one A, and the A surplus is the reservoir the
    swaps draw on.  Uniform random sequential addition rejecting distances <= min_dist (1.05 sigma:
    beyond the minimum r_min = 2^(1/100) sigma of the n = 100 swap term, whose wall a closer start
    would hit with forces of order 10^7)."""
    rng = np.random.default_rng(seed)
    L = fp32_box(N, density)
    nb = int(round(frac_b * N))
    tab = dumbbell_table(rcut)
    pos, types = rsa_positions(rng, L, [N - nb, nb], np.full((2, 2), min_dist))
    mass = np.ones(2)
    vel = maxwell_velocities(rng, types, mass, kT)
    return System(pos=pos, types=types, L=L, table=tab, mass=mass, vel=vel,
                  name=f"dumbbell mixture N={N} r_cut={rcut}")


def replica_set(R=256, seed=1004, n_lo=500, n_hi=20000, kT=0.1) -> List[System]:
    """Independent replicas with N ~ logU[n_lo, n_hi], rho ~ U[0.2, 0.4],
    lambda ~ U[0, 1.5] and inert WCA fraction ~ U[0, 0.5].

    Type 0 = reactive (swap eps 1, sigma 1, n 10, r_cut 1.5), type 1 = inert
    WCA (sigma 1) against everything.
    """
    rng = np.random.default_rng(seed)
    out = []
    for r in range(R):
        N = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        rho = float(rng.uniform(0.2, 0.4))
        lam = float(rng.uniform(0.0, 1.5))
        finert = float(rng.uniform(0.0, 0.5))
        n_inert = int(round(N * finert))
        L = fp32_box(N, rho)
        tab = PairTable.empty(2)
        tab.set(0, 0, KIND_SWAP, 1.0, 1.0, 10, 1.5, lam)
        tab.set(0, 1, KIND_WCA, 1.0, 1.0, 6)
        tab.set(1, 1, KIND_WCA, 1.0, 1.0, 6)
        pos, types = rsa_positions(rng, L, [N - n_inert, n_inert], np.full((2, 2), 0.8))
        mass = np.ones(2)
        vel = maxwell_velocities(rng, types, mass, kT)
        out.append(System(pos=pos, types=types, L=L, table=tab, mass=mass, vel=vel,
                          name=f"replica {r}", meta={"lam": lam, "rho": rho, "finert": finert}))
    return out


def cluster(coords, L=20.0, types=None, table: Optional[PairTable] = None) -> System:
    """A hand-placed configuration (coordinates are rounded to FP32)."""
    c = np.asarray(coords, dtype=np.float64).reshape(-1, 3)
    Lf = float(np.float32(L))
    tab = table if table is not None else swap_table_single()
    ty = np.zeros(c.shape[0], np.int32) if types is None else np.asarray(types, np.int32)
    return System(pos=wrap_fp32(c, Lf), types=ty, L=Lf, table=tab,
                  mass=np.ones(tab.ntypes), vel=np.zeros((c.shape[0], 3), np.float32),
                  name="cluster")


def vitrimer_table(eps_site=20.0, sigma_site=0.3, n=10, rcut_site=0.45, lam=1.0) -> PairTable:
    """Types: 0 backbone bead, 1 reactive chain site, 2 crosslinker bead.

    WCA (eps = sigma = 1) between backbone beads and everything, and between
    crosslinker beads; the swap potential between reactive sites and between
    a site and a crosslinker bead (sites are small patch-like beads that
    overlap their partner when bonded)."""
    t = PairTable.empty(3)
    t.set(0, 0, KIND_WCA, 1.0, 1.0, 6)
    t.set(0, 1, KIND_WCA, 1.0, 1.0, 6)
    t.set(0, 2, KIND_WCA, 1.0, 1.0, 6)
    t.set(2, 2, KIND_WCA, 1.0, 1.0, 6)
    t.set(1, 1, KIND_SWAP, eps_site, sigma_site, n, rcut_site, lam)
    t.set(1, 2, KIND_SWAP, eps_site, sigma_site, n, rcut_site, lam)
    return t


def _grow_chains(rng, L, n_chains, chain_len, n_dimers, bond, d_min, tries=24, patience=8, max_rounds=5000):
    """Self-avoiding growth of chains and dimers in a periodic box: every
    bead keeps a periodic distance > d_min from all other beads, and
    consecutive beads of a molecule sit ``bond`` apart.

    All molecules grow together, one bead per molecule and round: each
    proposes ``tries`` random directions from its last bead and takes the
    first candidate clear of every bead placed so far (a periodic k-d tree
    query, library primitive); of two molecules whose new beads clash in the
    same round the later one tries again.  A molecule that finds no clear
    candidate ``patience`` rounds in a row is taken out and started anew."""
    sizes = np.array([chain_len] * n_chains + [2] * n_dimers)
    M = len(sizes)
    P = np.zeros((M, int(sizes.max()), 3))     # bead positions in [0, L)
    n = np.zeros(M, np.int64)                  # beads placed per molecule
    fails = np.zeros(M, np.int64)
    d2 = d_min * d_min
    tree, recent = None, np.zeros((0, 3))
    for _ in range(max_rounds):
        active = np.nonzero(n < sizes)[0]
        if active.size == 0:
            break
        # the tree holds the beads placed up to its build; later ones are checked directly while
        # few candidates remain (the last rounds of the growth), else the tree is rebuilt
        if tree is None or active.size * tries * len(recent) > 2e7:
            placed = P[np.arange(P.shape[1])[None, :] < n[:, None]]
            tree = cKDTree(placed, boxsize=L) if len(placed) else None
            recent = np.zeros((0, 3))
        # candidates: a random start for empty molecules, bond-length steps from the last bead otherwise
        dirs = rng.standard_normal((active.size, tries, 3))
        dirs /= np.linalg.norm(dirs, axis=2)[:, :, None]
        last = P[active, np.maximum(n[active] - 1, 0)]
        cand = last[:, None, :] + bond * dirs
        empty = n[active] == 0
        cand[empty] = rng.uniform(0.0, L, size=(int(empty.sum()), tries, 3))
        cand = np.mod(cand, L)
        cand = np.where(cand >= L, 0.0, cand)
        flat = cand.reshape(-1, 3)
        clear = np.ones(flat.shape[0], bool)
        if tree is not None:
            dist, _ = tree.query(flat, k=1, distance_upper_bound=d_min)
            clear = dist > d_min
        if len(recent):
            d = flat[:, None, :] - recent[None, :, :]
            d -= L * np.round(d / L)
            clear &= ~np.any(np.einsum("cka,cka->ck", d, d) <= d2, axis=1)
        clear = clear.reshape(active.size, tries)
        has = clear.any(axis=1)
        pick = np.argmax(clear, axis=1)
        chosen = cand[np.arange(active.size), pick]
        ok = has.copy()
        # clashes among this round's new beads: the later molecule yields
        idx = np.nonzero(ok)[0]
        if idx.size > 1:
            t2 = cKDTree(chosen[idx], boxsize=L)
            for a, b in sorted(t2.query_pairs(d_min), key=lambda p: max(p)):
                ia, ib = idx[a], idx[b]
                if ok[ia] and ok[ib]:
                    ok[max(ia, ib)] = False
        mq = active[ok]
        P[mq, n[mq]] = chosen[ok]
        recent = np.concatenate([recent, chosen[ok]])
        n[mq] += 1
        fails[mq] = 0
        stuck = active[~has]
        fails[stuck] += 1
        dead = stuck[fails[stuck] >= patience]
        n[dead] = 0
        fails[dead] = 0
        if dead.size:
            tree = None          # their beads leave the box: rebuild from what stays
    else:
        raise RuntimeError(f"chain growth did not finish in {max_rounds} rounds")
    pts = P[np.arange(P.shape[1])[None, :] < sizes[:, None]]
    starts = np.concatenate([[0], np.cumsum(sizes)[:-1]])
    mols = [(int(s), int(z)) for s, z in zip(starts, sizes)]
    return pts - 0.5 * L, mols


def vitrimer_network(n_chains=4000, chain_len=16, n_dimers=1600, density=0.85, site_frac=0.1, seed=1002,
                     kT=1.0, K=30.0, R0=1.5, bond=0.97, d_min=0.8, lam=1.0) -> System:
    """Bead-spring chains with reactive sites and free crosslinker dimers.

    ``n_chains`` chains of ``chain_len`` beads (FENE K, R0 along each chain),
    a seeded ``site_frac`` of the chain beads turned into reactive sites, and
    ``n_dimers`` two-bead crosslinkers (one FENE spring each) whose beads bind
    to sites; density counts every bead.  Grown self-avoiding with bond
    length ``bond`` and no two beads closer than ``d_min``."""
    rng = np.random.default_rng(seed)
    N = n_chains * chain_len + 2 * n_dimers
    L = fp32_box(N, density)
    pos, mols = _grow_chains(rng, L, n_chains, chain_len, n_dimers, bond, d_min)
    types = np.zeros(N, np.int32)
    chain_beads = n_chains * chain_len
    sites = rng.choice(chain_beads, int(round(site_frac * chain_beads)), replace=False)
    types[sites] = 1
    types[chain_beads:] = 2
    bonds = np.full((N, 2), -1, np.int32)
    for start, size in mols:
        for k in range(start, start + size - 1):
            bonds[k, 1] = k + 1
            bonds[k + 1, 0] = k
    mass = np.ones(3)
    vel = maxwell_velocities(rng, types, mass, kT)
    return System(pos=wrap_fp32(pos, L), types=types, L=L, table=vitrimer_table(lam=lam), mass=mass, vel=vel,
                  name=f"vitrimer network N={N}", bonds=bonds, fene=(K, R0),
                  meta={"n_chains": n_chains, "chain_len": chain_len, "n_dimers": n_dimers})
