"""Tolerances of the parity tests (GPU FP32 path vs FP64 oracle).

The target is a relative error of 1e-5.  Relative to what: the swap pair
force vanishes at r_min through cancellation of the (sigma/r)^(2n) and
(sigma/r)^n parts, so a plain |dF|/|F| is ill-posed there.  The scale of
each quantity is therefore the sum of the magnitudes of the sub-terms that
form it (computed by the oracle): per particle, A_F = sum over the terms
touching it of 4 eps n (2 q^2 + q) / r (times the three-body multipliers);
for the total energy A_E = sum of 4 eps (q^2 + q) (+ eps for WCA) and of
|Lambda u u|; for the virial A_W = sum of r times the force scale.  FP32
evaluation of q^2 = (sigma^2/r^2)^(2n) with n = 10 carries about 20 ulp
(~1.2e-6) of relative error, so 1e-5 of these scales is met with a margin.
The scales themselves are pinned on the CPU (tests/test_oracle_scales.py).

Forces must also meet the whole-system criterion ||dF||_2 / ||F||_2 <= 1e-5
(over all particles and components).  Energies report |dE|/|E| beside the
scaled error.
"""
import numpy as np

TOL = 1e-5


def force_errors(F_gpu, ref):
    """Per-particle max-component error divided by the oracle's force scale."""
    F = np.asarray(F_gpu, dtype=np.float64)[:, :3]
    d = np.abs(F - ref["F"]).max(axis=1)
    scale = ref["A_F"]
    out = np.where(scale > 0, d / np.where(scale > 0, scale, 1.0), np.where(d > 0, np.inf, 0.0))
    return out


def global_force_error(F_gpu, ref):
    """||F_gpu - F_ref||_2 / ||F_ref||_2 over every particle and component."""
    F = np.asarray(F_gpu, dtype=np.float64)[:, :3]
    den = float(np.linalg.norm(ref["F"]))
    num = float(np.linalg.norm(F - ref["F"]))
    return num / den if den > 0 else (0.0 if num == 0 else np.inf)


def assert_forces(F_gpu, ref, tol=TOL):
    e = force_errors(F_gpu, ref)
    worst = int(np.argmax(e))
    assert e.max() <= tol, f"force error {e.max():.3e} x A_F at particle {worst} (tol {tol})"
    g = global_force_error(F_gpu, ref)
    assert g <= tol, f"global force error ||dF||/||F|| = {g:.3e} (tol {tol})"
    return float(e.max())


def assert_energy(E_gpu, ref, tol=TOL):
    err = abs(float(E_gpu) - ref["E"]) / ref["A_E"] if ref["A_E"] > 0 else abs(float(E_gpu))
    rel = abs(float(E_gpu) - ref["E"]) / abs(ref["E"]) if ref["E"] != 0 else float("nan")
    print(f"parity: energy err {err:.3e} x A_E, |dE|/|E| = {rel:.3e}")
    assert err <= tol, f"energy {E_gpu} vs {ref['E']} (err {err:.3e} x A_E, |dE|/|E| {rel:.3e})"
    return err


def assert_virial(W_gpu, ref, tol=TOL):
    W = np.asarray(W_gpu, dtype=np.float64)
    err = np.abs(W - ref["W"]).max() / ref["A_W"] if ref["A_W"] > 0 else np.abs(W).max()
    assert err <= tol, f"virial {W} vs {ref['W']} (err {err:.3e} x A_W)"
    return err


def assert_pe(pe_gpu, ref, tol=TOL):
    d = np.abs(np.asarray(pe_gpu, dtype=np.float64) - ref["pe"])
    s = ref["A_pe"]
    e = np.where(s > 0, d / np.where(s > 0, s, 1.0), np.where(d > 0, np.inf, 0.0))
    assert e.max() <= tol, f"per-particle energy err {e.max():.3e}"
    return float(e.max())


def vjp_scale(A_F, adj, table):
    """Error scale of sum_m adj_m . dF_m/dtheta for theta = (eps, sigma, lambda) of each table entry.

    Every sub-term of a force is a product of powers (sigma/r)^k (k <= 2n) times eps (times lambda and
    the other factor for three-body terms), so the size of its derivative is at most 1/eps, 4 n/sigma
    or 1/lambda times its own size; summed with |adj_m| over the particles, Sum_m |adj_m| A_F[m] times
    that factor bounds the derivative's terms without the cancellation of random-sign adjoints."""
    base = float(np.sum(np.linalg.norm(np.asarray(adj, dtype=np.float64)[:, :3], axis=1) * A_F))
    nt = table.kind.shape[0]
    out = np.zeros((nt, nt, 3))
    for a in range(nt):
        for b in range(nt):
            if table.kind[a, b] == 0:
                continue
            n = 6 if table.kind[a, b] == 2 else int(table.n[a, b])
            out[a, b, 0] = base / table.epsilon[a, b]
            out[a, b, 1] = base * 4.0 * n / table.sigma[a, b]
            lam = table.lam[a, b]
            out[a, b, 2] = base / lam if lam > 0 else 0.0
    return out
