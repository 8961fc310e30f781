"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer, on the CPU.

* The C brute-force oracle (oracle/brute.c) built with ASan + UBSan (gcc),
  driven by a small C program over a two-type swap/WCA system: full
  evaluation and the sampled-particle evaluation, two OpenMP threads.
* The engine's host code: every csrc source compiled with the sanitizers on
  the host pass only (-Xarch_host; device code is built as usual), linked into
  a C++ driver that runs the host logic no device is needed for: the
  coefficient-table compiler behind rc_create (valid and invalid tables), the
  batch layout behind rc_batch_create (uneven replicas), the box and cell-grid
  set-up and the workspace layouts.  Without a GPU the creators stop with
  RC_ERR_HIP at their first device call, after that host work.

Any sanitizer report aborts the driver (-fno-sanitize-recover), so each test
asserts a clean exit and the driver's own checks."""
import concurrent.futures as cf
import glob
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1912_08569_amd", "csrc")
ROCM = "/opt/rocm"

_BRUTE_MAIN = r"""
#include <stdio.h>
#include <stdlib.h>
int orc_evaluate(int N, const double* pos, const int* type, const double* L, int nt, const int* kind,
                 const double* eps, const double* sigma, const int* n, const double* rcut, const double* lam,
                 int nthreads, double* F, double* pe, double* out, long long* bonds, long long* ntrip);
int orc_forces_subset(int N, const double* pos, const int* type, const double* L, int nt, const int* kind,
                      const double* eps, const double* sigma, const int* n, const double* rcut, const double* lam,
                      int nthreads, int M, const int* idx, double* F, double* pe, int* degree);
int main(void) {
    enum { N = 400 };
    const double L[3] = {7.0, 7.0, 7.0};
    static double pos[3 * N], F[3 * N], pe[N], Fs[3 * 20], pes[20];
    static int type[N], idx[20], deg[20];
    unsigned s = 12345u;
    for (int i = 0; i < 3 * N; ++i) { s = s * 1664525u + 1013904223u; pos[i] = (s / 4294967296.0 - 0.5) * 7.0; }
    for (int i = 0; i < N; ++i) type[i] = i % 3 == 0;
    const int kind[4] = {1, 2, 2, 2}, n[4] = {10, 6, 6, 6};
    const double eps[4] = {1, 1, 1, 1}, sigma[4] = {1, 0.8, 0.8, 1}, rcut[4] = {1.5, 0.898, 0.898, 1.1225},
                 lam[4] = {1.0, 0, 0, 0};
    double out[9];
    long long bonds = 0, ntrip = 0;
    if (orc_evaluate(N, pos, type, L, 2, kind, eps, sigma, n, rcut, lam, 2, F, pe, out, &bonds, &ntrip)) return 2;
    for (int m = 0; m < 20; ++m) idx[m] = (37 * m) % N;
    if (orc_forces_subset(N, pos, type, L, 2, kind, eps, sigma, n, rcut, lam, 2, 20, idx, Fs, pes, deg)) return 3;
    double worst = 0.0;
    for (int m = 0; m < 20; ++m)
        for (int a = 0; a < 3; ++a) {
            double d = Fs[3 * m + a] - F[3 * idx[m] + a];
            if (d < 0) d = -d;
            double sc = 1.0 + (F[3 * idx[m] + a] < 0 ? -F[3 * idx[m] + a] : F[3 * idx[m] + a]);
            if (d / sc > worst) worst = d / sc;
        }
    printf("E %.10g bonds %lld triplets %lld subset-vs-full %.3g\n", out[0], bonds, ntrip, worst);
    return worst < 1e-9 ? 0 : 4;
}
"""

_HOST_MAIN = r"""
#include <cstdio>
#include <cstring>
#include <vector>
#include "rc_host.h"
using namespace rc;
using namespace rc::host;
static int fails = 0;
#define CHECK(x) do { if (!(x)) { std::printf("check failed: %s\n", #x); ++fails; } } while (0)
static rc_pair_coeff P(int kind, double e, double s, int n, double rc, double lam) {
    rc_pair_coeff p; std::memset(&p, 0, sizeof p);
    p.kind = kind; p.epsilon = e; p.sigma = s; p.n = n; p.r_cut = rc; p.lambda = lam; return p;
}
int main() {
    // a valid two-type table: swap, WCA cross, WCA
    std::vector<rc_pair_coeff> t = {P(RC_KIND_SWAP, 15, 0.3, 10, 0.45, 1.0), P(RC_KIND_WCA, 1, 0.65, 6, 0.7296, 0),
                                    P(RC_KIND_WCA, 1, 0.65, 6, 0.7296, 0), P(RC_KIND_WCA, 1, 1, 6, 1.1225, 0)};
    std::vector<DevEntry> ent(4);
    double rl = 0;
    std::string why;
    CHECK(compile_table(2, t.data(), 0.3, ent.data(), &rl, &why) == RC_OK);
    CHECK(rl > 1.42 && rl < 1.43);
    // invalid tables: asymmetric, r_cut inside r_min, negative lambda, unknown kind
    std::vector<rc_pair_coeff> bad = t;
    bad[1].sigma = 0.7;
    CHECK(compile_table(2, bad.data(), 0.3, ent.data(), &rl, &why) == RC_ERR_ARG && !why.empty());
    bad = t; bad[0].r_cut = 0.3;
    CHECK(compile_table(2, bad.data(), 0.3, ent.data(), &rl, &why) == RC_ERR_ARG);
    bad = t; bad[0].lambda = -1;
    CHECK(compile_table(2, bad.data(), 0.3, ent.data(), &rl, &why) == RC_ERR_ARG);
    bad = t; bad[3].kind = 9;
    CHECK(compile_table(2, bad.data(), 0.3, ent.data(), &rl, &why) == RC_ERR_ARG);
    rc_ctx* c = nullptr;
    CHECK(rc_create(&c, 2, bad.data(), 0.3) == RC_ERR_ARG && c == nullptr);
    CHECK(rc_create(&c, 2, t.data(), -1.0) == RC_ERR_ARG);
    const int cr = rc_create(&c, 2, t.data(), 0.3);   // no device here: stops at the first device call
    CHECK(cr == RC_ERR_HIP || cr == RC_OK);
    if (c) rc_destroy(c);
    // box, grid and layouts
    rc_ctx tmp;
    Box b;
    rc_box bx; bx.L[0] = 151.7607879638672; bx.L[1] = bx.L[0]; bx.L[2] = bx.L[0];
    CHECK(make_box(&tmp, bx, b) == RC_OK);
    Grid g;
    CHECK(make_grid(&tmp, rl, b, g) == RC_OK && g.nc[0] == 106 && g.nkeys == (1u << 21));
    rc_box small; small.L[0] = small.L[1] = small.L[2] = 3.0;
    CHECK(make_grid(&tmp, rl, (make_box(&tmp, small, b), b), g) == RC_ERR_ARG);
    rc_box nonfp32; nonfp32.L[0] = nonfp32.L[1] = nonfp32.L[2] = 0.1;
    CHECK(make_box(&tmp, nonfp32, b) == RC_ERR_ARG);
    const CellsLayout l = cells_layout(1048576, 1u << 21);
    CHECK(l.total > 16u * 1048576u * 3u && (l.tpos & 255) == 0);
    const WsLayout w = ws_layout(plist_entries(1000, 32), 1000, 64000);
    CHECK(plist_entries(1000, 32) == 1024u * 32u && (w.hsum & 255) == 0 && w.total >= w.hsum + 16u * 64000u);
    // a batch of uneven replicas: table compiler, boxes, grids and the slot and key layout on the host
    const int R = 7;
    std::vector<rc_pair_coeff> tabs;
    std::vector<int> counts;
    std::vector<rc_box> boxes;
    for (int r = 0; r < R; ++r) {
        for (const rc_pair_coeff& p : t) tabs.push_back(p);
        counts.push_back(40 + 300 * r);
        rc_box q; q.L[0] = q.L[1] = q.L[2] = 8.0 + r; boxes.push_back(q);
    }
    rc_batch* bb = nullptr;
    const int br = rc_batch_create(&bb, R, 2, tabs.data(), counts.data(), boxes.data(), 0.3);
    CHECK(br == RC_ERR_HIP || br == RC_OK);
    if (bb) rc_batch_destroy(bb);
    counts[3] = 0;
    CHECK(rc_batch_create(&bb, R, 2, tabs.data(), counts.data(), boxes.data(), 0.3) == RC_ERR_ARG);
    std::printf("host checks: %d failed\n", fails);
    return fails ? 1 : 0;
}
"""


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd[:3])} ...:\n{r.stdout[-3000:]}\n{r.stderr[-3000:]}"
    return r


def test_brute_oracle_clean_under_asan_ubsan(tmp_path):
    if not shutil.which("gcc"):
        pytest.skip("gcc not available")
    main = tmp_path / "main.c"
    main.write_text(_BRUTE_MAIN)
    exe = tmp_path / "brute_san"
    _run(["gcc", "-g", "-O1", "-fopenmp", "-ffp-contract=off", "-fsanitize=address,undefined",
          "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-o", str(exe), str(main),
          os.path.join(ROOT, "oracle", "brute.c"), "-lm"])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", OMP_NUM_THREADS="2")
    r = _run([str(exe)], env=env, timeout=300)
    assert "ERROR" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-3000:]
    assert r.stdout.startswith("E "), r.stdout


@pytest.mark.slow
def test_engine_host_code_clean_under_asan_ubsan(tmp_path):
    hipcc = os.path.join(ROCM, "bin", "hipcc")
    clang = os.path.join(ROCM, "lib", "llvm", "bin", "clang++")
    if not (os.path.exists(hipcc) and os.path.exists(clang)):
        pytest.skip("ROCm toolchain not available")
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
    flags = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-munsafe-fp-atomics",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-w", *san]
    main = tmp_path / "host_main.hip"
    main.write_text(_HOST_MAIN)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip"))) + [str(main)]

    def comp(src):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        _run([hipcc, *flags, "-I", CSRC, "-c", src, "-o", obj])
        return obj

    with cf.ThreadPoolExecutor(max_workers=8) as ex:
        objs = list(ex.map(comp, srcs))
    exe = str(tmp_path / "host_san")
    _run([clang, "-fsanitize=address,undefined", "-o", exe, *objs, f"-L{ROCM}/lib", "-lamdhip64",
          f"-Wl,-rpath,{ROCM}/lib"])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0", HIP_VISIBLE_DEVICES="")
    r = _run([exe], env=env, timeout=300)
    assert "host checks: 0 failed" in r.stdout, r.stdout + r.stderr[-3000:]
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-3000:]
