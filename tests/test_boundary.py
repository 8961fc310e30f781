"""The C-ABI library loads, exports every declared entry point, and the
Python binding's constants and struct layouts match include/rc.h.  No GPU."""
import ctypes
import os
import re
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rc.h")


@pytest.fixture(scope="module")
def lib():
    from paper_1912_08569_amd import _lib
    return _lib


def test_library_exports_every_declared_symbol(lib):
    names = lib.declared_symbols()
    assert len(names) >= 18
    cdll = ctypes.CDLL(lib.LIB_PATH)
    missing = [n for n in names if not hasattr(cdll, n)]
    assert not missing, f"not exported: {missing}"
    for n in ("rc_build_cells", "rc_build_nlist", "rc_compute_forces", "rc_integrate_step",
              "rc_bond_count", "rc_md_run", "rc_force_hvp", "rc_param_grad"):
        assert n in names


def test_version_call_needs_no_gpu(lib):
    assert lib.load().rc_version() >= 10000


def test_constants_match_header(lib):
    with open(HEADER) as f:
        text = f.read()
    defines = dict(re.findall(r"#define\s+(RC_\w+)\s+\(?(-?\d+)", text))
    checked = 0
    for name, val in defines.items():
        if hasattr(lib, name):
            assert getattr(lib, name) == int(val), name
            checked += 1
    assert checked >= 25


def test_struct_layouts_match_c(lib):
    src = r'''
#include <stdio.h>
#include <stddef.h>
#include "rc.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu\n", sizeof(rc_pair_coeff), sizeof(rc_box), sizeof(rc_integrator),
         sizeof(rc_md_buffers), sizeof(rc_md_options), sizeof(rc_md_stats));
  printf("%zu %zu %zu %zu\n", offsetof(rc_integrator, seed), offsetof(rc_integrator, mass),
         offsetof(rc_md_buffers, cells_ws_bytes), offsetof(rc_md_buffers, bonds_log));
  return 0;
}
'''
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "layout.c")
        exe = os.path.join(d, "layout")
        with open(c, "w") as f:
            f.write(src)
        subprocess.check_call(["gcc", "-I", os.path.dirname(HEADER), "-o", exe, c])
        out = subprocess.check_output([exe]).decode().split()
    sizes = [int(x) for x in out]
    L = lib
    assert sizes[:6] == [ctypes.sizeof(L.PairCoeff), ctypes.sizeof(L.Box), ctypes.sizeof(L.Integrator),
                         ctypes.sizeof(L.MdBuffers), ctypes.sizeof(L.MdOptions), ctypes.sizeof(L.MdStats)]
    assert sizes[6] == L.Integrator.seed.offset and sizes[7] == L.Integrator.mass.offset
    assert sizes[8] == L.MdBuffers.cells_ws_bytes.offset and sizes[9] == L.MdBuffers.bonds_log.offset


def test_binding_marshals_only():
    # the binding modules hold no arithmetic kernels: no numpy/torch math on particle data
    import inspect

    from paper_1912_08569_amd import api, engine
    for mod in (api, engine):
        src = inspect.getsource(mod)
        for bad in ("np.sqrt", "torch.sqrt", "np.power", "torch.pow", "np.exp", "oracle"):
            assert bad not in src, (mod.__name__, bad)


def test_oracle_is_not_imported_by_the_package():
    import subprocess
    import sys
    code = "import sys, paper_1912_08569_amd; print(any(m.startswith('oracle') for m in sys.modules))"
    out = subprocess.check_output([sys.executable, "-c", code], cwd=ROOT).decode().strip()
    assert out == "False"


_ONE_RUNTIME = r"""
import sys
sys.path.insert(0, {root!r})
import numpy
import workloads as W
W.patchy_mixture(n_tri=40, n_di=60, L=12.0)    # host-side set-up (scipy k-d trees) before the engine
import paper_1912_08569_amd  # noqa: F401      (torch not imported before)
hip = sorted(set(l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l))
hsa = sorted(set(l.split()[-1] for l in open('/proc/self/maps') if 'libhsa-runtime64' in l))
print(len(hip), len(hsa), hip, hsa)
"""


def test_one_hip_runtime_whatever_the_import_order():
    # librc.so binds to the HIP runtime torch brings (the one that owns the tensors it is given): a process
    # that sets up a workload and then imports the package, with torch never imported before, maps one
    # HIP and one HSA runtime, not the system ROCm's beside torch's
    out = subprocess.run(["python", "-c", _ONE_RUNTIME.format(root=ROOT)], capture_output=True, text=True,
                         timeout=300)
    assert out.returncode == 0, out.stderr[-2000:]
    n_hip, n_hsa = (int(x) for x in out.stdout.split()[:2])
    assert n_hip == 1 and n_hsa == 1, out.stdout
