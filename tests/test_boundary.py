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
