"""The C-ABI library loads and exports every function include/amg.h declares
(CPU only: no compute call is made)."""

import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "amg.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(amg_[a-z_0-9]+)\s*\(", text)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    from paper_2006_16147_amd import amg

    if not os.path.exists(amg.lib_path()):
        from paper_2006_16147_amd import build

        build.build()
    return ctypes.CDLL(amg.lib_path())


def test_header_declares_the_boundary():
    names = _declared()
    for required in ("amg_setup", "amg_pcg_solve", "amg_pcg_solve_batch", "amg_free",
                     "amg_vcycle_apply", "amg_params_default"):
        assert required in names


def test_every_declared_symbol_is_exported(lib):
    from paper_2006_16147_amd import amg

    names = _declared()
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(amg.EXPORTED_SYMBOLS) == names


def test_host_only_calls(lib):
    from paper_2006_16147_amd import amg

    p = amg.amg_params_default()
    assert (p.sweeps, p.max_coarse, p.pre, p.post, p.precision) == (3, 200, 1, 1, 0)
    assert (p.cycle, p.w_sweeps, p.coarse_solver) == (amg.CYCLE_V, 0, amg.COARSE_CHOLESKY)
    assert (p.coarse_rtol, p.coarse_maxit) == (1e-4, 30)  # Section 5's coarsest CG stop
    assert p.smooth_p == 0 and p.device == -1
    assert ctypes.sizeof(amg.Params) == 80  # the C struct, field for field
    assert amg.amg_status_string(amg.Status.ERR_STALL).startswith("coarsening")
    est = amg.amg_estimate_footprint(4096000, 28518400, p)
    assert 1e9 < est < 8e9
    # NULL handles are rejected without touching a device
    L = amg.load_library()
    n = ctypes.c_int32()
    assert L.amg_num_levels(None, ctypes.byref(n)) == amg.Status.ERR_ARG
    assert L.amg_wait(None) == amg.Status.ERR_ARG
    assert L.amg_query(None, ctypes.byref(n)) == amg.Status.ERR_ARG
    assert L.amg_get_aggregates(None, 0, None) == amg.Status.ERR_ARG
    L.amg_free(None)


def _c_layout(struct, fields, tmp_path):
    """sizeof and offsetof of a struct of amg.h, as the C compiler lays it out."""
    src = tmp_path / "layout.c"
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "amg.h"', "int main(void) {",
             '  printf("%%zu\\n", sizeof(%s));' % struct]
    lines += ['  printf("%%zu\\n", offsetof(%s, %s));' % (struct, f) for f in fields]
    lines += ["  return 0;", "}"]
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)],
                   check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()
    return int(out[0]), [int(v) for v in out[1:]]


@pytest.mark.parametrize("struct, cls", [("amg_params", "Params"),
                                         ("amg_solve_info", "SolveInfo"),
                                         ("amg_csr", "Csr")])
def test_binding_structs_match_the_header(struct, cls, tmp_path):
    """The ctypes structures of the binding have the C layout, field by field."""
    from paper_2006_16147_amd import amg

    C = getattr(amg, cls)
    fields = [f[0] for f in C._fields_]
    size, offsets = _c_layout(struct, fields, tmp_path)
    assert ctypes.sizeof(C) == size
    assert [getattr(C, f).offset for f in fields] == offsets
