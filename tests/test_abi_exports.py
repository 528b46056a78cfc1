"""The C-ABI library loads and exports every function include/amg.h declares
(CPU only: no compute call is made)."""

import ctypes
import os
import re

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
    assert p.smooth_p == 0
    assert ctypes.sizeof(amg.Params) == 80  # the C struct, field for field
    assert amg.amg_status_string(amg.Status.ERR_STALL).startswith("coarsening")
    est = amg.amg_estimate_footprint(4096000, 28518400, p)
    assert 1e9 < est < 8e9
    # NULL handles are rejected without touching a device
    L = amg.load_library()
    n = ctypes.c_int32()
    assert L.amg_num_levels(None, ctypes.byref(n)) == amg.Status.ERR_ARG
    L.amg_free(None)
