"""A plain C program calls the library through include/amg.h (no Python in
the path): it must compile and link against the built library here, and on
a GPU it must solve the Poisson problem with both cycles, and once more as a
non-blocking (AMG_ASYNC) solve on a named device, with the level-0 aggregates
read back through amg_get_aggregates."""

import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "c_abi", "poisson_solve.c")
PKG = os.path.join(ROOT, "paper_2006_16147_amd")


def _build(out):
    lib = os.path.join(PKG, "libamg_hip.so")
    if not os.path.exists(lib):
        pytest.skip("libamg_hip.so is not built")
    cmd = ["gcc", "-std=c99", "-O2", "-D__HIP_PLATFORM_AMD__", "-I" + os.path.join(ROOT, "include"),
           "-I/opt/rocm/include", SRC, "-o", out, "-L" + PKG, "-lamg_hip", "-L/opt/rocm/lib",
           "-lamdhip64", "-lm", "-Wl,-rpath," + PKG, "-Wl,-rpath,/opt/rocm/lib"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return out


def test_c_program_compiles_and_links(tmp_path):
    exe = _build(str(tmp_path / "poisson_solve"))
    assert os.path.exists(exe)


@pytest.mark.gpu
def test_c_program_solves_on_gpu(tmp_path):
    exe = _build(str(tmp_path / "poisson_solve"))
    r = subprocess.run([exe, "24"], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    lines = [l for l in r.stdout.splitlines() if l.startswith("cycle=")]
    assert len(lines) == 3 and all("converged=1" in l for l in lines)
    assert all("aggregates=cubes" in l for l in lines)
    assert lines[2].startswith("cycle=V async")
