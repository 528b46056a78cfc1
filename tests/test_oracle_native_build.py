"""The oracle's timing build (-O3 -march=native, still without FP
contraction or fast-math) computes the same bits as the test build: the
hierarchies, cycles and solutions of a few problems hash identically under
both libraries (each loaded through ORACLE_LIB in a child process)."""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

_SCRIPT = r"""
import hashlib, sys
sys.path.insert(0, sys.argv[1])
import numpy as np
import oracle
from paper_2006_16147_amd import inputs
h = hashlib.sha256()
def add(*arrays):
    for a in arrays:
        h.update(np.ascontiguousarray(a).tobytes())
cases = [("poisson20", inputs.small_case(20, seed=0)["A"], {}),
         ("aniso16", inputs.diffusion7(16, *inputs.block_log_uniform_eps(16, 4, np.random.default_rng(2)), 1.0), {}),
         ("smoothed12", inputs.laplacian7(12), {"smooth": True})]
for name, A, kw in cases:
    ho = oracle.Hierarchy(A, **kw)
    assert ho.ok
    for l in range(ho.num_levels):
        c = ho.level_csr(l)
        add(c.row_ptr, c.col, c.val)
        if l < ho.num_levels - 1:
            add(*ho.transfer(l), ho.l1diag(l))
    b = np.random.default_rng(1).uniform(-1, 1, A.n)
    x, info = ho.pcg(b, rtol=1e-10, maxit=300)
    add(x, ho.vcycle(b))
    if not kw:
        add(ho.fcg(b, rtol=1e-10, maxit=300, cycle="K")[0])
print(h.hexdigest())
"""


def _digest(lib):
    env = dict(os.environ, ORACLE_LIB=lib)
    r = subprocess.run([sys.executable, "-c", _SCRIPT, ROOT], env=env, capture_output=True,
                       text=True, timeout=600)
    assert r.returncode == 0, r.stderr
    return r.stdout.strip()


@pytest.mark.slow
def test_native_timing_build_is_bit_identical():
    import oracle

    base = oracle.build_oracle(force=False)
    native = oracle.build_oracle(native=True)
    assert _digest(native) == _digest(base)
