"""GPU test of amg_pcg_solve_noalloc, the solve entry point that allocates
nothing (its scratch is the library's static device array): through the C
ABI it must give the same results, bit for bit, as amg_pcg_solve on the same
hierarchy, on two calls in a row whose second has a smaller problem, and on
a K-cycle hierarchy (whose per-level scalars also live in that array),
without changing the device's free memory or the hierarchies' footprints."""

import ctypes

import numpy as np
import pytest

from paper_2006_16147_amd import inputs

from gpu_helpers import setup, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def _raw_solve(fn, h, b, x, rtol, maxit):
    from paper_2006_16147_amd import amg

    info = amg.SolveInfo()
    st = fn(h.handle, b.data_ptr(), x.data_ptr(), rtol, maxit, ctypes.byref(info))
    return st, info.as_dict()


def _free_bytes():
    import torch

    torch.cuda.synchronize()
    return torch.cuda.mem_get_info()[0]


@pytest.mark.parametrize("cycle", ["V", "K"])
def test_noalloc_solve_equals_solve_on_two_calls(cycle):
    import torch

    from paper_2006_16147_amd import amg

    L = amg.load_library()
    cyc = amg.CYCLE_V if cycle == "V" else amg.CYCLE_K
    cases = []
    for N, seed in ((40, 1), (20, 2)):  # the second call has the smaller input
        A = inputs.laplacian7(N)
        b = to_dev(np.random.default_rng(seed).uniform(-1, 1, A.n))
        cases.append((setup(A, cycle=cyc), b))
    feet = [h.footprint_bytes() for h, _ in cases]
    xs = [torch.zeros_like(b) for _, b in cases]  # every torch allocation made up front
    free0 = _free_bytes()
    got = []
    for (h, b), x in zip(cases, xs):
        st, info = _raw_solve(L.amg_pcg_solve_noalloc, h, b, x, 1e-10, 500)
        assert st == amg.Status.OK and info["converged"], info
        got.append((x, info))
    assert _free_bytes() == free0
    assert [h.footprint_bytes() for h, _ in cases] == feet
    for (h, b), (xn, infon) in zip(cases, got):
        x = torch.zeros_like(b)
        st, info = _raw_solve(L.amg_pcg_solve, h, b, x, 1e-10, 500)
        assert st == amg.Status.OK
        assert info["iterations"] == infon["iterations"]
        assert info["rel_res_recursive"] == infon["rel_res_recursive"]
        assert torch.equal(x, xn)


def test_noalloc_status_and_rejections():
    import torch

    from paper_2006_16147_amd import amg

    A = inputs.laplacian7(16)
    h = setup(A)
    b = to_dev(np.random.default_rng(3).uniform(-1, 1, A.n))
    x = torch.zeros_like(b)
    st, info = amg.amg_pcg_solve_noalloc(h, b, x, rtol=1e-14, maxit=3, raise_on_error=False)
    assert st == amg.Status.NOT_CONVERGED and info["iterations"] == 3
    x2 = torch.zeros_like(b)
    st2, info2 = amg.amg_pcg_solve(h, b, x2, rtol=1e-14, maxit=3, raise_on_error=False)
    assert st2 == st and torch.equal(x, x2)
    L = amg.load_library()
    hb = torch.zeros(A.n, dtype=torch.float64).pin_memory()
    assert L.amg_pcg_solve_noalloc(h.handle, hb.data_ptr(), x.data_ptr(), 1e-8, 10,
                                   None) == amg.Status.ERR_ARG
