"""GPU tests of the C ABI's calling conventions (include/amg.h): the
non-blocking solve (AMG_ASYNC with amg_wait / amg_query), the hierarchy's
device (amg_params.device), amg_get_aggregates, the argument checks that
reject mismatched caller arrays before any launch, and the batch solve's
recovery from a failed allocation."""

import ctypes
import os
import subprocess
import sys

import numpy as np
import pytest

from paper_2006_16147_amd import inputs

from gpu_helpers import setup, to_dev

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def test_async_solve_equals_blocking_solve():
    import torch

    from paper_2006_16147_amd import amg

    case = inputs.small_case(24, seed=0)
    A, b = case["A"], case["b"]
    hb = setup(A)
    ha = setup(A, flags=amg.FLAG_ASYNC, device=0)
    assert ha.is_async and ha.device == 0
    bd = to_dev(b)
    xb, xa = torch.zeros_like(bd), torch.zeros_like(bd)
    st, info_b = amg.amg_pcg_solve(hb, bd, xb, rtol=1e-8, maxit=200)
    assert st == amg.Status.OK and info_b["converged"]
    st, none = amg.amg_pcg_solve(ha, bd, xa, rtol=1e-8, maxit=200)
    assert st == amg.Status.OK and none is None
    st, info_a = amg.amg_wait(ha)
    assert st == amg.Status.OK and amg.amg_query(ha)
    assert info_a["iterations"] == info_b["iterations"]
    assert info_a["rel_res_recursive"] == info_b["rel_res_recursive"]
    assert torch.equal(xa, xb)
    # nothing in flight: amg_wait returns at once
    assert amg.amg_wait(ha) == (amg.Status.OK, None)


def test_async_batch_and_calls_that_wait_for_the_solve_in_flight():
    import torch

    from paper_2006_16147_amd import amg

    A = inputs.laplacian7(20)
    B = np.random.default_rng(3).uniform(-1, 1, (A.n, 6))
    hb = setup(A, precision=amg.FP32)
    ha = setup(A, precision=amg.FP32, flags=amg.FLAG_ASYNC)
    Bd = to_dev(B)
    Xb, Xa = torch.zeros_like(Bd), torch.zeros_like(Bd)
    st, infos_b = amg.amg_pcg_solve_batch(hb, Bd, Xb)
    assert st == amg.Status.OK
    assert amg.amg_pcg_solve_batch(ha, Bd, Xa) == (amg.Status.OK, None)
    # an introspection call orders itself after the solve in flight
    rp, ci, val = ha.level_csr(1)
    assert rp[-1] == len(ci) == len(val)
    st, infos_a = amg.amg_wait(ha)
    assert st == amg.Status.OK
    # each hierarchy autotunes its tiles on its first block solve; the tiles
    # fix the order of the per-column dot-product sums, so the two results
    # are bitwise equal when both chose the same tiles, else equal to rounding
    if ha.batch_tiles() == hb.batch_tiles():
        assert [i["iterations"] for i in infos_a] == [i["iterations"] for i in infos_b]
        assert torch.equal(Xa, Xb)
    else:
        assert all(abs(a["iterations"] - b["iterations"]) <= 1 for a, b in zip(infos_a, infos_b))
        assert torch.allclose(Xa, Xb, rtol=0, atol=1e-9 * Xb.abs().max().item())
    Xa1 = Xa.clone()
    # a second solve on the same hierarchy after the first was waited for
    Xa.zero_()
    assert amg.amg_pcg_solve_batch(ha, Bd, Xa)[0] == amg.Status.OK
    ha.close()  # amg_free waits for the solve in flight
    assert torch.equal(Xa, Xa1)


def test_async_not_converged_status_comes_from_wait():
    import torch

    from paper_2006_16147_amd import amg

    case = inputs.small_case(16, seed=0)
    ha = setup(case["A"], flags=amg.FLAG_ASYNC)
    bd = to_dev(case["b"])
    x = torch.zeros_like(bd)
    assert amg.amg_pcg_solve(ha, bd, x, rtol=1e-14, maxit=3)[0] == amg.Status.OK
    st, info = amg.amg_wait(ha, raise_on_error=False)
    assert st == amg.Status.NOT_CONVERGED and info["iterations"] == 3


def test_get_aggregates_is_the_transfer_map(orc):
    A = inputs.laplacian7(12)
    h = setup(A)
    ho = orc.Hierarchy(A)
    for l in range(ho.num_levels - 1):
        np.testing.assert_array_equal(h.aggregates(l), h.transfer(l)[0])
        np.testing.assert_array_equal(h.aggregates(l), ho.transfer(l)[0])


def test_device_parameter_out_of_range_is_rejected():
    import torch

    from paper_2006_16147_amd import amg

    A = inputs.laplacian7(8)
    rp, ci, va = to_dev(A.row_ptr), to_dev(A.col), to_dev(A.val)
    with pytest.raises(amg.AmgError) as e:
        amg.amg_setup(rp, ci, va, device=torch.cuda.device_count())
    assert e.value.status == amg.Status.ERR_ARG
    with pytest.raises(amg.AmgError) as e:
        amg.amg_setup(rp, ci, va, flags=64)  # no such flag
    assert e.value.status == amg.Status.ERR_ARG


def test_mismatched_caller_arrays_are_rejected_before_any_launch():
    import torch

    from paper_2006_16147_amd import amg

    A = inputs.laplacian7(10)
    h = setup(A)
    n = A.n
    good = torch.zeros(n, dtype=torch.float64, device="cuda:0")
    with pytest.raises(ValueError):
        amg.amg_pcg_solve(h, torch.zeros(n - 1, dtype=torch.float64, device="cuda:0"), good)
    with pytest.raises(ValueError):
        amg.amg_pcg_solve(h, good, torch.zeros(n + 1, dtype=torch.float64, device="cuda:0"))
    with pytest.raises(ValueError):
        amg.amg_vcycle_apply(h, good, torch.zeros((n, 1), dtype=torch.float64, device="cuda:0"))
    B = torch.zeros((n, 3), dtype=torch.float64, device="cuda:0")
    with pytest.raises(ValueError):
        amg.amg_pcg_solve_batch(h, good, B)  # B must be 2-D
    with pytest.raises(ValueError):
        amg.amg_pcg_solve_batch(h, B, torch.zeros((n, 2), dtype=torch.float64, device="cuda:0"))
    with pytest.raises(ValueError):
        amg.amg_pcg_solve_batch(h, torch.zeros((n - 1, 3), dtype=torch.float64, device="cuda:0"),
                                torch.zeros((n - 1, 3), dtype=torch.float64, device="cuda:0"))
    # host memory through the raw ABI: the library rejects it itself
    L = amg.load_library()
    hb = torch.zeros(n, dtype=torch.float64).pin_memory()
    st = L.amg_pcg_solve(h.handle, hb.data_ptr(), good.data_ptr(), 1e-8, 10, None)
    assert st == amg.Status.ERR_ARG
    # the hierarchy still solves afterwards
    b = to_dev(np.ones(n))
    x = torch.zeros_like(b)
    assert amg.amg_pcg_solve(h, b, x)[0] == amg.Status.OK


def _hip():
    lib = ctypes.CDLL("libamdhip64.so")
    lib.hipMalloc.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_size_t]
    lib.hipFree.argtypes = [ctypes.c_void_p]
    lib.hipMemGetAddressRange.argtypes = [ctypes.POINTER(ctypes.c_void_p),
                                          ctypes.POINTER(ctypes.c_size_t), ctypes.c_void_p]
    return lib


def test_too_short_device_array_is_rejected_through_the_raw_abi():
    """A device array shorter than the solve's extent is refused by the
    library (the allocation's range reported by the runtime) before any
    kernel runs. Checked only where the runtime reports that range exactly,
    which is what the library relies on."""
    import torch

    from paper_2006_16147_amd import amg

    A = inputs.laplacian7(16)
    h = setup(A)
    n = A.n
    hip = _hip()
    short = ctypes.c_void_p()
    nbytes = 8 * (n // 2)
    assert hip.hipMalloc(ctypes.byref(short), nbytes) == 0
    try:
        base, size = ctypes.c_void_p(), ctypes.c_size_t()
        assert hip.hipMemGetAddressRange(ctypes.byref(base), ctypes.byref(size),
                                         ctypes.c_void_p(short.value + 8)) == 0
        if base.value != short.value or size.value >= 8 * n:
            pytest.skip("the runtime does not report this allocation's range exactly")
        good = torch.zeros(n, dtype=torch.float64, device="cuda:0")
        L = amg.load_library()
        assert L.amg_pcg_solve(h.handle, short.value, good.data_ptr(), 1e-8, 10,
                               None) == amg.Status.ERR_ARG
        assert L.amg_vcycle_apply(h.handle, good.data_ptr(), short.value) == amg.Status.ERR_ARG
    finally:
        torch.cuda.synchronize()
        hip.hipFree(short)


_OOM_SCRIPT = r"""
import sys
sys.path.insert(0, sys.argv[1])
sys.path.insert(0, sys.argv[1] + "/tests")
import numpy as np, torch
from paper_2006_16147_amd import amg, inputs
from gpu_helpers import setup, to_dev
torch.cuda.set_device(0)
A = inputs.laplacian7(32)
k = 512  # block buffers ~1.2 GB, far above what setup left in the library's pool
h = setup(A, precision=amg.FP32)
B = to_dev(np.random.default_rng(5).uniform(-1, 1, (A.n, k)))
X = torch.zeros_like(B)
torch.cuda.synchronize()
free, _ = torch.cuda.mem_get_info()
# leave 32 MiB: the block solve of 32^3 x 512 needs about 1.2 GB more
filler = torch.empty(free - (32 << 20), dtype=torch.uint8, device="cuda:0")
print("filled", filler.numel() >> 20, "MiB", flush=True)
st1, _ = amg.amg_pcg_solve_batch(h, B, X, raise_on_error=False)
st2, _ = amg.amg_pcg_solve_batch(h, B, X, raise_on_error=False)
print("under pressure", st1, st2, h.footprint_bytes(), flush=True)
del filler
torch.cuda.empty_cache()
st3, infos = amg.amg_pcg_solve_batch(h, B, X, raise_on_error=False)
ok = all(i["converged"] and i["rel_res_true"] <= 1.001e-8 for i in infos)
print("after release", st3, ok, flush=True)
"""


def test_batch_allocation_failure_leaves_no_half_built_state():
    """Fills the device (in a fresh process, whose library pool holds no
    reserve), so that the block solve's buffers cannot be allocated: both
    calls return AMG_ERR_OOM (the second allocates again instead of using a
    partial batch), and once memory is released the same call succeeds."""
    r = subprocess.run([sys.executable, "-c", _OOM_SCRIPT, ROOT], capture_output=True,
                       text=True, timeout=180)
    assert r.returncode == 0, r.stdout + r.stderr
    lines = r.stdout.splitlines()
    pressure = [l for l in lines if l.startswith("under pressure")][0].split()
    assert pressure[2:4] == ["5", "5"], r.stdout  # AMG_ERR_OOM twice
    assert [l for l in lines if l.startswith("after release")][0].split()[2:] == ["0", "True"]
