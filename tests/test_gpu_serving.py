"""Serving on the GPU: concurrent slots, cached hierarchies, and each
request's result identical alone and in the mix."""

import numpy as np
import pytest

from paper_2006_16147_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def backend():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2006_16147_amd.serve import GpuBackend

    return GpuBackend(keep_x=True)


def test_gpu_serving_alone_vs_mix(backend):
    from paper_2006_16147_amd.serve import Request, Server, requests_from_stream, summarize

    stream = inputs.serving_requests(24, rate=300.0, seed=4, sizes=(16, 24, 32))
    reqs = requests_from_stream(stream)
    srv = Server(backend, slots=4, budget_bytes=8 << 30)
    mix = srv.run(reqs)
    stats = dict(srv.stats)
    srv.close()
    s = summarize(mix)
    assert s["completed"] == len(reqs) and s["all_converged"]
    assert stats["hits"] > 0 and stats["max_concurrency"] >= 2
    for r in mix:
        assert r.rel_res_true <= 1.01e-8
    for r, req in list(zip(mix, reqs))[:8]:
        alone_srv = Server(backend, slots=1, budget_bytes=8 << 30)
        (a,) = alone_srv.run([Request(0, 0.0, req.op_id, req.N, req.eps, req.rhs_seed)])
        alone_srv.close()
        assert a.iterations == r.iterations
        np.testing.assert_array_equal(a.x, r.x)


def test_gpu_serving_eviction_under_small_budget(backend):
    from paper_2006_16147_amd.serve import Server, requests_from_stream, summarize

    stream = inputs.serving_requests(12, rate=500.0, seed=5, sizes=(24, 32))
    reqs = requests_from_stream(stream)
    one = backend.estimate_bytes(reqs[0]) + backend.solve_bytes(reqs[0])
    budget = int(1.6 * max(backend.estimate_bytes(r) + backend.solve_bytes(r) for r in reqs))
    srv = Server(backend, slots=4, budget_bytes=max(budget, one))
    res = srv.run(reqs)
    srv.close()
    assert summarize(res)["completed"] == len(reqs)
    assert srv.peak_used <= srv.budget


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_footprint_estimate_bounds_the_hierarchy(backend, precision):
    """Admission reserves amg_estimate_footprint: it must cover what a
    hierarchy keeps, for isotropic and anisotropic operators of the stream."""
    import torch

    from paper_2006_16147_amd import amg

    prec = amg.FP32 if precision == "fp32" else amg.FP64
    params = amg.amg_params_default(precision=prec)
    for N, eps in ((32, (1.0, 1.0)), (48, (1e-3, 1.0)), (64, (0.05, 0.3))):
        rp, ci, va = inputs.constant_diffusion7_arrays(N, eps[0], eps[1], 1.0, torch,
                                                       device="cuda")
        h = amg.amg_setup(rp, ci, va, precision=prec)
        est = amg.amg_estimate_footprint(N ** 3, int(va.numel()), params)
        assert h.footprint_bytes() <= est, (N, eps, h.footprint_bytes(), est)
        h.close()
