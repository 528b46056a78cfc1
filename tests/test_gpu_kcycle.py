"""GPU K-cycle (Section 3.1) and flexible CG against the oracle.

The K-cycle is not a fixed linear operator (its inner flexible-CG steps
depend on the vector), so one application is compared with the oracle's on
the same vector, and solves are compared at equal iteration counts.
"""

import numpy as np
import pytest

from paper_2006_16147_amd import inputs

from gpu_helpers import setup, solve, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


CASES = {
    "poisson20": (lambda: inputs.laplacian7(20), {}),        # one intermediate level
    "poisson40": (lambda: inputs.laplacian7(40), {}),        # two intermediate levels
    "poisson40_pre2post2": (lambda: inputs.laplacian7(40), {"pre": 2, "post": 2}),
    "aniso24": (lambda: inputs.diffusion7(24, *inputs.block_log_uniform_eps(
        24, 8, np.random.default_rng(2)), 1.0), {}),
    "random": (lambda: inputs.random_spd_graph(4000, 6.0, seed=3), {}),
}


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("case", sorted(CASES))
def test_kcycle_application_matches_oracle(orc, case, precision):
    import torch

    from paper_2006_16147_amd import amg

    make, sm = CASES[case]
    A = make()
    prec = amg.FP32 if precision == "fp32" else amg.FP64
    h = setup(A, cycle=amg.CYCLE_K, precision=prec, **sm)
    ho = orc.Hierarchy(A)
    assert h.sizes() == [ho.level_n(l) for l in range(ho.num_levels)]
    r = np.random.default_rng(7).uniform(-1, 1, A.n)
    z = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    amg.amg_vcycle_apply(h, to_dev(r), z)
    zo = ho.kcycle(r, pre=sm.get("pre", 1), post=sm.get("post", 1))
    tol = 1e-10 if precision == "fp64" else 1e-4
    np.testing.assert_allclose(z.cpu().numpy(), zo, rtol=0, atol=tol * np.abs(zo).max())


@pytest.mark.parametrize("case", ["poisson20", "poisson40", "aniso24", "random"])
def test_fcg_kcycle_matches_oracle_at_equal_iterations(orc, case):
    from paper_2006_16147_amd import amg

    make, sm = CASES[case]
    A = make()
    b = np.random.default_rng(11).uniform(-1, 1, A.n)
    h = setup(A, cycle=amg.CYCLE_K)
    ho = orc.Hierarchy(A)
    st, info, x = solve(h, b, rtol=1e-8, maxit=300)
    assert st == 0 and info["converged"] and info["rel_res_true"] <= 1.001e-8
    _, io = ho.fcg(b, rtol=1e-8, maxit=300, cycle="K")
    assert abs(info["iterations"] - io["iterations"]) <= 1, (info, io)
    xo, _ = ho.fcg(b, rtol=0.0, maxit=info["iterations"], cycle="K")
    assert np.linalg.norm(x - xo) / np.linalg.norm(xo) < 1e-8


def test_fcg_kcycle_fp32_hierarchy_reaches_fp64_residual(orc):
    from paper_2006_16147_amd import amg

    c = inputs.small_case(32, seed=0)
    A, b = c["A"], c["b"]
    h = setup(A, cycle=amg.CYCLE_K, precision=amg.FP32)
    st, info, x = solve(h, b, rtol=1e-8, maxit=300)
    assert st == 0 and info["rel_res_true"] <= 1.01e-8
    _, io = orc.Hierarchy(A).fcg(b, rtol=1e-8, maxit=300, cycle="K")
    assert abs(info["iterations"] - io["iterations"]) <= 2


def test_kcycle_two_levels_is_the_vcycle():
    import torch

    from paper_2006_16147_amd import amg

    A = inputs.laplacian7(8)
    hk = setup(A, cycle=amg.CYCLE_K)
    hv = setup(A)
    assert hk.sizes() == [512, 64]
    r = to_dev(np.random.default_rng(1).uniform(-1, 1, A.n))
    zk = torch.zeros_like(r)
    zv = torch.zeros_like(r)
    amg.amg_vcycle_apply(hk, r, zk)
    amg.amg_vcycle_apply(hv, r, zv)
    assert torch.equal(zk, zv)


def test_kcycle_edge_cases_and_batch_rejected(orc):
    import torch

    from paper_2006_16147_amd import amg

    c = inputs.small_case(16, seed=0)
    A, b = c["A"], c["b"]
    h = setup(A, cycle=amg.CYCLE_K, max_coarse=20)
    st, info, x = solve(h, np.zeros(A.n), x0=np.ones(A.n))
    assert st == 0 and info["iterations"] == 0 and not x.any()
    st, info, x = solve(h, b, rtol=0.0, maxit=4)
    assert st == amg.Status.NOT_CONVERGED and info["iterations"] == 4
    xo, _ = orc.Hierarchy(A, max_coarse=20).fcg(b, rtol=0.0, maxit=4, cycle="K")
    assert np.linalg.norm(x - xo) / np.linalg.norm(xo) < 1e-10
    B = to_dev(np.ascontiguousarray(np.random.default_rng(0).uniform(-1, 1, (A.n, 3))))
    X = torch.zeros_like(B)
    st, _ = amg.amg_pcg_solve_batch(h, B, X, raise_on_error=False)
    assert st == amg.Status.ERR_ARG


def test_kcycle_headline_size_against_oracle(orc):
    """160^3 Poisson (b = A u): K-cycle flexible CG reaches rtol 1e-8 within
    one iteration of the oracle's count and agrees with it at equal counts."""
    from paper_2006_16147_amd import amg

    c = inputs.headline_case(160, seed=1)
    A, b = c["A"], c["b"]
    h = setup(A, cycle=amg.CYCLE_K)
    st, info, x = solve(h, b, rtol=1e-8, maxit=200)
    assert st == 0 and info["rel_res_true"] <= 1.001e-8
    ho = orc.Hierarchy(A)
    xo, io = ho.fcg(b, rtol=0.0, maxit=info["iterations"], cycle="K")
    assert np.linalg.norm(x - xo) / np.linalg.norm(xo) < 1e-8
    h.close()
