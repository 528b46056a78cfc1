"""GPU smoothed aggregation (the alternative to the K-cycle in Section 3.2)
against the oracle: omega, Pbar = (I - omega D^-1 A) P and every coarse
matrix Pbar^T A Pbar bit for bit (both sum every entry in the same fixed
order), the V-cycle with Pbar^T / Pbar to FP64 rounding, and solves at equal
iteration counts.
"""

import numpy as np
import pytest

from paper_2006_16147_amd import inputs

from gpu_helpers import assert_same_hierarchy, setup, setup_status, solve, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


CASES = {
    "poisson16": lambda: inputs.laplacian7(16),
    "poisson24": lambda: inputs.laplacian7(24),
    "aniso16": lambda: inputs.diffusion7(16, *inputs.block_log_uniform_eps(
        16, 4, np.random.default_rng(2)), 1.0),
    "random": lambda: inputs.random_spd_graph(3000, 6.0, seed=3),
}


def _apply(h, r):
    import torch

    from paper_2006_16147_amd import amg

    z = torch.zeros(len(r), dtype=torch.float64, device="cuda")
    amg.amg_vcycle_apply(h, to_dev(r), z)
    return z.cpu().numpy()


@pytest.mark.parametrize("case", sorted(CASES))
def test_smoothed_hierarchy_is_bit_exact(orc, case):
    A = CASES[case]()
    h = setup(A, smooth_p=1)
    ho = orc.Hierarchy(A, smooth=True)
    assert ho.ok
    assert_same_hierarchy(h, ho)
    for l in range(ho.num_levels - 1):
        (rp, ci, val), om = h.prolongator(l)
        rpo, cio, valo = ho.pbar(l)
        assert om == ho.omega(l)
        np.testing.assert_array_equal(rp, rpo)
        np.testing.assert_array_equal(ci, cio)
        np.testing.assert_array_equal(val.view(np.uint64), valo.view(np.uint64))


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("sweeps", [1, 4])
@pytest.mark.parametrize("case", ["poisson24", "aniso16", "random"])
def test_smoothed_vcycle_matches_oracle(orc, case, sweeps, precision):
    from paper_2006_16147_amd import amg

    A = CASES[case]()
    prec = amg.FP32 if precision == "fp32" else amg.FP64
    h = setup(A, smooth_p=1, pre=sweeps, post=sweeps, precision=prec)
    ho = orc.Hierarchy(A, smooth=True)
    r = np.random.default_rng(7).uniform(-1, 1, A.n)
    z, zo = _apply(h, r), ho.vcycle(r, pre=sweeps, post=sweeps)
    tol = 1e-10 if precision == "fp64" else 1e-4
    np.testing.assert_allclose(z, zo, rtol=0, atol=tol * np.abs(zo).max())


@pytest.mark.parametrize("case", ["poisson24", "aniso16", "random"])
def test_smoothed_pcg_matches_oracle_at_equal_iterations(orc, case):
    A = CASES[case]()
    b = np.random.default_rng(11).uniform(-1, 1, A.n)
    h = setup(A, smooth_p=1)
    st, info, x = solve(h, b, rtol=1e-8, maxit=300)
    assert st == 0 and info["rel_res_true"] <= 1.001e-8
    ho = orc.Hierarchy(A, smooth=True)
    _, io = ho.pcg(b, rtol=1e-8, maxit=300)
    assert abs(info["iterations"] - io["iterations"]) <= 1, (info, io)
    xo, _ = ho.pcg(b, rtol=0.0, maxit=info["iterations"])
    assert np.linalg.norm(x - xo) / np.linalg.norm(xo) < 1e-8


def test_paper_gpu_preconditioner_with_smoothed_prolongator(orc):
    """Section 5's GPU preconditioner in full: smoothed prolongator from three
    sweeps of matching, 4 l1-Jacobi pre/post sweeps, CG coarsest solve, FCG
    outside; agrees with the oracle at equal iteration counts."""
    from paper_2006_16147_amd import amg

    c = inputs.small_case(32, seed=0)
    A, b = c["A"], c["b"]
    h = setup(A, smooth_p=1, pre=4, post=4, coarse_solver=amg.COARSE_PCG)
    st, info, x = solve(h, b, rtol=1e-6, maxit=100)
    assert st == 0 and 6 <= info["iterations"] <= 9
    ho = orc.Hierarchy(A, smooth=True, coarse=(1e-4, 30))
    xo, _ = ho.fcg(b, rtol=0.0, maxit=info["iterations"], pre=4, post=4, cycle="V")
    assert np.linalg.norm(x - xo) / np.linalg.norm(xo) < 1e-8


def test_smoothed_rejections_and_byte_count():
    import torch

    from paper_2006_16147_amd import amg

    c = inputs.small_case(16, seed=0)
    A = c["A"]
    assert setup_status(A, smooth_p=1, cycle=amg.CYCLE_K)[0] == amg.Status.ERR_ARG
    assert setup_status(A, smooth_p=2)[0] == amg.Status.ERR_ARG
    h = setup(A, smooth_p=1)
    B = to_dev(np.ascontiguousarray(np.random.default_rng(0).uniform(-1, 1, (A.n, 2))))
    st, _ = amg.amg_pcg_solve_batch(h, B, torch.zeros_like(B), raise_on_error=False)
    assert st == amg.Status.ERR_ARG
    for k in (0, 2, 3):
        with pytest.raises(amg.AmgError):
            h.time_kernel(k, 0, reps=1)
    ms, by = h.time_kernel(5, 0, reps=2)
    assert ms > 0 and by > 0
    with pytest.raises(amg.AmgError):
        setup(A).prolongator(0)
    # a one-level hierarchy has no prolongator and solves exactly
    h1 = setup(inputs.laplacian7(5), smooth_p=1)
    assert h1.sizes() == [125]
    st, info, _ = solve(h1, np.ones(125), rtol=1e-10)
    assert st == 0 and info["iterations"] == 1


def test_smoothed_hierarchy_at_80_matches_oracle(orc):
    """80^3 Poisson (512k unknowns, the paper's per-core size): the smoothed
    hierarchy is bit-exact with the oracle's; opc 2.025 with omega =
    4 / (3 ||D^-1 A||_inf) (the paper prints 1.835)."""
    A = inputs.laplacian7(80)
    h = setup(A, smooth_p=1)
    ho = orc.Hierarchy(A, smooth=True)
    assert h.sizes() == ho.sizes() == [512000, 64000, 8056, 1019, 129]
    assert h.nnzs() == ho.nnzs()
    for l in range(1, ho.num_levels):
        _, _, val = h.level_csr(l)
        np.testing.assert_array_equal(val.view(np.uint64), ho.level_csr(l).val.view(np.uint64))
    assert abs(h.opc() - 2.0255) < 1e-3
