"""GPU iterative coarsest solve (Section 5: CG with the l1-Jacobi diagonal,
stopped at relative residual 1e-4 or after 30 iterations) against the
oracle, inside the V-cycle, the K-cycle and the flexible-CG solve.

The cycle with this coarsest solve is not a fixed linear operator, so one
application is compared with the oracle's on the same vector, and solves at
equal iteration counts.
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


def _apply(h, r, kcycle=False):
    import torch

    from paper_2006_16147_amd import amg

    z = torch.zeros(len(r), dtype=torch.float64, device="cuda")
    amg.amg_vcycle_apply(h, to_dev(r), z)
    return z.cpu().numpy()


CASES = {
    "poisson16": lambda: inputs.laplacian7(16),          # 4096 -> 512 -> 64
    "poisson40": lambda: inputs.laplacian7(40),          # coarsest 125
    "aniso24": lambda: inputs.diffusion7(24, *inputs.block_log_uniform_eps(
        24, 8, np.random.default_rng(2)), 1.0),
    "random": lambda: inputs.random_spd_graph(4000, 6.0, seed=3),
}


@pytest.mark.parametrize("coarse", [(1e-4, 30), (0.0, 30), (0.0, 3)])
@pytest.mark.parametrize("sweeps", [1, 4])
@pytest.mark.parametrize("case", sorted(CASES))
def test_vcycle_with_cg_coarsest_matches_oracle(orc, case, sweeps, coarse):
    from paper_2006_16147_amd import amg

    A = CASES[case]()
    h = setup(A, coarse_solver=amg.COARSE_PCG, coarse_rtol=coarse[0], coarse_maxit=coarse[1],
              pre=sweeps, post=sweeps)
    ho = orc.Hierarchy(A, coarse=coarse)
    assert h.sizes() == ho.sizes()
    L = ho.num_levels - 1
    np.testing.assert_array_equal(h.l1diag(L), ho.l1diag(L))
    r = np.random.default_rng(7).uniform(-1, 1, A.n)
    z, zo = _apply(h, r), ho.vcycle(r, pre=sweeps, post=sweeps)
    np.testing.assert_allclose(z, zo, rtol=0, atol=1e-10 * np.abs(zo).max())


@pytest.mark.parametrize("case", ["poisson16", "poisson40", "aniso24"])
def test_kcycle_with_cg_coarsest_matches_oracle(orc, case):
    from paper_2006_16147_amd import amg

    A = CASES[case]()
    h = setup(A, cycle=amg.CYCLE_K, coarse_solver=amg.COARSE_PCG)
    ho = orc.Hierarchy(A, coarse=(1e-4, 30))
    r = np.random.default_rng(8).uniform(-1, 1, A.n)
    z, zo = _apply(h, r), ho.kcycle(r)
    np.testing.assert_allclose(z, zo, rtol=0, atol=1e-10 * np.abs(zo).max())


def test_one_level_hierarchy_is_the_coarse_cg(orc):
    from paper_2006_16147_amd import amg

    A = inputs.laplacian7(5)  # 125 unknowns: no coarsening
    h = setup(A, coarse_solver=amg.COARSE_PCG)
    assert h.sizes() == [125]
    r = np.random.default_rng(3).uniform(-1, 1, A.n)
    x, it = orc.coarse_pcg(A, orc.l1_diag(A), r, 1e-4, 30)
    assert 1 < it < 30
    np.testing.assert_allclose(_apply(h, r), x, rtol=0, atol=1e-12 * np.abs(x).max())
    b = np.random.default_rng(4).uniform(-1, 1, A.n)
    st, info, xs = solve(h, b, rtol=1e-10, maxit=100)
    assert st == 0 and info["rel_res_true"] <= 1.001e-10
    _, io = orc.Hierarchy(A, coarse=(1e-4, 30)).fcg(b, rtol=1e-10, maxit=100, cycle="V")
    assert abs(info["iterations"] - io["iterations"]) <= 1


@pytest.mark.parametrize("case,sweeps", [("poisson40", 4), ("aniso24", 4), ("random", 1),
                                         ("poisson40", 1)])
def test_fcg_with_cg_coarsest_matches_oracle_at_equal_iterations(orc, case, sweeps):
    from paper_2006_16147_amd import amg

    A = CASES[case]()
    b = np.random.default_rng(11).uniform(-1, 1, A.n)
    h = setup(A, coarse_solver=amg.COARSE_PCG, pre=sweeps, post=sweeps)
    st, info, x = solve(h, b, rtol=1e-8, maxit=300)
    assert st == 0 and info["converged"] and info["rel_res_true"] <= 1.001e-8
    ho = orc.Hierarchy(A, coarse=(1e-4, 30))
    _, io = ho.fcg(b, rtol=1e-8, maxit=300, pre=sweeps, post=sweeps, cycle="V")
    assert abs(info["iterations"] - io["iterations"]) <= 1, (info, io)
    xo, _ = ho.fcg(b, rtol=0.0, maxit=info["iterations"], pre=sweeps, post=sweeps, cycle="V")
    assert np.linalg.norm(x - xo) / np.linalg.norm(xo) < 1e-8


def test_fp32_hierarchy_with_cg_coarsest_reaches_fp64_residual(orc):
    from paper_2006_16147_amd import amg

    c = inputs.small_case(32, seed=0)
    A, b = c["A"], c["b"]
    h = setup(A, coarse_solver=amg.COARSE_PCG, precision=amg.FP32, pre=4, post=4)
    st, info, x = solve(h, b, rtol=1e-8, maxit=300)
    assert st == 0 and info["rel_res_true"] <= 1.01e-8
    _, io = orc.Hierarchy(A, coarse=(1e-4, 30)).fcg(b, rtol=1e-8, maxit=300, pre=4, post=4,
                                                      cycle="V")
    assert abs(info["iterations"] - io["iterations"]) <= 2


def test_cg_coarsest_edge_cases_and_rejections():
    import torch

    from paper_2006_16147_amd import amg

    from gpu_helpers import setup_status

    c = inputs.small_case(16, seed=0)
    A, b = c["A"], c["b"]
    h = setup(A, coarse_solver=amg.COARSE_PCG)
    # zero right-hand side; zero coarse residual inside the cycle
    st, info, x = solve(h, np.zeros(A.n), x0=np.ones(A.n))
    assert st == 0 and info["iterations"] == 0 and not x.any()
    assert not _apply(h, np.zeros(A.n)).any()
    # the block solve runs the Cholesky coarsest only
    B = to_dev(np.ascontiguousarray(np.random.default_rng(0).uniform(-1, 1, (A.n, 3))))
    st, _ = amg.amg_pcg_solve_batch(h, B, torch.zeros_like(B), raise_on_error=False)
    assert st == amg.Status.ERR_ARG
    for bad in ({"coarse_solver": 2}, {"coarse_solver": amg.COARSE_PCG, "coarse_maxit": 0},
                {"coarse_solver": amg.COARSE_PCG, "coarse_rtol": -1.0},
                {"coarse_solver": amg.COARSE_PCG, "coarse_rtol": float("nan")}):
        assert setup_status(A, **bad)[0] == amg.Status.ERR_ARG, bad
    # the whole-cycle timer leaves the iterative coarsest solve out of its bytes
    hc = setup(A)
    _, by_c = hc.time_kernel(5, 0, reps=2)
    _, by_p = h.time_kernel(5, 0, reps=2)
    nL = hc.sizes()[-1]
    assert by_c - by_p == 8.0 * nL * nL + 8.0 * nL


def test_paper_gpu_configuration_at_160(orc):
    """Section 5's GPU preconditioner on the 160^3 Poisson problem: V-cycle,
    l1-Jacobi with 4 pre/post sweeps, CG coarsest at 1e-4 / 30, flexible
    CG outside; agrees with the oracle at equal iteration counts."""
    from paper_2006_16147_amd import amg

    c = inputs.headline_case(160, seed=1)
    A, b = c["A"], c["b"]
    h = setup(A, coarse_solver=amg.COARSE_PCG, pre=4, post=4)
    st, info, x = solve(h, b, rtol=1e-8, maxit=200)
    assert st == 0 and info["rel_res_true"] <= 1.001e-8
    ho = orc.Hierarchy(A, coarse=(1e-4, 30))
    xo, _ = ho.fcg(b, rtol=0.0, maxit=info["iterations"], pre=4, post=4, cycle="V")
    assert np.linalg.norm(x - xo) / np.linalg.norm(xo) < 1e-8
    h.close()
