"""Parity at the benchmark's full size and launch configuration.

160^3 Poisson (n = 4 096 000) with b = A u: the whole GPU hierarchy is
compared bit for bit with the oracle's (its serial setup takes seconds at
this size), the closed-form cube aggregates are checked, and the solve is
compared with the oracle at an equal iteration count. The 256^3 anisotropic
case checks properties that hold at any size.
"""

import numpy as np
import pytest

from paper_2006_16147_amd import inputs

from gpu_helpers import assert_same_hierarchy, setup, solve

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


@pytest.fixture(scope="module")
def headline():
    return inputs.headline_case(160, seed=1)


def _cubes(N):
    idx = np.arange(N ** 3)
    x, y, z = idx % N, (idx // N) % N, idx // (N * N)
    return (x // 2) + (N // 2) * ((y // 2) + (N // 2) * (z // 2))


def test_headline_hierarchy_bit_exact(orc, headline):
    A = headline["A"]
    h = setup(A)
    assert h.sizes() == [4096000, 512000, 64000, 8000, 1000, 125]
    agg, p = h.transfer(0)
    np.testing.assert_array_equal(agg, _cubes(160))
    ho = orc.Hierarchy(A)
    assert_same_hierarchy(h, ho)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_headline_solve(orc, headline, precision):
    from paper_2006_16147_amd import amg

    A, b, u = headline["A"], headline["b"], headline["u"]
    prec = amg.FP64 if precision == "fp64" else amg.FP32
    h = setup(A, precision=prec)
    st, info, x = solve(h, b, rtol=1e-8, maxit=200)
    assert st == 0 and info["converged"]
    assert info["rel_res_true"] <= 1.001e-8
    # error bound ||x - u|| <= kappa(A) ||r|| / ||b|| ||u|| with kappa < 2e4
    assert np.linalg.norm(x - u) / np.linalg.norm(u) < 1e-8 * 1.2e4
    if precision == "fp64":
        ho = orc.Hierarchy(A)
        xo, io = ho.pcg(b, rtol=0.0, maxit=info["iterations"])
        assert np.linalg.norm(x - xo) / np.linalg.norm(xo) < 1e-8
        _, io_conv = ho.pcg(b, rtol=1e-8, maxit=200)
        assert abs(io_conv["iterations"] - info["iterations"]) <= 1


def test_headline_vcycle_sampled_against_oracle(orc, headline):
    """One V-cycle on a random vector: every 997th entry checked."""
    import torch

    from paper_2006_16147_amd import amg

    A = headline["A"]
    h = setup(A)
    ho = orc.Hierarchy(A)
    r = np.random.default_rng(11).uniform(-1, 1, A.n)
    z = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    amg.amg_vcycle_apply(h, torch.from_numpy(r).cuda(), z)
    zg = z.cpu().numpy()
    zo = ho.vcycle(r)
    sel = np.arange(0, A.n, 997)
    np.testing.assert_allclose(zg[sel], zo[sel], rtol=0, atol=1e-12 * np.abs(zo).max())


def test_aniso_256_fp32_vs_fp64():
    """256^3 anisotropic blocks: both hierarchies reach the FP64 residual and
    agree within the conditioning bound."""
    from paper_2006_16147_amd import amg

    import torch

    ex, ey, b = inputs.aniso_blocks_coefficients(256, 16, seed=2)
    rp, ci, va = inputs.diffusion7_torch(256, torch.from_numpy(ex), torch.from_numpy(ey), 1.0,
                                         "cuda")
    h64 = amg.amg_setup(rp, ci, va)
    st, i64, x64 = solve(h64, b, rtol=1e-8, maxit=500)
    h64.close()
    h32 = amg.amg_setup(rp, ci, va, precision=amg.FP32)
    st32, i32, x32 = solve(h32, b, rtol=1e-8, maxit=500)
    h32.close()
    assert st == 0 and st32 == 0
    assert i64["rel_res_true"] <= 1.001e-8 and i32["rel_res_true"] <= 1.01e-8
    assert np.linalg.norm(x32 - x64) / np.linalg.norm(x64) < 1e-4


def test_batch_128_k32_sampled_against_oracle(orc):
    """Multi-RHS at its full size and launch configuration (128^3, k = 32,
    FP32 hierarchy, autotuned tile): every column reaches the FP64 true
    residual, and two sampled columns match the oracle's FP64 solve."""
    import torch

    from paper_2006_16147_amd import amg

    c = inputs.multi_rhs_case(128, 32, seed=3)
    A, B = c["A"], c["B"]
    h = setup(A, precision=amg.FP32)
    Bd = torch.from_numpy(B).cuda()
    X = torch.zeros_like(Bd)
    st, infos = amg.amg_pcg_solve_batch(h, Bd, X, rtol=1e-8, maxit=200)
    assert st == 0
    assert all(i["converged"] and i["rel_res_true"] <= 1.01e-8 for i in infos)
    Xh = X.cpu().numpy()
    ho = orc.Hierarchy(A)
    for j in (0, 31):
        xo, io = ho.pcg(B[:, j], rtol=1e-8, maxit=200)
        assert abs(io["iterations"] - infos[j]["iterations"]) <= 2
        # both solutions within the conditioning bound of the exact one
        assert np.linalg.norm(Xh[:, j] - xo) / np.linalg.norm(xo) < 1e-8 * 1.2e4
    h.close()


def test_smoothed_hierarchy_and_paper_gpu_preconditioner_at_160(orc, headline):
    """Smoothed aggregation at the benchmark size: the GPU hierarchy (levels,
    every coarse matrix, every Pbar) bit-exact with the oracle's, and Section
    5's GPU preconditioner (Pbar, 4 l1-Jacobi pre/post sweeps, CG coarsest)
    reaching 1e-6 in 7 flexible-CG iterations, equal to the oracle's iterate."""
    from paper_2006_16147_amd import amg

    A, b = headline["A"], headline["b"]
    h = setup(A, smooth_p=1, pre=4, post=4, coarse_solver=amg.COARSE_PCG)
    ho = orc.Hierarchy(A, smooth=True, coarse=(1e-4, 30))
    assert h.sizes() == ho.sizes() and h.nnzs() == ho.nnzs()
    for l in range(1, ho.num_levels):
        _, _, val = h.level_csr(l)
        np.testing.assert_array_equal(val.view(np.uint64), ho.level_csr(l).val.view(np.uint64))
    for l in range(ho.num_levels - 1):
        (_, _, pv), om = h.prolongator(l)
        assert om == ho.omega(l)
        np.testing.assert_array_equal(pv.view(np.uint64), ho.pbar(l)[2].view(np.uint64))
    st, info, x = solve(h, b, rtol=1e-6, maxit=100)
    assert st == 0 and info["iterations"] == 7 and info["rel_res_true"] <= 1.001e-6
    xo, _ = ho.fcg(b, rtol=0.0, maxit=7, pre=4, post=4, cycle="V")
    assert np.linalg.norm(x - xo) / np.linalg.norm(xo) < 1e-8
    h.close()
