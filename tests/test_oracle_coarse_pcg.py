"""Pins of the oracle's iterative coarsest solver (Section 5: CG with a
Jacobi-type preconditioner on the coarsest level, stopped at relative
residual 1e-4 or after 30 iterations; the GPU runs use l1-Jacobi there).

Nothing here retypes the recurrence: it must reproduce SciPy's
preconditioned CG iterate for iterate and stop at the same step, reach the
exact solution after n steps on an n-row system, give the closed-form
energy minimiser along M^-1 b after one step, and, inside the cycle, be the
coarse solve itself.
"""

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spl

from paper_2006_16147_amd import inputs


def _sp(A):
    return sp.csr_matrix((A.val, A.col, A.row_ptr), shape=(A.n, A.n))


def _coarsest(orc, A):
    ho = orc.Hierarchy(A)
    L = ho.num_levels - 1
    return ho.level_csr(L), ho.l1diag(L)


def _systems(orc):
    rng = np.random.default_rng(4)
    out = {"poisson16_coarsest": _coarsest(orc, inputs.laplacian7(16)),
           "poisson32_coarsest": _coarsest(orc, inputs.laplacian7(32)),
           "aniso_coarsest": _coarsest(orc, inputs.diffusion7(
               24, *inputs.block_log_uniform_eps(24, 8, rng), 1.0)),
           "random_graph": None}
    G = inputs.random_spd_graph(300, 6.0, seed=5)
    out["random_graph"] = (G, orc.l1_diag(G))
    return out


@pytest.mark.parametrize("rtol,maxit", [(1e-4, 30), (1e-8, 30), (1e-4, 3), (1e-12, 200)])
def test_coarse_pcg_is_scipy_cg_with_the_l1_diagonal(orc, rtol, maxit):
    for name, (A, m) in _systems(orc).items():
        b = np.random.default_rng(len(name)).uniform(-1, 1, A.n)
        x, it = orc.coarse_pcg(A, m, b, rtol, maxit)
        count = [0]

        def cb(_):
            count[0] += 1

        xs, info = spl.cg(_sp(A), b, x0=np.zeros(A.n), rtol=rtol, atol=0.0, maxiter=maxit,
                          M=sp.diags(1.0 / m), callback=cb)
        assert it == count[0], (name, it, count[0])
        assert it <= maxit
        assert np.linalg.norm(x - xs) <= 1e-10 * np.linalg.norm(xs), name
        r = b - _sp(A) @ x
        if it < maxit:  # stopped by the test: ||r|| < rtol ||b||
            assert np.linalg.norm(r) < rtol * np.linalg.norm(b) * (1 + 1e-8)


def test_coarse_pcg_terminates_at_the_exact_solution(orc):
    """CG reaches the solution in at most n steps in exact arithmetic; with
    rtol = 0 it runs all n of them."""
    for A in (inputs.laplacian7(4), _coarsest(orc, inputs.laplacian7(16))[0]):
        m = orc.l1_diag(A)
        b = np.random.default_rng(1).uniform(-1, 1, A.n)
        x, it = orc.coarse_pcg(A, m, b, 0.0, A.n)
        assert it == A.n
        xs = np.linalg.solve(_sp(A).toarray(), b)
        assert np.linalg.norm(x - xs) <= 1e-10 * np.linalg.norm(xs)


def test_one_iteration_is_the_energy_minimiser_along_m_inverse_b(orc):
    A = inputs.laplacian7(5)
    m = orc.l1_diag(A)
    b = np.random.default_rng(2).uniform(-1, 1, A.n)
    x, it = orc.coarse_pcg(A, m, b, 1e-4, 1)
    z = b / m
    ref = (z @ b) / (z @ (_sp(A) @ z)) * z
    assert it == 1
    np.testing.assert_allclose(x, ref, rtol=1e-14, atol=0)


def test_zero_rhs_and_zero_maxit(orc):
    A = inputs.laplacian7(4)
    m = orc.l1_diag(A)
    x, it = orc.coarse_pcg(A, m, np.zeros(A.n), 1e-4, 30)
    assert it == 0 and not x.any()
    x, it = orc.coarse_pcg(A, m, np.ones(A.n), 1e-4, 0)
    assert it == 0 and not x.any()


def test_vcycle_with_iterative_coarsest_solves_the_coarsest_system(orc):
    # a one-level hierarchy: the cycle is the coarsest solve itself
    A = inputs.laplacian7(5)  # 125 <= max_coarse
    h1 = orc.Hierarchy(A, coarse=(1e-4, 30))
    assert h1.num_levels == 1
    r = np.random.default_rng(3).uniform(-1, 1, A.n)
    x, it = orc.coarse_pcg(A, orc.l1_diag(A), r, 1e-4, 30)
    assert 1 < it < 30
    np.testing.assert_array_equal(h1.vcycle(r), x)
    # run to the exact solution it gives the Cholesky cycle
    A = inputs.laplacian7(16)
    hc = orc.Hierarchy(A)
    nL = hc.level_n(hc.num_levels - 1)
    he = orc.Hierarchy(A, coarse=(0.0, nL))
    r = np.random.default_rng(4).uniform(-1, 1, A.n)
    zc, ze = hc.vcycle(r), he.vcycle(r)
    assert np.linalg.norm(ze - zc) <= 1e-10 * np.linalg.norm(zc)
    # stopped at 1e-4 it is a perturbation of that cycle, not the same one
    ha = orc.Hierarchy(A, coarse=(1e-4, 30))
    za = ha.vcycle(r)
    d = np.linalg.norm(za - zc) / np.linalg.norm(zc)
    assert 0 < d < 1e-2


@pytest.mark.parametrize("sweeps", [1, 4])
def test_flexible_cg_with_iterative_coarsest_converges(orc, sweeps):
    """Section 5's GPU configuration: l1-Jacobi with 4 pre/post sweeps and
    the CG coarsest solver, inside flexible CG; the iteration count stays
    within two of the exact coarsest solve's."""
    c = inputs.small_case(24, seed=0)
    A, b = c["A"], c["b"]
    _, ic = orc.Hierarchy(A).fcg(b, rtol=1e-8, maxit=300, pre=sweeps, post=sweeps, cycle="V")
    x, ia = orc.Hierarchy(A, coarse=(1e-4, 30)).fcg(b, rtol=1e-8, maxit=300, pre=sweeps,
                                                      post=sweeps, cycle="V")
    assert ia["converged"] and ia["rel_res_true"] <= 1.001e-8
    assert abs(ia["iterations"] - ic["iterations"]) <= 2, (ia, ic)
    _, ik = orc.Hierarchy(A, coarse=(1e-4, 30)).fcg(b, rtol=1e-8, maxit=300, pre=sweeps,
                                                      post=sweeps, cycle="K")
    assert ik["converged"] and ik["iterations"] <= ia["iterations"]
