"""Pins of the oracle's K-cycle and flexible CG (Section 3.1, Section 5).

Nothing here is the formula retyped: flexible CG with a fixed s.p.d.
preconditioner must reproduce preconditioned CG; the two inner FCG
iterations must satisfy the Galerkin conditions of the A-orthogonal
projection onto the two preconditioned residuals they generate; a hierarchy
without intermediate levels has no FCG to apply; and the paper's reason for
the K-cycle (the V-cycle with unsmoothed aggregation is not optimal, its
iteration count grows with the grid) must show up.
"""

import numpy as np
import pytest
import scipy.sparse as sp

from paper_2006_16147_amd import inputs


def _csr(ho, l):
    M = ho.level_csr(l)
    return sp.csr_matrix((M.val, M.col, M.row_ptr), shape=(M.n, M.n))


@pytest.mark.parametrize("k", [1, 3, 8])
def test_fcg_with_vcycle_equals_pcg(orc, k):
    """FCG (truncation 1) and PCG coincide for a fixed s.p.d. preconditioner
    (Section 5 uses FCG; the V-cycle with Cholesky coarsest is fixed)."""
    c = inputs.small_case(20, seed=0)
    ho = orc.Hierarchy(c["A"])
    xp, ip = ho.pcg(c["b"], rtol=0.0, maxit=k)
    xf, jf = ho.fcg(c["b"], rtol=0.0, maxit=k, cycle="V")
    assert ip["iterations"] == jf["iterations"] == k
    assert np.linalg.norm(xf - xp) / np.linalg.norm(xp) < 1e-12


@pytest.mark.parametrize("m", [1, 2])
def test_fcg2_is_the_galerkin_projection(orc, m):
    """Two FCG iterations from zero return the A-orthogonal projection of the
    solution onto span{c1, c2}, c1 = K(b), c2 = K(b - s1 A c1) with s1 the
    first step length: x lies in that span and its residual is orthogonal to
    both vectors."""
    A0 = inputs.laplacian7(40)  # levels 64000, 8000, 1000, 125
    ho = orc.Hierarchy(A0)
    assert ho.num_levels == 4
    Am = _csr(ho, m)
    b = np.random.default_rng(m).uniform(-1, 1, ho.level_n(m))
    x = ho.fcg2(b, m)
    c1 = ho.kcycle(b, l=m)
    v1 = Am @ c1
    s1 = (c1 @ b) / (c1 @ v1)
    c2 = ho.kcycle(b - s1 * v1, l=m)
    C = np.stack([c1, c2], axis=1)
    coef, *_ = np.linalg.lstsq(C, x, rcond=None)
    assert np.linalg.norm(C @ coef - x) <= 1e-12 * np.linalg.norm(x)
    res = b - Am @ x
    for cv in (c1, c2):
        assert abs(cv @ res) <= 1e-12 * np.linalg.norm(cv) * np.linalg.norm(b)
    # and it improves on the first step alone in the energy norm
    xs = np.linalg.solve(Am.toarray(), b) if Am.shape[0] <= 8000 else None
    if xs is not None:
        e2 = (xs - x) @ (Am @ (xs - x))
        e1 = (xs - s1 * c1) @ (Am @ (xs - s1 * c1))
        assert e2 <= e1 * (1 + 1e-12)


def test_kcycle_without_intermediate_levels_is_the_vcycle(orc):
    """With two levels there is no level between the finest and the coarsest,
    so the K-cycle applies no FCG and is the V-cycle."""
    A = inputs.laplacian7(8)  # 512 -> 64
    ho = orc.Hierarchy(A)
    assert ho.num_levels == 2
    r = np.random.default_rng(2).uniform(-1, 1, A.n)
    np.testing.assert_array_equal(ho.kcycle(r), ho.vcycle(r))


def test_kcycle_iterations_do_not_grow_with_the_grid(orc):
    """Section 3.1: with the piecewise-constant prolongator the V-cycle is not
    an optimal AMG, and the K-cycle is the remedy. V-cycle PCG iterations grow
    from 20^3 to 40^3; K-cycle FCG iterations stay flat and fewer."""
    its = {}
    for N in (20, 32, 40):
        c = inputs.small_case(N, seed=0)
        ho = orc.Hierarchy(c["A"])
        _, iv = ho.pcg(c["b"], rtol=1e-8, maxit=300)
        xk, ik = ho.fcg(c["b"], rtol=1e-8, maxit=300, cycle="K")
        assert ik["converged"] and ik["rel_res_true"] <= 1.001e-8
        its[N] = (iv["iterations"], ik["iterations"])
    assert its[40][0] >= its[20][0] + 5  # V-cycle grows
    assert its[40][1] <= its[20][1] + 2  # K-cycle does not
    assert all(k <= v - 3 for v, k in its.values())


def test_fcg_kcycle_solution_and_zero_rhs(orc):
    c = inputs.small_case(24, seed=1)
    A = c["A"]
    ho = orc.Hierarchy(A)
    Asp = sp.csr_matrix((A.val, A.col, A.row_ptr), shape=(A.n, A.n))
    x, info = ho.fcg(c["b"], rtol=1e-10, maxit=200, cycle="K")
    assert info["converged"]
    xs = sp.linalg.spsolve(Asp.tocsc(), c["b"])
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) < 1e-10 * 1e3
    x0, i0 = ho.fcg(np.zeros(A.n), x0=np.ones(A.n), cycle="K")
    assert i0["iterations"] == 0 and not x0.any()
