"""Pins of the oracle's smoothed aggregation (the alternative to the K-cycle
in Section 3.2): Pbar = (I - omega D^-1 A) P with omega = 4 / (3 ||D^-1 A||_inf),
and the Galerkin product Pbar^T A Pbar. (The choice of omega is pinned to the
supplement's smoothed-prolongator convergence constant in
test_oracle_paper_pins.py.)

Each pin uses an independent computation: dense NumPy products from the
definitions, SciPy sparse products on the oracle's own aggregates, the
pairwise product (a different code path) for an unsmoothed P, the dense
two-level error-propagation operator, closed-form values for the Poisson
matrix, and the paper's claim that the smoothed prolongator makes the
V-cycle iteration count flat.
"""

import numpy as np
import pytest
import scipy.sparse as sp

from paper_2006_16147_amd import inputs


def _sp(A, ncols=None):
    return sp.csr_matrix((A.val, A.col, A.row_ptr), shape=(A.n, ncols or A.n))


def _rect(rp, ci, val, ncols):
    return sp.csr_matrix((val, ci, rp), shape=(len(rp) - 1, ncols))


def _cases():
    rng = np.random.default_rng(1)
    return {"poisson12": inputs.laplacian7(12),
            "aniso12": inputs.diffusion7(12, *inputs.block_log_uniform_eps(12, 4, rng), 1.0),
            "random": inputs.random_spd_graph(700, 6.0, seed=2)}


@pytest.mark.parametrize("case", ["poisson12", "aniso12", "random"])
def test_omega_is_four_thirds_over_the_inf_norm_of_the_scaled_matrix(orc, case):
    A = _cases()[case]
    D = _sp(A).toarray()
    ref = 4.0 / (3.0 * np.max(np.abs(D).sum(axis=1) / np.diag(D)))
    assert orc.smoothing_omega(A) == pytest.approx(ref, rel=1e-15)


def test_omega_closed_form_for_the_poisson_matrix(orc):
    # interior rows: (6 + 6) / 6 = 2, so omega = 4 / 6 = 2/3 (correctly rounded)
    assert orc.smoothing_omega(inputs.laplacian7(10)) == 4.0 / 6.0


@pytest.mark.parametrize("case", ["poisson12", "aniso12", "random"])
def test_pbar_is_the_dense_formula(orc, case):
    A = _cases()[case]
    ho = orc.Hierarchy(A, smooth=True)
    assert ho.ok, ho.status
    nc = ho.level_n(1)
    agg, p = ho.transfer(0)
    P = np.zeros((A.n, nc))
    P[np.arange(A.n), agg] = p
    D = _sp(A).toarray()
    om = ho.omega(0)
    assert om == orc.smoothing_omega(A)
    ref = P - om * ((D / np.diag(D)[:, None]) @ P)
    Pb = _rect(*ho.pbar(0), nc)
    np.testing.assert_allclose(Pb.toarray(), ref, rtol=0, atol=1e-14 * np.abs(ref).max())
    # one entry per aggregate reached from the row: the pattern of |A| |P|
    pat = ((np.abs(D) > 0).astype(int) @ (P != 0).astype(int)) > 0
    rp, ci, _ = ho.pbar(0)
    assert np.array_equal(np.diff(rp), pat.sum(axis=1))
    for i in range(A.n):
        assert np.array_equal(ci[rp[i]:rp[i + 1]], np.flatnonzero(pat[i]))


@pytest.mark.parametrize("case", ["poisson12", "aniso12", "random"])
def test_galerkin_with_pbar_is_the_dense_product(orc, case):
    A = _cases()[case]
    ho = orc.Hierarchy(A, smooth=True)
    assert ho.ok, ho.status
    nc = ho.level_n(1)
    Pb = _rect(*ho.pbar(0), nc).toarray()
    ref = Pb.T @ _sp(A).toarray() @ Pb
    Ac = ho.level_csr(1)
    S = _sp(Ac)
    np.testing.assert_allclose(S.toarray(), ref, rtol=0, atol=1e-13 * np.abs(ref).max())
    # bitwise symmetric, and the pattern of Pbar^T |A| Pbar
    assert (S != S.T).nnz == 0
    pat = ((Pb != 0).T.astype(int) @ (np.abs(_sp(A).toarray()) > 0).astype(int)
           @ (Pb != 0).astype(int)) > 0
    assert np.array_equal(np.diff(Ac.row_ptr), pat.sum(axis=1))
    assert np.all(np.linalg.eigvalsh(S.toarray()) > 0)


def test_general_product_with_a_pairwise_p_is_the_pairwise_product(orc):
    """With the (unsmoothed) prolongator of one pairwise sweep, the general
    Galerkin product is the pairwise one up to the order of its sums."""
    A = inputs.laplacian7(9)
    lo, hi, c = orc.edge_weights(A)
    mate, _ = orc.greedy_matching(A.n, lo, hi, c)
    agg, nc = orc.number_aggregates(mate)
    p = orc.pairwise_prolongator(mate, np.ones(A.n))
    P = (np.arange(A.n + 1, dtype=np.int32), agg.astype(np.int32), p)
    G = orc.galerkin_general(A, P, nc)
    Q = orc.galerkin_pairwise(A, agg, p, nc)
    assert np.array_equal(G.row_ptr, Q.row_ptr) and np.array_equal(G.col, Q.col)
    np.testing.assert_allclose(G.val, Q.val, rtol=1e-15, atol=1e-15)


def test_every_level_matches_scipy_products_on_the_same_aggregates(orc):
    A = inputs.laplacian7(16)
    ho = orc.Hierarchy(A, smooth=True)
    assert ho.ok, ho.status
    S = _sp(A)
    for l in range(ho.num_levels - 1):
        nc = ho.level_n(l + 1)
        agg, p = ho.transfer(l)
        P = sp.csr_matrix((p, (np.arange(len(agg)), agg)), shape=(len(agg), nc))
        d = S.diagonal()
        om = 4.0 / (3.0 * np.max(abs(S).sum(axis=1).A.ravel() / d))
        Pb = (P - om * (sp.diags(1.0 / d) @ S @ P)).tocsr()
        S = (Pb.T @ S @ Pb).tocsr()
        assert S.nnz == ho.level_nnz(l + 1)
        Ao = _sp(ho.level_csr(l + 1))
        assert abs(Ao - S).max() <= 1e-12 * abs(S).max()
    assert ho.sizes() == [4096, 512, 68]


def test_two_level_vcycle_is_the_error_propagation_product(orc):
    A = inputs.laplacian7(8)
    ho = orc.Hierarchy(A, smooth=True, max_coarse=100)
    assert ho.ok and ho.num_levels == 2
    nc = ho.level_n(1)
    D = _sp(A).toarray()
    Pb = _rect(*ho.pbar(0), nc).toarray()
    Ac = _sp(ho.level_csr(1)).toarray()
    Minv = np.diag(1.0 / orc.l1_diag(A))
    n = A.n
    I = np.eye(n)
    S = I - Minv @ D
    C = I - Pb @ np.linalg.solve(Ac, Pb.T @ D)
    B = (I - S @ C @ S) @ np.linalg.inv(D)  # pre, coarse correction, post
    r = np.random.default_rng(0).uniform(-1, 1, n)
    np.testing.assert_allclose(ho.vcycle(r), B @ r, rtol=0, atol=1e-12 * np.abs(B @ r).max())


def test_smoothed_prolongator_makes_the_vcycle_iterations_flat(orc):
    """Section 3.2: with the piecewise-constant P the V-cycle is not optimal;
    the smoothed P keeps a single V-cycle and fixes that: its PCG iteration
    count stays flat from 16^3 to 40^3 and is well below the unsmoothed one."""
    its = {}
    for N in (16, 24, 40):
        c = inputs.small_case(N, seed=0)
        _, iu = orc.Hierarchy(c["A"]).pcg(c["b"], rtol=1e-8, maxit=300)
        _, isv = orc.Hierarchy(c["A"], smooth=True).pcg(c["b"], rtol=1e-8, maxit=300)
        assert isv["converged"] and isv["rel_res_true"] <= 1.001e-8
        its[N] = (iu["iterations"], isv["iterations"])
    assert its[40][1] <= its[16][1] + 2
    assert its[40][0] >= its[16][0] + 5
    assert all(s <= u - 5 for u, s in its.values()), its


def test_paper_gpu_preconditioner_needs_about_seven_iterations(orc):
    """Section 5's GPU preconditioner (smoothed prolongator from 3 sweeps of
    matching, 4 l1-Jacobi pre/post sweeps) needs 7 FCG iterations to 1e-6 on
    one GPU; the oracle's V-cycle with the exact coarsest solve needs 7-8 on
    24^3 and 40^3 grids."""
    for N in (24, 40):
        c = inputs.small_case(N, seed=0)
        _, info = orc.Hierarchy(c["A"], smooth=True).pcg(c["b"], rtol=1e-6, maxit=100, pre=4,
                                                          post=4)
        assert info["converged"] and 6 <= info["iterations"] <= 9, (N, info)
