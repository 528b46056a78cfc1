"""Pins of the oracle's smooth vector w (the remark after eq. (prolongator):
a few iterations of an A-convergent smoother on an arbitrary sample vector).

The l1-Jacobi smoother is A-convergent (2M - A is s.p.d., Section 3.3), so
every sweep on A w = 0 lowers the energy (w, A w); the iterate equals the
dense power (I - M^-1 A)^nu w0 with M built from the l1 definition; and for
an M-matrix with non-negative row sums the ones vector stays in (0, 1] and
decays toward the boundary, where the Dirichlet rows are not in the kernel.
"""

import numpy as np
import pytest
import scipy.sparse as sp

from paper_2006_16147_amd import inputs


def _sp(A):
    return sp.csr_matrix((A.val, A.col, A.row_ptr), shape=(A.n, A.n))


def test_zero_sweeps_is_the_sample(orc):
    A = inputs.laplacian7(6)
    w0 = np.random.default_rng(0).uniform(0.5, 1.5, A.n)
    np.testing.assert_array_equal(orc.smooth_w(A, 0, w0), w0)


@pytest.mark.parametrize("case", ["poisson", "aniso"])
def test_every_sweep_lowers_the_energy(orc, case):
    if case == "poisson":
        A = inputs.laplacian7(12)
    else:
        ex, ey = inputs.block_log_uniform_eps(12, 4, np.random.default_rng(1))
        A = inputs.diffusion7(12, ex, ey, 1.0)
    S = _sp(A)
    w = np.random.default_rng(3).uniform(-1, 1, A.n)
    e_prev = w @ (S @ w)
    for nu in range(1, 9):
        w = orc.smooth_w(A, 1, w)
        e = w @ (S @ w)
        assert e < e_prev
        e_prev = e


def test_equals_the_dense_power_with_the_l1_diagonal(orc):
    A = inputs.laplacian7(6)
    D = _sp(A).toarray()
    m = np.abs(D).sum(axis=1)  # a_ii > 0, so a_ii + sum_{j != i} |a_ij|
    G = np.eye(A.n) - D / m[:, None]
    w0 = np.random.default_rng(5).uniform(-1, 1, A.n)
    for nu in (1, 3, 6):
        ref = np.linalg.matrix_power(G, nu) @ w0
        np.testing.assert_allclose(orc.smooth_w(A, nu, w0), ref, rtol=0, atol=1e-14)


def test_ones_stay_positive_and_decay_toward_the_boundary(orc):
    N = 10
    A = inputs.laplacian7(N)
    w = orc.smooth_w(A, 6)
    assert np.all(w > 0) and np.all(w <= 1.0)
    g = w.reshape(N, N, N)
    assert g[0, 0, 0] < g[1, 1, 1] < g[N // 2, N // 2, N // 2]
