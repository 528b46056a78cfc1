"""Input generators: structure of the operators and equality of the numpy
and torch (device) builders."""

import numpy as np
import torch

from paper_2006_16147_amd import inputs


def test_laplacian_structure():
    A = inputs.laplacian7(6)
    assert A.n == 216 and A.nnz == 7 * 216 - 6 * 36
    d = A.to_dense()
    assert np.array_equal(d, d.T) and np.all(np.diag(d) == 6.0)
    rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr))
    for r in range(A.n):  # strictly ascending columns, diagonal present
        c = A.col[A.row_ptr[r]:A.row_ptr[r + 1]]
        assert np.all(np.diff(c) > 0) and r in c
    assert rows.shape[0] == A.nnz


def test_torch_diffusion_generator_matches_numpy():
    ex, ey, b = inputs.aniso_blocks_coefficients(16, 8, seed=2)
    A = inputs.diffusion7(16, ex, ey, 1.0)
    rp, ci, va = inputs.diffusion7_torch(16, torch.from_numpy(ex), torch.from_numpy(ey), 1.0,
                                         "cpu")
    assert np.array_equal(A.row_ptr, rp.numpy()) and np.array_equal(A.col, ci.numpy())
    assert np.array_equal(A.val.view(np.uint64), va.numpy().view(np.uint64))
    assert np.array_equal(inputs.aniso_blocks_case(16, 8, seed=2)["b"], b)


def test_constant_generator_matches_laplacian():
    L = inputs.laplacian7(7)
    for xp in (np, torch):
        rp, ci, va = inputs.constant_diffusion7_arrays(7, 1.0, 1.0, 1.0, xp, device="cpu")
        rp, ci, va = [np.asarray(a) for a in (rp, ci, va)]
        assert np.array_equal(L.row_ptr, rp) and np.array_equal(L.col, ci)
        assert np.array_equal(L.val, va)


def test_headline_rhs_is_a_times_u():
    c = inputs.headline_case(8, seed=1)
    np.testing.assert_allclose(c["b"], c["A"].to_dense() @ c["u"], rtol=1e-14, atol=1e-14)
    u = np.random.default_rng(1).uniform(-1, 1, 512)
    assert np.array_equal(c["u"], u)
