"""GPU tests of the multi-right-hand-side solve (amg_pcg_solve_batch).

Each column runs its own CG recurrence; the V-cycle is applied to the whole
block. A column must match the single-vector solve of the same right-hand
side and, at equal iteration counts, the CPU oracle.
"""

import numpy as np
import pytest

from paper_2006_16147_amd import inputs

from gpu_helpers import setup, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def _batch(h, B, X0=None, rtol=1e-8, maxit=500):
    import torch

    from paper_2006_16147_amd import amg

    Bd = to_dev(np.ascontiguousarray(B))
    X = torch.zeros_like(Bd) if X0 is None else to_dev(np.ascontiguousarray(X0))
    st, infos = amg.amg_pcg_solve_batch(h, Bd, X, rtol=rtol, maxit=maxit, raise_on_error=False)
    return st, infos, X.cpu().numpy()


def _single(h, b, rtol=1e-8, maxit=500):
    import torch

    from paper_2006_16147_amd import amg

    bd = to_dev(b)
    x = torch.zeros_like(bd)
    st, info = amg.amg_pcg_solve(h, bd, x, rtol=rtol, maxit=maxit, raise_on_error=False)
    return st, info, x.cpu().numpy()


@pytest.mark.parametrize("k", [1, 5, 32])
def test_batch_columns_equal_single_solves_fp64(orc, k):
    A = inputs.laplacian7(16)
    B = np.random.default_rng(3).uniform(-1, 1, (A.n, k))
    h = setup(A)
    st, infos, X = _batch(h, B)
    assert st == 0 and all(i["converged"] for i in infos)
    kt, vshift = h.batch_tiles()
    assert kt in (4, 8, 16, 32, 64) and vshift in (-1, 0, 1)
    ho = orc.Hierarchy(A)
    for j in range(k):
        st1, i1, x1 = _single(h, B[:, j])
        assert abs(i1["iterations"] - infos[j]["iterations"]) <= 1
        assert np.linalg.norm(X[:, j] - x1) / np.linalg.norm(x1) < 1e-9
        xo, _ = ho.pcg(B[:, j], rtol=0.0, maxit=infos[j]["iterations"])
        assert np.linalg.norm(X[:, j] - xo) / np.linalg.norm(xo) < 1e-8
        assert infos[j]["rel_res_true"] <= 1.001e-8


def test_batch_fp32_hierarchy(orc):
    from paper_2006_16147_amd import amg

    A = inputs.laplacian7(24)
    k = 32
    B = np.random.default_rng(3).uniform(-1, 1, (A.n, k))
    h = setup(A, precision=amg.FP32)
    st, infos, X = _batch(h, B)
    assert st == 0
    ho = orc.Hierarchy(A)
    for j in (0, 7, 31):
        assert infos[j]["rel_res_true"] <= 1.01e-8
        xo, _ = ho.pcg(B[:, j], rtol=1e-12)
        assert np.linalg.norm(X[:, j] - xo) / np.linalg.norm(xo) < 1e-6
    # a column of the FP32 batch equals the FP32 single solve closely
    st1, i1, x1 = _single(h, B[:, 7])
    assert abs(i1["iterations"] - infos[7]["iterations"]) <= 1
    assert np.linalg.norm(X[:, 7] - x1) / np.linalg.norm(x1) < 1e-8


@pytest.mark.parametrize("k,precision", [(2, "fp64"), (6, "fp64"), (12, "fp64"), (130, "fp64"),
                                         (2, "fp32"), (6, "fp32"), (12, "fp32")])
def test_batch_vector_and_one_value_forms_agree(orc, k, precision):
    """The level-0 kernels move two FP64 or four FP32 columns per lane when k
    allows it. With k = 2 and 6 the FP32 hierarchy mixes the two-column FP64
    kernels (outer SpMV, CG update, p = z + b p) with the one-value forms of
    the FP32 ones; k = 12 takes the vector forms throughout. FP64 with
    k = 130 needs more than 64 two-column lanes per row, so the column
    reductions come from two blocks along the grid's second dimension.
    Every column matches its single solve and, at equal iterations, the
    oracle."""
    from paper_2006_16147_amd import amg

    A = inputs.laplacian7(16)
    B = np.random.default_rng(9 + k).uniform(-1, 1, (A.n, k))
    fp32 = precision == "fp32"
    h = setup(A, precision=amg.FP32 if fp32 else amg.FP64)
    st, infos, X = _batch(h, B)
    assert st == 0 and all(i["converged"] for i in infos)
    ho = orc.Hierarchy(A)
    for j in range(k):
        _, i1, x1 = _single(h, B[:, j])
        assert abs(i1["iterations"] - infos[j]["iterations"]) <= 1
        assert np.linalg.norm(X[:, j] - x1) / np.linalg.norm(x1) < (1e-8 if fp32 else 1e-9)
        assert infos[j]["rel_res_true"] <= (1.01e-8 if fp32 else 1.001e-8)
        if not fp32:
            xo, _ = ho.pcg(B[:, j], rtol=0.0, maxit=infos[j]["iterations"])
            assert np.linalg.norm(X[:, j] - xo) / np.linalg.norm(xo) < 1e-8


def test_batch_edge_cases(orc):
    import torch

    from paper_2006_16147_amd import amg

    A = inputs.laplacian7(10)
    h = setup(A, max_coarse=60)
    # k = 0 is a no-op
    L = amg.load_library()
    e = torch.zeros(1, dtype=torch.float64, device="cuda")
    assert L.amg_pcg_solve_batch(h.handle, 0, e.data_ptr(), e.data_ptr(), 1e-8, 10, None) == 0
    # a zero column stops at iteration 0 with x = 0; the others converge
    B = np.random.default_rng(0).uniform(-1, 1, (A.n, 3))
    B[:, 1] = 0.0
    st, infos, X = _batch(h, B, X0=np.ones((A.n, 3)))
    assert st == 0
    assert infos[1]["iterations"] == 0 and not X[:, 1].any()
    assert infos[0]["converged"] and infos[2]["converged"]
    # maxit reached on every column
    st, infos, X = _batch(h, B, rtol=0.0, maxit=2)
    assert st == amg.Status.NOT_CONVERGED
    assert infos[0]["iterations"] == 2 and infos[2]["iterations"] == 2
    ho = orc.Hierarchy(A, max_coarse=60)
    xo, _ = ho.pcg(B[:, 0], rtol=0.0, maxit=2)
    assert np.linalg.norm(X[:, 0] - xo) / np.linalg.norm(xo) < 1e-10


def test_batch_single_level_hierarchy():
    A = inputs.laplacian7(5)
    h = setup(A)
    B = np.random.default_rng(1).uniform(-1, 1, (A.n, 4))
    st, infos, X = _batch(h, B, rtol=1e-12)
    assert st == 0
    for j in range(4):
        assert infos[j]["iterations"] == 1
        np.testing.assert_allclose(A.to_dense() @ X[:, j], B[:, j], atol=1e-10)


def test_batch_deterministic():
    A = inputs.laplacian7(12)
    h = setup(A)
    B = np.random.default_rng(5).uniform(-1, 1, (A.n, 8))
    _, i1, X1 = _batch(h, B)
    _, i2, X2 = _batch(h, B)
    assert [i["iterations"] for i in i1] == [i["iterations"] for i in i2]
    np.testing.assert_array_equal(X1.view(np.uint64), X2.view(np.uint64))


@pytest.mark.parametrize("k", [6, 12])
@pytest.mark.parametrize("pre,post", [(2, 2), (3, 1), (1, 2)])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batch_extra_sweeps_match_single_and_oracle(orc, pre, post, precision, k):
    """The block V-cycle applies the hierarchy's pre/post sweep counts. With
    k = 12 an FP32 hierarchy takes the four-column down step before the
    one-value post-smoothing and residual kernels of the extra sweeps."""
    from paper_2006_16147_amd import amg

    A = inputs.laplacian7(20)
    B = np.random.default_rng(5).uniform(-1, 1, (A.n, k))
    prec = amg.FP32 if precision == "fp32" else amg.FP64
    h = setup(A, pre=pre, post=post, precision=prec)
    st, infos, X = _batch(h, B)
    assert st == 0 and all(i["converged"] for i in infos)
    ho = orc.Hierarchy(A)
    for j in range(k):
        _, i1, x1 = _single(h, B[:, j])
        assert abs(i1["iterations"] - infos[j]["iterations"]) <= 1
        assert np.linalg.norm(X[:, j] - x1) / np.linalg.norm(x1) < (1e-9 if prec == amg.FP64
                                                                   else 1e-6)
        if prec == amg.FP64:
            xo, _ = ho.pcg(B[:, j], rtol=0.0, maxit=infos[j]["iterations"], pre=pre, post=post)
            assert np.linalg.norm(X[:, j] - xo) / np.linalg.norm(xo) < 1e-8
