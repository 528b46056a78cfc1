"""Shared helpers of the GPU tests: device copies of inputs and a setup
wrapper. Imports torch lazily so CPU-only collection stays light."""

import numpy as np


def device():
    import torch

    return torch.device("cuda:0")


def to_dev(a, dtype=None):
    import torch

    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(device())


def setup(A, **params):
    from paper_2006_16147_amd import amg

    rp, ci, va = to_dev(A.row_ptr), to_dev(A.col), to_dev(A.val)
    return amg.amg_setup(rp, ci, va, **params)


def setup_status(A, w=None, **params):
    """Returns the amg_setup status code instead of raising."""
    from paper_2006_16147_amd import amg

    try:
        kw = dict(params)
        if w is not None:
            kw["w"] = to_dev(w)
        h = setup(A, **kw)
    except amg.AmgError as e:
        return e.status, None
    return amg.Status.OK, h


def solve(h, b, x0=None, rtol=1e-8, maxit=1000):
    import torch

    from paper_2006_16147_amd import amg

    bd = to_dev(b)
    x = torch.zeros_like(bd) if x0 is None else to_dev(np.array(x0, dtype=np.float64))
    st, info = amg.amg_pcg_solve(h, bd, x, rtol=rtol, maxit=maxit, raise_on_error=False)
    return st, info, x.cpu().numpy()


def assert_same_hierarchy(h, ho, values_exact=True):
    """Level sizes, sparsity, aggregates and prolongator bit-exact vs the oracle."""
    assert h.sizes() == ho.sizes(), (h.sizes(), ho.sizes())
    assert h.nnzs() == ho.nnzs(), (h.nnzs(), ho.nnzs())
    for l in range(ho.num_levels):
        rp, ci, val = h.level_csr(l)
        Ao = ho.level_csr(l)
        np.testing.assert_array_equal(rp, Ao.row_ptr)
        np.testing.assert_array_equal(ci, Ao.col)
        if values_exact:
            np.testing.assert_array_equal(val.view(np.uint64), Ao.val.view(np.uint64))
        np.testing.assert_array_equal(h.w(l).view(np.uint64), ho.w(l).view(np.uint64))
        if l < ho.num_levels - 1:
            agg, p = h.transfer(l)
            agg_o, p_o = ho.transfer(l)
            np.testing.assert_array_equal(agg, agg_o)
            np.testing.assert_array_equal(p.view(np.uint64), p_o.view(np.uint64))
            np.testing.assert_array_equal(h.l1diag(l).view(np.uint64),
                                          ho.l1diag(l).view(np.uint64))
