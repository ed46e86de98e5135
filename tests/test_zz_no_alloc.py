"""ecg_spmm_noalloc (the entry point that allocates no device memory) through
the C ABI, against ecg_spmm on the same inputs: the same kernels, so the two
must agree bit for bit, and both within the rounding bound of A X.  Two calls
in a row on one GPU, the second with a smaller input, in device-pointer and
host-pointer mode, and the size limit."""
import ctypes

import numpy as np
import pytest

import oracle as O
import problems as P

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def E():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    import paper_1804_10629_amd as E
    return E


def _bound(A, X):
    return 8 * np.finfo(float).eps * (abs(A) @ np.abs(X)) + 1e-300


def _noalloc_dev(E, sol, X):
    import torch
    Xd = torch.as_tensor(X).cuda().contiguous()
    out = torch.full_like(Xd, float("nan"))
    sol.spmm_noalloc(Xd, out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("permute", [True, False])
def test_noalloc_matches_spmm_device_ptrs(E, permute):
    # first call: n x 64 = 4,096,000 staging entries, just under the limit
    big = P.make_problem("rb", (40, 40, 40), P.kappa_random_blocks((40, 40, 40), 5, block=4),
                         seed=7, t=1, s=1, parts=(1, 1, 1))
    assert big.n * 64 <= E.SPMM_NOALLOC_MAX
    dom = O.partition_grid(big.shape, (2, 2, 2))
    sol = E.Solver(big.rowptr, big.colind, big.vals, dom, 8, 2, permute_domains=permute)
    A = big.scipy()
    for k, seed in ((64, 1), (5, 2)):      # the second call has a smaller input
        X = np.random.default_rng(seed).standard_normal((big.n, k))
        Y0 = sol.spmm(X).cpu().numpy()
        Y1 = _noalloc_dev(E, sol, X)
        assert np.array_equal(Y1, Y0), f"k={k}"
        assert (np.abs(Y1 - A @ X) <= _bound(A, X)).all(), f"k={k}"
    # a smaller problem on a second context shares the same array
    small = P.poisson2d(30, t=4, parts=(2, 2, 1))
    dom2 = O.partition_grid(small.shape, (2, 2, 1))
    sol2 = E.Solver(small.rowptr, small.colind, small.vals, dom2, 4, 2, permute_domains=permute)
    X = np.random.default_rng(3).standard_normal((small.n, 17))
    Y0 = sol2.spmm(X).cpu().numpy()
    Y1 = _noalloc_dev(E, sol2, X)
    assert np.array_equal(Y1, Y0)
    A2 = small.scipy()
    assert (np.abs(Y1 - A2 @ X) <= _bound(A2, X)).all()


def _raw_ctx(E, p, dom, t, s):
    o = E._Opts()
    E.lib.ecg_opts_default(ctypes.byref(o))
    o.device_ptrs = 0
    ctx = ctypes.c_void_p()
    args = [np.ascontiguousarray(a) for a in (p.rowptr, p.colind, p.vals, dom)]
    code = E.lib.ecg_setup(ctypes.byref(ctx), p.n, *(a.ctypes.data for a in args), t, s,
                           ctypes.byref(o))
    assert code == 0, E.lib.ecg_last_error().decode()
    return ctx


def test_noalloc_matches_spmm_host_ptrs(E):
    p = P.make_problem("rb", (23, 19, 7), P.kappa_random_blocks((23, 19, 7), 5, block=4),
                       seed=5, t=1, s=1, parts=(1, 1, 1))   # n = 3059: ragged tail
    dom = O.partition_grid(p.shape, (2, 2, 1))
    ctx = _raw_ctx(E, p, dom, 4, 2)
    A = p.scipy()
    try:
        for k, seed in ((33, 4), (16, 5)):     # padded widths 64, then 16
            X = np.ascontiguousarray(np.random.default_rng(seed).standard_normal((p.n, k)))
            Y0 = np.full_like(X, np.nan)
            Y1 = np.full_like(X, np.nan)
            assert E.lib.ecg_spmm(ctx, X.ctypes.data, Y0.ctypes.data, k) == 0
            assert E.lib.ecg_spmm_noalloc(ctx, X.ctypes.data, Y1.ctypes.data, k) == 0, \
                E.lib.ecg_last_error().decode()
            assert np.array_equal(Y1, Y0), f"k={k}"
            assert (np.abs(Y1 - A @ X) <= _bound(A, X)).all(), f"k={k}"
    finally:
        E.lib.ecg_destroy(ctx)


def test_noalloc_rejects_beyond_limit(E):
    # n = 70,000: n x 64 exceeds the limit, n x 16 fits
    p = P.make_problem("rb", (70, 100, 10), P.kappa_random_blocks((70, 100, 10), 3, block=4),
                       seed=9, t=1, s=1, parts=(1, 1, 1))
    assert p.n * 64 > E.SPMM_NOALLOC_MAX >= p.n * 16
    dom = O.partition_grid(p.shape, (2, 1, 1))
    ctx = _raw_ctx(E, p, dom, 2, 2)
    try:
        X = np.ascontiguousarray(np.random.default_rng(6).standard_normal((p.n, 40)))
        Y = np.full_like(X, np.nan)
        assert E.lib.ecg_spmm_noalloc(ctx, X.ctypes.data, Y.ctypes.data, 40) == E.EINVAL
        assert "ECG_SPMM_NOALLOC_MAX" in E.lib.ecg_last_error().decode()
        assert np.isnan(Y).all()                 # rejected before any work
        X16 = np.ascontiguousarray(X[:, :16])
        Y16 = np.full_like(X16, np.nan)
        assert E.lib.ecg_spmm_noalloc(ctx, X16.ctypes.data, Y16.ctypes.data, 16) == 0
        A = p.scipy()
        assert (np.abs(Y16 - A @ X16) <= _bound(A, X16)).all()
        assert E.lib.ecg_spmm_noalloc(ctx, X.ctypes.data, Y.ctypes.data, 0) == E.EINVAL
        assert E.lib.ecg_spmm_noalloc(None, X.ctypes.data, Y.ctypes.data, 4) == E.EINVAL
    finally:
        E.lib.ecg_destroy(ctx)
