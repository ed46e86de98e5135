"""GPU solve parity through the C ABI against the FP64 oracle.

Tolerances (spec contract): domain partitions and T(r) bit-exact
(test_gpu_kernels.py); FP64 solutions with true relative residual <= 1e-8,
||x - x_oracle|| / ||x_oracle|| <= 1e-6 and iteration counts within +-2 --
on problems whose iteration is itself sensitive to rounding, relative to
that sensitivity (tests/parity.py).
Iterates of the first s-step iterations agree to 1e-10 (the two sides round
differently: the device keeps each block unnormalised and folds R^{-1} into
small coefficient matrices).
"""
import numpy as np
import pytest

import oracle as O
import problems as P
from tests.parity import check_parity, oracle_ensemble

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def E():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    import paper_1804_10629_amd as E
    return E


def _setup(E, p, t, s, parts, **kw):
    dom = O.partition_grid(p.shape, parts)
    return E.Solver(p.rowptr, p.colind, p.vals, dom, t, s, **kw), dom


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def c1(E):
    p = P.poisson2d()
    A = p.scipy()
    sol, dom = _setup(E, p, 8, 2, p.parts)
    ref = O.sstep_srecg(A, dom, 8, 2, p.b, tol=1e-8, record=True)
    return p, A, dom, sol, ref


def test_c1_full_solve_parity(E, c1):
    p, A, dom, sol, ref = c1
    x, info = sol.solve(p.b, tol=1e-8, maxit=1000)
    x = x.cpu().numpy()
    assert info.status == E.OK
    assert abs(info.iters - ref.iters) <= 2
    assert info.true_relres <= 1e-8
    assert np.linalg.norm(p.b - A @ x) / np.linalg.norm(p.b) <= 1e-8
    assert _rel(x, ref.x) <= 1e-6
    assert abs(info.rho0 - ref.hist[0]) <= 1e-14 * ref.hist[0]
    k = min(len(info.hist), len(ref.hist))
    # recursive residual histories agree while far above rounding level
    for a, b in zip(info.hist[:k], ref.hist[:k]):
        if b > 1e-6 * ref.hist[0]:
            assert abs(a - b) <= 1e-8 * b


@pytest.mark.parametrize("kmax", [1, 2, 3, 8])
def test_c1_first_iterations(E, c1, kmax):
    p, A, dom, sol, ref = c1
    x, info = sol.solve(p.b, tol=1e-8, maxit=kmax)
    assert info.status == E.MAXIT and info.iters == kmax
    assert _rel(x.cpu().numpy(), ref.extra["xs"][kmax]) <= 1e-10
    V, AV = (a.cpu().numpy() for a in sol.basis())
    Vr, AVr = ref.extra["V"][kmax - 1]
    assert np.abs(V - Vr).max() <= 1e-10 * np.abs(Vr).max()
    assert np.abs(AV - AVr).max() <= 1e-10 * np.abs(AVr).max()
    G = V.T @ (A @ V)
    assert np.abs(G - np.eye(G.shape[0])).max() <= 1e-10


@pytest.mark.parametrize("m,t,s,parts", [
    (30, 1, 1, (1, 1, 1)), (30, 1, 3, (1, 1, 1)), (37, 3, 2, (3, 1, 1)), (40, 8, 1, (2, 4, 1)),
    (40, 8, 5, (2, 4, 1)), (45, 16, 3, (4, 4, 1)), (41, 20, 2, (5, 4, 1)), (48, 32, 2, (4, 8, 1)),
    (64, 64, 2, (8, 8, 1))])
def test_solve_parity_shapes(E, m, t, s, parts):
    p = P.poisson2d(m, t=t, parts=parts, seed=m)
    A = p.scipy()
    sol, dom = _setup(E, p, t, s, parts)
    ref = O.sstep_srecg(A, dom, t, s, p.b, tol=1e-8)
    x, info = sol.solve(p.b, tol=1e-8, maxit=2000)
    x = x.cpu().numpy()
    assert info.status == E.OK
    assert abs(info.iters - ref.iters) <= 2
    assert info.true_relres <= 1e-8
    assert _rel(x, ref.x) <= 1e-6


def test_t1_s1_is_cg(E):
    p = P.poisson2d(50, t=1, parts=(1, 1, 1), seed=7)
    A = p.scipy()
    sol, _ = _setup(E, p, 1, 1, (1, 1, 1))
    x, info = sol.solve(p.b, tol=1e-8, maxit=5000)
    c = O.cg(A, p.b, tol=1e-8)
    assert info.status == E.OK and abs(info.iters - c.iters) <= 2
    assert _rel(x.cpu().numpy(), c.x) <= 1e-6


def test_heterogeneous_3d_parity(E):
    shape = (24, 24, 24)
    p = P.make_problem("sky", shape, P.kappa_skyscraper(shape, 2, tile=4), seed=2, t=16, s=4,
                       parts=(4, 4, 1))
    A = p.scipy()
    sol, dom = _setup(E, p, 16, 4, (4, 4, 1))
    runs = oracle_ensemble(A, dom, 16, 4, p.b)
    x, info = sol.solve(p.b, tol=1e-8, maxit=2000)
    assert info.status == E.OK and info.true_relres <= 1e-8
    print(check_parity(info.iters, x.cpu().numpy(), runs, A))


def test_bitwise_reproducible(E, c1):
    p, A, dom, sol, ref = c1
    x1, i1 = sol.solve(p.b, tol=1e-8, maxit=1000)
    x2, i2 = sol.solve(p.b, tol=1e-8, maxit=1000)
    assert i1.iters == i2.iters
    assert np.array_equal(x1.cpu().numpy(), x2.cpu().numpy())
    assert np.array_equal(i1.hist, i2.hist)


def test_x0_warm_start(E, c1):
    p, A, dom, sol, ref = c1
    x0 = ref.extra["xs"][5]
    x, info = sol.solve(p.b, x0=x0, tol=1e-8, maxit=1000)
    r2 = O.sstep_srecg(A, dom, 8, 2, p.b, x0=x0, tol=1e-8)
    assert info.status == E.OK and abs(info.iters - r2.iters) <= 2
    assert abs(info.rho0 - r2.hist[0]) <= 1e-12 * r2.hist[0]


def test_zero_rhs(E, c1):
    p, A, dom, sol, ref = c1
    x, info = sol.solve(np.zeros(p.n), tol=1e-8)
    assert info.status == E.OK and info.iters == 0 and not x.cpu().numpy().any()


def test_breakdown_zero_domain(E, c1):
    p, A, dom, sol, ref = c1
    b = p.b.copy()
    b[dom == 3] = 0.0
    x, info = sol.solve(b, tol=1e-8, maxit=100)
    r = O.sstep_srecg(A, dom, 8, 2, b, tol=1e-8, maxit=100)
    assert r.status == O.BREAKDOWN
    assert info.status == E.BREAKDOWN and info.iters == r.iters == 0
    assert not x.cpu().numpy().any()      # x is the last completed iterate: x0


def test_breakdown_indefinite(E):
    p = P.poisson2d(20, t=2, parts=(2, 1, 1))
    vals = p.vals.copy()
    diag = np.repeat(np.arange(p.n), np.diff(p.rowptr)) == p.colind
    vals[np.nonzero(diag)[0][:50]] *= -1.0
    dom = O.partition_grid(p.shape, p.parts)
    sol = E.Solver(p.rowptr, p.colind, vals, dom, 2, 2)
    r = O.sstep_srecg(O.csr(p.rowptr, p.colind, vals), dom, 2, 2, p.b, tol=1e-8, maxit=100)
    x, info = sol.solve(p.b, tol=1e-8, maxit=100)
    assert r.status == O.BREAKDOWN and info.status == E.BREAKDOWN
    assert abs(info.iters - r.iters) <= 2


def test_invalid_solve_arguments(E, c1):
    p, A, dom, sol, ref = c1
    b = p.b.copy()
    b[7] = np.nan
    with pytest.raises(E.EcgError):
        sol.solve(b)
    with pytest.raises(E.EcgError):
        sol.solve(p.b, tol=0.0)
    with pytest.raises(E.EcgError):
        sol.solve(p.b, maxit=-1)


def test_mixed_precision_reaches_tolerance(E, c1):
    p, A, dom, _, ref = c1
    sol, _ = _setup(E, p, 8, 2, p.parts, precision=E.MIXED)
    x, info = sol.solve(p.b, tol=1e-8, maxit=2000)
    x = x.cpu().numpy()
    assert info.status == E.OK and info.restarts >= 1
    assert np.linalg.norm(p.b - A @ x) / np.linalg.norm(p.b) <= 1e-8
    # error against the FP64 oracle: both solutions satisfy the 1e-8
    # residual, so they agree to about cond(A) * 1e-8
    assert _rel(x, ref.x) <= 1e-5
    m32 = O.sstep_srecg(A, dom, 8, 2, p.b, tol=1e-8, basis_dtype=np.float32, inner_tol=1e-4)
    assert abs(info.iters - m32.iters) <= max(3, 0.1 * m32.iters)


def test_stats_account_every_kernel(E):
    p = P.poisson2d(60, t=8, parts=(2, 4, 1))
    sol, _ = _setup(E, p, 8, 3, (2, 4, 1), collect_stats=True)
    x, info = sol.solve(p.b, tol=1e-8, maxit=500)
    st = sol.stats()
    assert st["spmm"]["launches"] == info.blocks
    assert st["xr_update"]["launches"] == info.iters or info.status != E.OK
    assert all(v["ms"] >= 0 for v in st.values())
    assert st["spmm"]["ms"] > 0 and st["cgs_gram"]["ms"] > 0


@pytest.mark.parametrize("m,t,s,parts", [(48, 32, 2, (4, 8, 1)), (64, 64, 2, (8, 8, 1))])
def test_mixed_precision_wide_blocks(E, m, t, s, parts):
    # binary32 blocks of 32 and 64 stored columns (the 64-column updates run
    # on the matrix cores)
    p = P.poisson2d(m, t=t, parts=parts, seed=m)
    A = p.scipy()
    sol, dom = _setup(E, p, t, s, parts, precision=E.MIXED)
    x, info = sol.solve(p.b, tol=1e-8, maxit=2000)
    x = x.cpu().numpy()
    assert info.status == E.OK
    assert np.linalg.norm(p.b - A @ x) / np.linalg.norm(p.b) <= 1e-8
    ref = O.sstep_srecg(A, dom, t, s, p.b, tol=1e-8)
    assert _rel(x, ref.x) <= 1e-5
    m32 = O.sstep_srecg(A, dom, t, s, p.b, tol=1e-8, basis_dtype=np.float32, inner_tol=1e-4)
    assert abs(info.iters - m32.iters) <= max(3, 0.1 * m32.iters)


@pytest.mark.parametrize("m,t,s,parts", [(40, 8, 3, (2, 4, 1)), (48, 32, 2, (4, 8, 1)),
                                         (64, 64, 2, (8, 8, 1))])
@pytest.mark.parametrize("grid", [1, 7, 2048])
def test_custom_grid_matches_default(E, m, t, s, parts, grid):
    # launch grids that are not a multiple of the 8 XCDs (plain striding),
    # a single work-group, and more work-groups than the default: the same
    # iterates up to the order of the work-group sums
    p = P.poisson2d(m, t=t, parts=parts, seed=m + 5)
    A = p.scipy()
    ref, _ = _setup(E, p, t, s, parts)
    xr, ir = ref.solve(p.b, tol=1e-8, maxit=2000)
    sol, _ = _setup(E, p, t, s, parts, grid=grid)
    x, info = sol.solve(p.b, tol=1e-8, maxit=2000)
    assert info.status == E.OK and abs(info.iters - ir.iters) <= 1
    assert _rel(x.cpu().numpy(), xr.cpu().numpy()) <= 1e-9
    assert np.linalg.norm(p.b - A @ x.cpu().numpy()) / np.linalg.norm(p.b) <= 1e-8
    ref.close()
    sol.close()


def test_long_rows_64_columns(E):
    # rows of 13 entries (the square of the 5-point Laplacian, SPD): at 64
    # columns the general product kernel runs (the producer/consumer form
    # takes rows of at most 7 entries); parity with the oracle on every
    # iterate
    p = P.poisson2d(24, t=64, parts=(8, 8, 1))
    L = p.scipy()
    A = (L @ L).tocsr()
    A.sort_indices()
    assert np.diff(A.indptr).max() == 13
    b = A @ p.xstar
    dom = O.partition_grid(p.shape, (8, 8, 1))
    sol = E.Solver(A.indptr.astype(np.int32), A.indices.astype(np.int32), A.data, dom, 64, 2)
    ref = O.sstep_srecg(A, dom, 64, 2, b, tol=1e-8, maxit=100, record=True)
    x, info = sol.solve(b, tol=1e-8, maxit=100)
    assert info.status == E.OK and info.iters == ref.iters
    assert _rel(x.cpu().numpy(), ref.x) <= 1e-8
    x1, _ = sol.solve(b, tol=1e-8, maxit=1)
    assert _rel(x1.cpu().numpy(), ref.extra["xs"][1]) <= 1e-10
    sol.close()
