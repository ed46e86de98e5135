"""GPU parity of the s-step SRE-CG2 variant (every block A-orthonormalised
against all blocks since the last restart), of Pre-CholQR (a Euclidean
CholQR before the A-CholQR), both from the algorithms of Section 3.1, and
of s-step MSDO-CG (Section 3.2),
through the C ABI against the FP64 oracle.  Same bar as test_gpu_solve.py:
first iterates and basis to 1e-10, full solves with the iteration count
within +-2 and x within 1e-6 (ensemble criterion on rounding-sensitive
problems)."""
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


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _kw(E, variant, orth):
    return dict(variant=E.SRECG2 if variant == "srecg2" else E.SRECG,
                orth=E.PRECHOLQR if orth == "precholqr" else E.ACHOLQR)


@pytest.fixture(scope="module")
def poisson():
    p = P.poisson2d()
    return p, p.scipy(), O.partition_grid(p.shape, p.parts)


@pytest.mark.parametrize("variant,orth", [("srecg2", "acholqr"), ("srecg", "precholqr"),
                                          ("srecg2", "precholqr")])
def test_first_iterations_and_basis(E, poisson, variant, orth):
    # s = 2 and 5 iterations: blocks 1..10, so the SRE-CG2 chunks cover one,
    # two and three chunks of earlier blocks
    p, A, dom = poisson
    ref = O.sstep_srecg(A, dom, 8, 2, p.b, tol=1e-8, maxit=5, variant=variant, orth=orth,
                        record=True)
    sol = E.Solver(p.rowptr, p.colind, p.vals, dom, 8, 2, **_kw(E, variant, orth))
    for kmax in (1, 2, 3, 5):
        x, info = sol.solve(p.b, tol=1e-8, maxit=kmax)
        assert info.status == E.MAXIT and info.iters == kmax
        assert _rel(x.cpu().numpy(), ref.extra["xs"][kmax]) <= 1e-10, kmax
        V, AV = (a.cpu().numpy() for a in sol.basis())
        Vr, AVr = ref.extra["V"][kmax - 1]
        assert np.abs(V - Vr).max() <= 1e-10 * np.abs(Vr).max(), kmax
        assert np.abs(AV - AVr).max() <= 1e-10 * np.abs(AVr).max(), kmax
    sol.close()


@pytest.mark.parametrize("variant,orth", [("srecg2", "acholqr"), ("srecg", "precholqr"),
                                          ("srecg2", "precholqr")])
def test_full_solve_parity(E, poisson, variant, orth):
    p, A, dom = poisson
    ref = O.sstep_srecg(A, dom, 8, 2, p.b, tol=1e-8, variant=variant, orth=orth)
    sol = E.Solver(p.rowptr, p.colind, p.vals, dom, 8, 2, **_kw(E, variant, orth))
    x, info = sol.solve(p.b, tol=1e-8, maxit=1000)
    x = x.cpu().numpy()
    assert info.status == E.OK
    assert abs(info.iters - ref.iters) <= 2, (info.iters, ref.iters)
    assert info.true_relres <= 1e-8
    assert _rel(x, ref.x) <= 1e-6
    sol.close()


@pytest.mark.parametrize("m,t,s,parts", [
    (37, 3, 3, (3, 1, 1)), (41, 20, 2, (5, 4, 1)), (48, 32, 2, (4, 8, 1)), (64, 64, 2, (8, 8, 1)),
    (40, 8, 5, (2, 4, 1))])
def test_srecg2_shapes(E, m, t, s, parts):
    # block widths padded to 16, 32 and 64 columns (chunks of three and two
    # earlier blocks) and a ragged last work-group
    p = P.poisson2d(m, t=t, parts=parts, seed=m)
    A = p.scipy()
    dom = O.partition_grid(p.shape, parts)
    ref = O.sstep_srecg(A, dom, t, s, p.b, tol=1e-8, variant="srecg2", maxit=3, record=True)
    sol = E.Solver(p.rowptr, p.colind, p.vals, dom, t, s, variant=E.SRECG2)
    x, info = sol.solve(p.b, tol=1e-8, maxit=3)
    kk = info.iters
    assert kk == ref.iters
    assert _rel(x.cpu().numpy(), ref.extra["xs"][kk]) <= 1e-10
    full = O.sstep_srecg(A, dom, t, s, p.b, tol=1e-8, variant="srecg2")
    x, info = sol.solve(p.b, tol=1e-8, maxit=2000)
    assert info.status == E.OK and info.true_relres <= 1e-8
    assert abs(info.iters - full.iters) <= 2, (info.iters, full.iters)
    assert _rel(x.cpu().numpy(), full.x) <= 1e-6
    sol.close()


@pytest.mark.parametrize("cap", [2, 5, 9])
def test_srecg2_block_cap_restarts(E, poisson, cap):
    # a cap of q blocks: once another s blocks would exceed it, the solve
    # restarts from x with r = b - A x (the same rule in the oracle)
    p, A, dom = poisson
    ref = O.sstep_srecg(A, dom, 8, 2, p.b, tol=1e-8, maxit=30, variant="srecg2",
                        q_cap_blocks=cap, max_restarts=0)
    sol = E.Solver(p.rowptr, p.colind, p.vals, dom, 8, 2, variant=E.SRECG2, q_cap_blocks=cap,
                   max_restarts=0)
    x, info = sol.solve(p.b, tol=1e-8, maxit=30)
    assert ref.status == O.MAXIT and info.status == E.MAXIT
    assert info.iters == ref.iters == 30
    assert info.restarts == ref.restarts >= 1
    assert info.blocks == ref.blocks
    assert len(info.hist) == len(ref.hist)
    np.testing.assert_allclose(info.hist, ref.hist, rtol=1e-8)
    assert _rel(x.cpu().numpy(), ref.x) <= 1e-9
    sol.close()


def test_srecg2_block_cap_full_solve(E, poisson):
    p, A, dom = poisson
    ref = O.sstep_srecg(A, dom, 8, 2, p.b, tol=1e-8, variant="srecg2", q_cap_blocks=40)
    sol = E.Solver(p.rowptr, p.colind, p.vals, dom, 8, 2, variant=E.SRECG2, q_cap_blocks=40)
    x, info = sol.solve(p.b, tol=1e-8, maxit=1000)
    assert ref.status == O.OK and info.status == E.OK
    assert abs(info.iters - ref.iters) <= 2, (info.iters, ref.iters)
    assert abs(info.restarts - ref.restarts) <= 1
    assert info.true_relres <= 1e-8
    assert _rel(x.cpu().numpy(), ref.x) <= 1e-6
    sol.close()


def test_srecg2_heterogeneous_3d(E):
    # 16^3 skyscraper field: SRE-CG2 needs far fewer iterations than SRE-CG
    shape = (16, 16, 16)
    p = P.make_problem("sky", shape, P.kappa_skyscraper(shape, 2, tile=4), seed=2, t=16, s=4,
                       parts=(4, 4, 1))
    A = p.scipy()
    dom = O.partition_grid(shape, (4, 4, 1))
    runs = oracle_ensemble(A, dom, 16, 4, p.b, k=3, variant="srecg2")
    sol = E.Solver(p.rowptr, p.colind, p.vals, dom, 16, 4, variant=E.SRECG2)
    x, info = sol.solve(p.b, tol=1e-8, maxit=2000)
    assert info.status == E.OK and info.true_relres <= 1e-8
    print(check_parity(info.iters, x.cpu().numpy(), runs, A))
    sol.close()


def test_srecg2_breakdown_zero_domain(E, poisson):
    # b zero on one domain: T(r) has a zero column, A-CholQR meets a zero pivot
    p, A, dom = poisson
    b = p.b.copy()
    b[dom == 3] = 0.0
    sol = E.Solver(p.rowptr, p.colind, p.vals, dom, 8, 2, variant=E.SRECG2,
                   orth=E.PRECHOLQR)
    x, info = sol.solve(b, tol=1e-8, maxit=100)
    r = O.sstep_srecg(A, dom, 8, 2, b, tol=1e-8, maxit=100, variant="srecg2", orth="precholqr")
    assert r.status == O.BREAKDOWN
    assert info.status == E.BREAKDOWN and info.iters == r.iters == 0
    assert not x.cpu().numpy().any()      # x is the last completed iterate: x0
    sol.close()


def test_srecg2_mixed_precision(E, poisson):
    p, A, dom = poisson
    sol = E.Solver(p.rowptr, p.colind, p.vals, dom, 8, 2, variant=E.SRECG2,
                   precision=E.MIXED)
    x, info = sol.solve(p.b, tol=1e-8, maxit=1000)
    x = x.cpu().numpy()
    assert info.status == E.OK and info.restarts >= 1
    assert np.linalg.norm(p.b - A @ x) / np.linalg.norm(p.b) <= 1e-8
    ref = O.sstep_srecg(A, dom, 8, 2, p.b, tol=1e-8, variant="srecg2", basis_dtype=np.float32,
                        inner_tol=1e-4)
    assert abs(info.iters - ref.iters) <= max(2, ref.iters // 10), (info.iters, ref.iters)
    sol.close()


def test_srecg2_stats_classes(E, poisson):
    p, A, dom = poisson
    sol = E.Solver(p.rowptr, p.colind, p.vals, dom, 8, 2, variant=E.SRECG2, orth=E.PRECHOLQR,
                   collect_stats=True)
    x, info = sol.solve(p.b, tol=1e-8, maxit=6)
    st = sol.stats()
    assert st["gram"]["launches"] > 0 and st["update"]["launches"] > 0
    assert st["spmm"]["launches"] == info.blocks
    sol.close()


# ---------------------------------------------------------------------------
# s-step MSDO-CG (Section 3.2)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("s", [1, 2, 3])
def test_msdo_first_iterations_and_basis(E, poisson, s):
    # s = 1: every block is T(r_{k-1}); s = 2, 3: first blocks from T(r)
    # followed by SRE-CG2 blocks (one to three chunks of earlier blocks)
    p, A, dom = poisson
    ref = O.sstep_srecg(A, dom, 8, s, p.b, tol=1e-8, maxit=5, variant="msdo", record=True)
    sol = E.Solver(p.rowptr, p.colind, p.vals, dom, 8, s, variant=E.MSDO)
    for kmax in (1, 2, 3, 5):
        x, info = sol.solve(p.b, tol=1e-8, maxit=kmax)
        assert info.status == E.MAXIT and info.iters == kmax
        assert _rel(x.cpu().numpy(), ref.extra["xs"][kmax]) <= 1e-10, kmax
        V, AV = (a.cpu().numpy() for a in sol.basis())
        Vr, AVr = ref.extra["V"][kmax - 1]
        assert np.abs(V - Vr).max() <= 1e-10 * np.abs(Vr).max(), kmax
        assert np.abs(AV - AVr).max() <= 1e-10 * np.abs(AVr).max(), kmax
    sol.close()


@pytest.mark.parametrize("m,t,s,parts,orth", [
    (100, 8, 2, (2, 4, 1), "acholqr"), (100, 8, 2, (2, 4, 1), "precholqr"),
    (41, 20, 2, (5, 4, 1), "acholqr"), (64, 64, 1, (8, 8, 1), "acholqr")])
def test_msdo_full_solve_parity(E, m, t, s, parts, orth):
    p = P.poisson2d(m, t=t, parts=parts, seed=m + 1)
    A = p.scipy()
    dom = O.partition_grid(p.shape, parts)
    ref = O.sstep_srecg(A, dom, t, s, p.b, tol=1e-8, variant="msdo", orth=orth)
    sol = E.Solver(p.rowptr, p.colind, p.vals, dom, t, s, variant=E.MSDO,
                   orth=E.PRECHOLQR if orth == "precholqr" else E.ACHOLQR)
    x, info = sol.solve(p.b, tol=1e-8, maxit=2000)
    assert info.status == E.OK and info.true_relres <= 1e-8
    assert abs(info.iters - ref.iters) <= 2, (info.iters, ref.iters)
    assert _rel(x.cpu().numpy(), ref.x) <= 1e-6
    sol.close()


def test_msdo_block_cap_restarts(E, poisson):
    p, A, dom = poisson
    ref = O.sstep_srecg(A, dom, 8, 2, p.b, tol=1e-8, maxit=30, variant="msdo", q_cap_blocks=5,
                        max_restarts=0)
    sol = E.Solver(p.rowptr, p.colind, p.vals, dom, 8, 2, variant=E.MSDO, q_cap_blocks=5,
                   max_restarts=0)
    x, info = sol.solve(p.b, tol=1e-8, maxit=30)
    assert info.iters == ref.iters and info.restarts == ref.restarts >= 1
    assert len(info.hist) == len(ref.hist)
    np.testing.assert_allclose(info.hist, ref.hist, rtol=1e-8)
    assert _rel(x.cpu().numpy(), ref.x) <= 1e-9
    sol.close()


def test_msdo_mixed_precision(E, poisson):
    p, A, dom = poisson
    sol = E.Solver(p.rowptr, p.colind, p.vals, dom, 8, 2, variant=E.MSDO, precision=E.MIXED)
    x, info = sol.solve(p.b, tol=1e-8, maxit=1000)
    x = x.cpu().numpy()
    assert info.status == E.OK and info.restarts >= 1
    assert np.linalg.norm(p.b - A @ x) / np.linalg.norm(p.b) <= 1e-8
    sol.close()


@pytest.mark.parametrize("m,t,s,parts,variant,orth", [
    (48, 32, 2, (4, 8, 1), "srecg2", "acholqr"), (64, 64, 2, (8, 8, 1), "srecg2", "acholqr"),
    (64, 64, 1, (8, 8, 1), "msdo", "acholqr"), (64, 64, 2, (8, 8, 1), "srecg", "precholqr")])
def test_variants_mixed_wide_blocks(E, m, t, s, parts, variant, orth):
    # binary32 blocks of 32 and 64 columns through the Gram/update chunks,
    # the MSDO restart passes and the Pre-CholQR scaling (all on the matrix
    # cores at these widths)
    p = P.poisson2d(m, t=t, parts=parts, seed=m + 3)
    A = p.scipy()
    dom = O.partition_grid(p.shape, parts)
    var = {"srecg": E.SRECG, "srecg2": E.SRECG2, "msdo": E.MSDO}[variant]
    sol = E.Solver(p.rowptr, p.colind, p.vals, dom, t, s, variant=var, precision=E.MIXED,
                   orth=E.PRECHOLQR if orth == "precholqr" else E.ACHOLQR)
    x, info = sol.solve(p.b, tol=1e-8, maxit=2000)
    x = x.cpu().numpy()
    assert info.status == E.OK
    assert np.linalg.norm(p.b - A @ x) / np.linalg.norm(p.b) <= 1e-8
    ref = O.sstep_srecg(A, dom, t, s, p.b, tol=1e-8, variant=variant, orth=orth)
    assert _rel(x, ref.x) <= 1e-5
    m32 = O.sstep_srecg(A, dom, t, s, p.b, tol=1e-8, variant=variant, orth=orth,
                        basis_dtype=np.float32, inner_tol=1e-4)
    assert abs(info.iters - m32.iters) <= max(3, m32.iters // 10), (info.iters, m32.iters)
    sol.close()
