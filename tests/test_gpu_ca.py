"""GPU parity of the CA forms (opts.ca = 1: CA SRE-CG, CA SRE-CG2, CA
MSDO-CG with the modified CA-Arnoldi A-orthonormalization of Section 4)
through the C ABI against the float64 oracle (sstep_srecg(..., ca=True)).

The GPU A-orthonormalizes the s t columns block by block (each power
against the kept blocks and the iteration's earlier blocks with CGS2, then
A-CholQR); the oracle does CGS2 of all s t columns against the kept blocks
and one A-CholQR of them.  The two are equal in exact arithmetic (the
A-orthonormal factor with an upper triangular right factor is unique) and
differ in rounding, so first iterates and bases are compared to 1e-9 and
full solves with the usual bar: counts within 2 and x within 1e-6, or the
ensemble criterion on rounding-sensitive problems."""
import numpy as np
import pytest

import oracle as O
import problems as P
from tests.parity import check_parity, oracle_ensemble

pytestmark = pytest.mark.gpu

VARIANTS = ("srecg", "srecg2", "msdo")


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


def _v(E, variant):
    return {"srecg": E.SRECG, "srecg2": E.SRECG2, "msdo": E.MSDO}[variant]


@pytest.fixture(scope="module")
def poisson():
    p = P.poisson2d()
    return p, p.scipy(), O.partition_grid(p.shape, p.parts)


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("s", [2, 3])
def test_ca_first_iterations_and_basis(E, poisson, variant, s):
    p, A, dom = poisson
    ref = O.sstep_srecg(A, dom, 8, s, p.b, tol=1e-8, maxit=4, variant=variant, ca=True,
                        record=True)
    sol = E.Solver(p.rowptr, p.colind, p.vals, dom, 8, s, variant=_v(E, variant), ca=True)
    for kmax in (1, 2, 4):
        x, info = sol.solve(p.b, tol=1e-8, maxit=kmax)
        assert info.status == E.MAXIT and info.iters == kmax
        assert info.blocks == kmax * s
        assert _rel(x.cpu().numpy(), ref.extra["xs"][kmax]) <= 1e-9, kmax
        V, AV = (a.cpu().numpy() for a in sol.basis())
        Vr, AVr = ref.extra["V"][kmax - 1]
        assert np.abs(V - Vr).max() <= 1e-9 * np.abs(Vr).max(), kmax
        assert np.abs(AV - AVr).max() <= 1e-9 * np.abs(AVr).max(), kmax
    sol.close()


@pytest.mark.parametrize("variant,s,orth", [
    ("srecg", 2, "acholqr"), ("srecg", 4, "acholqr"), ("srecg2", 3, "acholqr"),
    ("msdo", 3, "acholqr"), ("srecg", 3, "precholqr"), ("msdo", 2, "precholqr")])
def test_ca_full_solve_parity(E, poisson, variant, s, orth):
    p, A, dom = poisson
    ref = O.sstep_srecg(A, dom, 8, s, p.b, tol=1e-8, variant=variant, orth=orth, ca=True)
    sol = E.Solver(p.rowptr, p.colind, p.vals, dom, 8, s, variant=_v(E, variant), ca=True,
                   orth=E.PRECHOLQR if orth == "precholqr" else E.ACHOLQR)
    x, info = sol.solve(p.b, tol=1e-8, maxit=1000)
    assert ref.status == O.OK and info.status == E.OK
    assert abs(info.iters - ref.iters) <= 2, (info.iters, ref.iters)
    assert info.true_relres <= 1e-8
    assert _rel(x.cpu().numpy(), ref.x) <= 1e-6
    sol.close()


@pytest.mark.parametrize("m,t,s,parts,variant", [
    (37, 3, 3, (3, 1, 1), "srecg"), (41, 20, 2, (5, 4, 1), "srecg2"),
    (48, 32, 2, (4, 8, 1), "srecg"), (64, 64, 2, (8, 8, 1), "srecg"),
    (40, 8, 5, (2, 4, 1), "msdo")])
def test_ca_shapes(E, m, t, s, parts, variant):
    # widths padded to 16, 32 and 64 columns and a ragged last work-group
    p = P.poisson2d(m, t=t, parts=parts, seed=m)
    A = p.scipy()
    dom = O.partition_grid(p.shape, parts)
    ref = O.sstep_srecg(A, dom, t, s, p.b, tol=1e-8, variant=variant, ca=True, maxit=2,
                        record=True)
    sol = E.Solver(p.rowptr, p.colind, p.vals, dom, t, s, variant=_v(E, variant), ca=True)
    x, info = sol.solve(p.b, tol=1e-8, maxit=2)
    assert info.iters == ref.iters
    assert _rel(x.cpu().numpy(), ref.extra["xs"][info.iters]) <= 1e-9
    full = O.sstep_srecg(A, dom, t, s, p.b, tol=1e-8, variant=variant, ca=True)
    x, info = sol.solve(p.b, tol=1e-8, maxit=2000)
    assert info.status == E.OK and info.true_relres <= 1e-8
    assert abs(info.iters - full.iters) <= 2, (info.iters, full.iters)
    assert _rel(x.cpu().numpy(), full.x) <= 1e-6
    sol.close()


@pytest.mark.parametrize("variant,s", [("srecg2", 2), ("msdo", 3)])
def test_ca_heterogeneous_3d(E, variant, s):
    # 16^3 skyscraper field; ensemble criterion.  (CA SRE-CG2 at s = 3
    # is unstable here, as the paper finds for its skyscraper matrices with
    # growing s: its oracle ensemble spreads over 31 .. 57 iterations, so
    # no parity criterion applies)
    shape = (16, 16, 16)
    p = P.make_problem("sky", shape, P.kappa_skyscraper(shape, 2, tile=4), seed=2, t=16, s=s,
                       parts=(4, 4, 1))
    A = p.scipy()
    dom = O.partition_grid(shape, (4, 4, 1))
    runs = oracle_ensemble(A, dom, 16, s, p.b, k=3, variant=variant, ca=True)
    sol = E.Solver(p.rowptr, p.colind, p.vals, dom, 16, s, variant=_v(E, variant), ca=True)
    x, info = sol.solve(p.b, tol=1e-8, maxit=2000)
    assert info.status == E.OK and info.true_relres <= 1e-8
    print(check_parity(info.iters, x.cpu().numpy(), runs, A))
    sol.close()


@pytest.mark.parametrize("cap", [4, 9])
def test_ca_block_cap_restarts(E, poisson, cap):
    p, A, dom = poisson
    ref = O.sstep_srecg(A, dom, 8, 2, p.b, tol=1e-8, maxit=20, variant="srecg2", ca=True,
                        q_cap_blocks=cap, max_restarts=0)
    sol = E.Solver(p.rowptr, p.colind, p.vals, dom, 8, 2, variant=E.SRECG2, ca=True,
                   q_cap_blocks=cap, max_restarts=0)
    x, info = sol.solve(p.b, tol=1e-8, maxit=20)
    assert ref.status == O.MAXIT and info.status == E.MAXIT
    assert info.iters == ref.iters == 20
    assert info.restarts == ref.restarts >= 1
    assert info.blocks == ref.blocks
    np.testing.assert_allclose(info.hist, ref.hist, rtol=1e-8)
    assert _rel(x.cpu().numpy(), ref.x) <= 1e-9
    sol.close()


@pytest.mark.parametrize("variant", VARIANTS)
def test_ca_breakdown_zero_domain(E, poisson, variant):
    p, A, dom = poisson
    b = p.b.copy()
    b[dom == 3] = 0.0
    sol = E.Solver(p.rowptr, p.colind, p.vals, dom, 8, 2, variant=_v(E, variant), ca=True)
    x, info = sol.solve(b, tol=1e-8, maxit=100)
    r = O.sstep_srecg(A, dom, 8, 2, b, tol=1e-8, maxit=100, variant=variant, ca=True)
    assert r.status == O.BREAKDOWN
    assert info.status == E.BREAKDOWN and info.iters == r.iters == 0
    assert not x.cpu().numpy().any()
    sol.close()


@pytest.mark.parametrize("variant", ["srecg", "msdo"])
def test_ca_mixed_precision(E, poisson, variant):
    p, A, dom = poisson
    sol = E.Solver(p.rowptr, p.colind, p.vals, dom, 8, 2, variant=_v(E, variant), ca=True,
                   precision=E.MIXED)
    x, info = sol.solve(p.b, tol=1e-8, maxit=1000)
    x = x.cpu().numpy()
    assert info.status == E.OK and info.restarts >= 1
    assert np.linalg.norm(p.b - A @ x) / np.linalg.norm(p.b) <= 1e-8
    ref = O.sstep_srecg(A, dom, 8, 2, p.b, tol=1e-8, variant=variant, ca=True,
                        basis_dtype=np.float32, inner_tol=1e-4)
    assert abs(info.iters - ref.iters) <= max(2, ref.iters // 10), (info.iters, ref.iters)
    sol.close()


@pytest.mark.parametrize("variant,s", [("srecg", 3), ("srecg2", 2), ("msdo", 3)])
def test_ca_preconditioned(E, variant, s):
    # block Jacobi IC(0) (Section 5): every raw block multiplied by M^{-1}
    p = P.poisson2d(60, t=16, parts=(4, 4, 1))
    A = p.scipy()
    dom = O.partition_grid(p.shape, (4, 4, 1))
    blk = O.partition_grid(p.shape, (8, 8, 1))
    M = O.apply_llt_inverse(O.block_jacobi_ic0(A, blk))
    ref = O.sstep_srecg(A, dom, 16, s, p.b, tol=1e-8, maxit=500, variant=variant, ca=True,
                        precond=M, record=True)
    sol = E.Solver(p.rowptr, p.colind, p.vals, dom, 16, s, variant=_v(E, variant), ca=True,
                   precond_blocks=blk)
    x, info = sol.solve(p.b, tol=1e-8, maxit=500)
    assert info.status == E.OK and info.true_relres <= 1e-8
    assert abs(info.iters - ref.iters) <= 2, (info.iters, ref.iters)
    assert _rel(x.cpu().numpy(), ref.x) <= 1e-6
    x1, _ = sol.solve(p.b, tol=1e-8, maxit=1)
    assert _rel(x1.cpu().numpy(), ref.extra["xs"][1]) <= 1e-9
    sol.close()


def test_ca_bitwise_reproducible(E, poisson):
    p, A, dom = poisson
    sol = E.Solver(p.rowptr, p.colind, p.vals, dom, 8, 3, variant=E.SRECG, ca=True)
    x1, i1 = sol.solve(p.b, tol=1e-8, maxit=1000)
    x2, i2 = sol.solve(p.b, tol=1e-8, maxit=1000)
    assert i1.iters == i2.iters
    assert np.array_equal(x1.cpu().numpy(), x2.cpu().numpy())
    sol.close()


@pytest.mark.parametrize("variant,s", [("srecg", 2), ("srecg2", 3), ("msdo", 2), ("msdo", 3)])
def test_plain_ca_parity(E, poisson, variant, s):
    # the CA-Arnoldi of Section 3.1 (ca = 2): first iterates and full solve
    p, A, dom = poisson
    ref = O.sstep_srecg(A, dom, 8, s, p.b, tol=1e-8, variant=variant, ca="plain", record=True)
    sol = E.Solver(p.rowptr, p.colind, p.vals, dom, 8, s, variant=_v(E, variant), ca=E.CA_PLAIN)
    for kmax in (1, 3):
        x, info = sol.solve(p.b, tol=1e-8, maxit=kmax)
        assert info.iters == kmax
        assert _rel(x.cpu().numpy(), ref.extra["xs"][kmax]) <= 1e-9, kmax
    x, info = sol.solve(p.b, tol=1e-8, maxit=1000)
    assert ref.status == O.OK and info.status == E.OK
    assert abs(info.iters - ref.iters) <= 2, (info.iters, ref.iters)
    assert info.true_relres <= 1e-8
    assert _rel(x.cpu().numpy(), ref.x) <= 1e-6
    sol.close()


def test_ca_first_iteration_breakdown_ends_the_solve(E, poisson):
    # b zero on one domain: T(r) has a zero column, the first block breaks
    # down; in the plain form the zero column reaches the powers too
    p, A, dom = poisson
    b = p.b.copy()
    b[dom == 5] = 0.0
    for ca, oca in ((E.CA_MODIFIED, True), (E.CA_PLAIN, "plain")):
        sol = E.Solver(p.rowptr, p.colind, p.vals, dom, 8, 3, ca=ca)
        x, info = sol.solve(b, tol=1e-8, maxit=100)
        r = O.sstep_srecg(A, dom, 8, 3, b, tol=1e-8, maxit=100, ca=oca)
        assert r.status == O.BREAKDOWN and info.status == E.BREAKDOWN
        assert info.iters == r.iters == 0 and info.restarts == r.restarts == 0
        sol.close()
