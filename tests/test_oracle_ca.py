"""Pins of the oracle's communication-avoiding forms (ca=True): CA SRE-CG,
CA SRE-CG2 and CA MSDO-CG with the modified CA-Arnoldi A-orthonormalization
(Section 4).  Each iteration A-orthonormalizes its first block W_j against
the kept blocks Q and itself, forms the monomial powers A W_j, ..,
A^{s-1} W_j, and A-orthonormalizes all s t vectors against Q and then
against themselves as one block.

Pinned by: the exact-arithmetic identity with the s-step methods (for
SRE-CG and SRE-CG2 the CA basis spans the same enlarged Krylov subspace, so
the iterates agree up to rounding; Section 3.1 derives why (s+1) t kept
vectors suffice), the paper's Tables 2-4 Poisson2D counts for the CA
columns (soft band), t = s = 1 is CG, dense solves, A-orthonormality of the
whole basis, the Petrov-Galerkin condition, the A-norm error-drop identity,
the split residuals lying in the CA MSDO-CG basis, and planted mistakes."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
import oracle.ecg_oracle as E
import problems as P
from tests import pinlib

PARTS = {2: (2, 1, 1), 4: (2, 2, 1), 8: (2, 4, 1), 16: (4, 4, 1), 32: (4, 8, 1), 64: (8, 8, 1)}


def _band(got, want):
    # geometric box domains and another generator for x, not Metis k-way
    # domains and MATLAB's rand: the same soft band as for the s-step rows
    return abs(got - want) <= max(2, 0.10 * want)


def _rand_spd(n, seed, cond):
    rng = np.random.default_rng(seed)
    Qm, _ = np.linalg.qr(rng.standard_normal((n, n)))
    return (Qm * np.geomspace(1.0, cond, n)) @ Qm.T


@pytest.fixture(scope="module")
def p30():
    p = P.poisson2d(30, t=4, parts=(2, 2, 1), seed=3)
    return p, p.scipy(), O.partition_grid(p.shape, (2, 2, 1))


def _rel_iterate_gap(a, b, upto):
    xa, xb = a.extra["xs"], b.extra["xs"]
    n = min(len(xa), len(xb), upto + 1)
    return max(np.linalg.norm(xa[i] - xb[i]) / np.linalg.norm(xa[i]) for i in range(1, n))


@pytest.mark.parametrize("variant,s", [("srecg", 2), ("srecg", 3), ("srecg2", 2),
                                       ("srecg2", 3), ("msdo", 1), ("msdo", 2)])
def test_ca_iterates_equal_sstep(p30, variant, s):
    # Same subspace after every iteration, hence the same A-norm-optimal
    # iterate in exact arithmetic (MSDO-CG: only up to s = 2, since its
    # s-step form multiplies orthonormalized blocks that are not powers of
    # one block)
    p, A, dom = p30
    a = O.sstep_srecg(A, dom, 4, s, p.b, tol=1e-8, variant=variant, record=True)
    b = O.sstep_srecg(A, dom, 4, s, p.b, tol=1e-8, variant=variant, record=True, ca=True)
    assert a.status == b.status == O.OK
    assert a.iters == b.iters
    assert _rel_iterate_gap(a, b, 6) <= 1e-10


@pytest.mark.parametrize("table,variant,t,svals", [
    ("ca-sre-cg", "srecg", 2, (2, 3, 4)), ("ca-sre-cg", "srecg", 16, (2, 4)),
    ("ca-sre-cg2", "srecg2", 8, (2, 4)),
    ("ca-msdo", "msdo", 4, (2, 3, 5)), ("ca-msdo", "msdo", 16, (2, 7))])
def test_ca_poisson_tables(table, variant, t, svals):
    p = P.poisson2d(rhs="unit", tol=1e-6)
    A = p.scipy()
    dom = O.partition_grid(p.shape, PARTS[t])
    row = pinlib.read_ca_table()[(table, t)]
    for s in svals:
        want = row[pinlib.CA_SVALS.index(s)]
        got = O.sstep_srecg(A, dom, t, s, p.b, tol=1e-6, variant=variant, ca=True).iters
        assert _band(got, want), (table, t, s, got, want)


@pytest.mark.parametrize("variant,s", [("srecg", 2), ("srecg", 3), ("srecg2", 3)])
def test_plain_ca_iterates_equal_modified(p30, variant, s):
    # the CA-Arnoldi of Section 3.1 (powers of the raw block) spans the same
    # space as the modified one for SRE-CG and SRE-CG2: equal iterates in
    # exact arithmetic
    p, A, dom = p30
    a = O.sstep_srecg(A, dom, 4, s, p.b, tol=1e-8, variant=variant, record=True, ca=True)
    b = O.sstep_srecg(A, dom, 4, s, p.b, tol=1e-8, variant=variant, record=True, ca="plain")
    assert a.status == b.status == O.OK
    assert a.iters == b.iters
    assert _rel_iterate_gap(a, b, 6) <= 1e-10


@pytest.mark.parametrize("t,svals", [(4, (2, 3, 5)), (16, (2, 5))])
def test_plain_ca_msdo_poisson_table4(t, svals):
    p = P.poisson2d(rhs="unit", tol=1e-6)
    A = p.scipy()
    dom = O.partition_grid(p.shape, PARTS[t])
    row = pinlib.read_ca_table()[("ca5-msdo", t)]
    for s in svals:
        want = row[pinlib.CA_SVALS.index(s)]
        got = O.sstep_srecg(A, dom, t, s, p.b, tol=1e-6, variant="msdo", ca="plain").iters
        assert _band(got, want), (t, s, got, want)


def test_plain_ca_basis_properties():
    p = P.poisson2d(40, t=8, parts=(2, 4, 1), seed=12)
    A = p.scipy()
    dom = O.partition_grid(p.shape, p.parts)
    for variant in ("srecg", "msdo"):
        r = O.sstep_srecg(A, dom, 8, 3, p.b, tol=1e-8, maxit=5, variant=variant, ca="plain",
                          record=True)
        assert pinlib.orthonormality_violation(r, A) <= 1e-10
        assert _whole_basis_violation(r, A) <= 1e-8
        assert pinlib.petrov_galerkin_violation(r) <= 1e-10
        assert pinlib.error_drop_violation(r, A, p.xstar) <= 1e-8


@pytest.mark.parametrize("variant", ["srecg", "srecg2", "msdo"])
def test_ca_t1_s1_is_cg(variant):
    p = P.poisson2d(20, t=1, parts=(1, 1, 1), seed=4)
    A = p.scipy()
    dom = np.zeros(p.n, dtype=np.int32)
    cg = O.cg(A, p.b, tol=1e-10, record=True)
    ca = O.sstep_srecg(A, dom, 1, 1, p.b, tol=1e-10, variant=variant, ca=True, record=True)
    assert ca.iters == cg.iters
    for k in (1, 5, 20):
        xc, xa = cg.extra["xs"][k], ca.extra["xs"][k]
        assert np.linalg.norm(xa - xc) <= 1e-10 * np.linalg.norm(xc)


@pytest.mark.parametrize("variant", ["srecg", "srecg2", "msdo"])
@pytest.mark.parametrize("t,s", [(2, 2), (4, 3), (3, 2)])
def test_ca_matches_dense_solve(variant, t, s):
    A = sp.csr_matrix(_rand_spd(48, 7, cond=50.0))
    xs = np.random.default_rng(8).standard_normal(48)
    dom = O.partition_grid((48, 1, 1), (t, 1, 1))
    r = O.sstep_srecg(A, dom, t, s, A @ xs, tol=1e-12, maxit=200, variant=variant, ca=True)
    assert r.status == O.OK
    assert np.linalg.norm(r.x - xs) / np.linalg.norm(xs) < 1e-9


def _whole_basis_violation(res, A):
    Q = np.hstack([V for V, _ in res.extra["V"]])
    G = Q.T @ (A @ Q)
    return float(np.abs(G - np.eye(G.shape[0])).max())


@pytest.mark.parametrize("variant", ["srecg", "srecg2", "msdo"])
def test_ca_basis_properties(variant):
    p = P.poisson2d(40, t=8, parts=(2, 4, 1), seed=12)
    A = p.scipy()
    dom = O.partition_grid(p.shape, p.parts)
    r = O.sstep_srecg(A, dom, 8, 3, p.b, tol=1e-8, maxit=5, variant=variant, ca=True,
                      record=True)
    assert pinlib.orthonormality_violation(r, A) <= 1e-10
    assert pinlib.cross_block_violation(r, A) <= 1e-9
    # SRE-CG keeps (s+1) t vectors; in exact arithmetic that keeps V_k
    # A-orthogonal to every earlier block (Section 3.1), which five
    # iterations on a small Poisson problem show to ~1e-9
    assert _whole_basis_violation(r, A) <= 1e-8
    assert pinlib.petrov_galerkin_violation(r) <= 1e-10
    assert pinlib.error_drop_violation(r, A, p.xstar) <= 1e-8


def test_ca_msdo_basis_spans_split_residuals():
    # every iteration's first block is T(r_{k-1}) A-orthonormalized against
    # the kept blocks, so each split residual lies in the basis
    p = P.poisson2d(30, t=4, parts=(2, 2, 1), seed=11)
    A = p.scipy()
    dom = O.partition_grid(p.shape, p.parts)
    for s in (2, 3):
        r = O.sstep_srecg(A, dom, 4, s, p.b, tol=1e-10, maxit=3, variant="msdo", ca=True,
                          record=True)
        Q = np.hstack([V for V, _ in r.extra["V"]])
        B = np.hstack([O.split_T(r.extra["rs"][i], dom, 4) for i in range(3)])
        coef, *_ = np.linalg.lstsq(Q, B, rcond=None)
        assert np.linalg.norm(Q @ coef - B) / np.linalg.norm(B) <= 1e-10, s


def test_ca_first_block_breakdown():
    # b zero on one domain and x0 = 0: T(r_0) has a zero column, the first
    # A-CholQR breaks down, and no iteration is done
    p = P.poisson2d(12, t=3, parts=(3, 1, 1), seed=2)
    A = p.scipy()
    dom = O.partition_grid(p.shape, (3, 1, 1))
    b = p.b.copy()
    b[dom == 1] = 0.0
    r = O.sstep_srecg(A, dom, 3, 2, b, tol=1e-8, ca=True)
    assert r.status == O.BREAKDOWN and r.iters == 0


# ---------------------------------------------------------------------------
# Planted mistakes (in the oracle, on the CPU)
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def p40():
    p = P.poisson2d(40, t=8, parts=(2, 4, 1), seed=12)
    return p, p.scipy(), O.partition_grid(p.shape, p.parts)


def _ca_run(p40, **kw):
    p, A, dom = p40
    return O.sstep_srecg(A, dom, 8, 3, p.b, tol=1e-8, maxit=5, ca=True, record=True, **kw)


def test_planted_no_projection_of_powers_is_caught(p40, monkeypatch):
    # V = [W_j, A W_j, ..] not A-orthonormalized against Q
    p, A, _ = p40
    good = _ca_run(p40)
    real = E.cgs2_a

    def skip_wide(Z, Wp, AWp, dtype=np.float64):
        return Z if Z.shape[1] > 8 else real(Z, Wp, AWp, dtype)

    monkeypatch.setattr(E, "cgs2_a", skip_wide)
    bad = _ca_run(p40)
    assert pinlib.cross_block_violation(good, A) <= 1e-9
    assert pinlib.cross_block_violation(bad, A) > 1e-4


def test_planted_q_of_one_block_is_caught(p40, monkeypatch):
    # Q = the last block only: with W_j A-orthonormal to the earlier blocks,
    # A^i W_j has components along blocks j-i .. j-1, so at s = 3 one kept
    # block is too few (the paper keeps s + 1, more than the s - 1 the
    # modified CA-Arnoldi needs in exact arithmetic)
    p, A, _ = p40
    good = _ca_run(p40)
    real = E._BlockStore

    class Short(real):
        def __init__(self, n, dtype, keep_last=None):
            super().__init__(n, dtype, None if keep_last is None else 1)

    monkeypatch.setattr(E, "_BlockStore", Short)
    bad = _ca_run(p40)
    assert _whole_basis_violation(good, A) <= 1e-8
    assert _whole_basis_violation(bad, A) > 1e-5


def test_planted_blockwise_cholqr_of_v_is_caught(p40, monkeypatch):
    # A-CholQR of each t-column block of V on its own (no cross terms)
    p, A, _ = p40
    real = E.a_cholqr

    def blockwise(Ab, Z, dtype=np.float64, trace=None):
        if Z.shape[1] <= 8:
            return real(Ab, Z, dtype, trace)
        parts = [real(Ab, Z[:, i:i + 8], dtype) for i in range(0, Z.shape[1], 8)]
        return (np.hstack([q[0] for q in parts]), np.hstack([q[1] for q in parts]), None)

    monkeypatch.setattr(E, "a_cholqr", blockwise)
    bad = _ca_run(p40)
    assert pinlib.orthonormality_violation(bad, A) > 1e-3
