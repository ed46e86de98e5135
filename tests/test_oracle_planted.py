"""Planted mistakes: each plausible error in the oracle must fail a pin.

A mistake is planted in the oracle (on the CPU, by replacing one of its
functions for the duration of a test) and the test asserts that at least
one of the pins of tests/pinlib.py, or the paper's Poisson2D counts, now
reports a violation.  The unmodified oracle passing the same pins is
checked in test_oracle_pins.py.
"""
import numpy as np
import pytest

import oracle as O
import oracle.ecg_oracle as E
import problems as P
from tests import pinlib


@pytest.fixture(scope="module")
def c1():
    p = P.poisson2d()
    return p, p.scipy(), O.partition_grid(p.shape, p.parts)


def _run(c1, s=3, maxit=25, **kw):
    p, A, dom = c1
    return O.sstep_srecg(A, dom, 8, s, p.b, tol=1e-8, maxit=maxit, record=True, **kw)


def _pins(c1, res):
    p, A, _ = c1
    return {
        "orth": pinlib.orthonormality_violation(res, A) > 1e-10,
        "cross": pinlib.cross_block_violation(res, A) > 1e-10,
        "pg": pinlib.petrov_galerkin_violation(res) > 1e-10,
        "drop": pinlib.error_drop_violation(res, A, p.xstar) > 1e-8,
    }


def test_clean_oracle_passes(c1):
    assert not any(_pins(c1, _run(c1)).values())


def test_single_gram_schmidt_pass_is_caught(c1, monkeypatch):
    # CGS instead of CGS2: one pass leaves O(eps * growth) components along
    # earlier blocks; on a skyscraper-like problem it shows in orthogonality
    shape = (24, 24, 1)
    p = P.make_problem("sky", shape, P.kappa_skyscraper(shape, 2, tile=4, high=1e5),
                       seed=2, t=4, s=4, parts=(2, 2, 1))
    A = p.scipy()
    dom = O.partition_grid(shape, (2, 2, 1))

    def cgs1(Z, Wp, AWp, dtype=np.float64):
        if Wp is None or Wp.shape[1] == 0:
            return Z
        return Z - Wp @ (AWp.T @ Z)

    good = O.sstep_srecg(A, dom, 4, 4, p.b, tol=1e-8, maxit=30, record=True)
    monkeypatch.setattr(E, "cgs2_a", cgs1)
    bad = O.sstep_srecg(A, dom, 4, 4, p.b, tol=1e-8, maxit=30, record=True)
    assert pinlib.orthonormality_violation(bad, A) > 10 * pinlib.orthonormality_violation(good, A)


def test_dropped_older_block_is_caught(c1, monkeypatch):
    # orthogonalizing W_j against W_{j-1} only (not W_{j-2})
    orig = E.cgs2_a

    def last_block_only(Z, Wp, AWp, dtype=np.float64):
        if Wp is not None and Wp.shape[1] > Z.shape[1]:
            Wp, AWp = Wp[:, -Z.shape[1]:], AWp[:, -Z.shape[1]:]
        return orig(Z, Wp, AWp, dtype)

    monkeypatch.setattr(E, "cgs2_a", last_block_only)
    r = _pins(c1, _run(c1))
    assert r["orth"] or r["cross"]


def test_transposed_projection_is_caught(c1, monkeypatch):
    def transposed(Z, Wp, AWp, dtype=np.float64):
        if Wp is None or Wp.shape[1] == 0:
            return Z
        for _ in range(2):
            H = AWp.T @ Z
            Z = Z - Wp @ (H.T if H.shape[0] == H.shape[1] else H[:, ::-1])
        return Z

    monkeypatch.setattr(E, "cgs2_a", transposed)
    r = _pins(c1, _run(c1))
    assert r["orth"] or r["cross"]


# the planted mistake makes the blocks grow until they overflow: the
# overflow warnings are part of what it does
@pytest.mark.filterwarnings("ignore::RuntimeWarning")
def test_unscaled_a_image_is_caught(c1, monkeypatch):
    # returning A Z instead of (A Z) R^{-1} as the A-image of W
    orig = E.a_cholqr

    def bad(Ab, Z, dtype=np.float64):
        W, AW, R = orig(Ab, Z, dtype)
        return W, Ab @ Z, R

    monkeypatch.setattr(E, "a_cholqr", bad)
    r = _pins(c1, _run(c1))
    assert r["pg"] or r["drop"]


def test_wrong_residual_sign_is_caught(c1, monkeypatch):
    # r_k = r_{k-1} + A V alpha: plant it by negating the stored A-images
    orig = E.a_cholqr

    def neg(Ab, Z, dtype=np.float64):
        W, AW, R = orig(Ab, Z, dtype)
        return W, -AW, R

    monkeypatch.setattr(E, "a_cholqr", neg)
    r = _pins(c1, _run(c1))
    assert r["pg"] or r["drop"] or r["orth"]


def test_split_into_wrong_domains_is_caught(c1):
    p, _, dom = c1
    r = np.random.default_rng(0).standard_normal(p.n)
    Z = O.split_T(r, (dom + 1) % 8, 8)                 # planted: shifted domain index
    col_ok = all(np.array_equal(np.nonzero(Z[:, d])[0], np.nonzero(dom == d)[0])
                 for d in range(8))
    assert np.array_equal(Z.sum(axis=1), r)            # this pin alone would miss it
    assert not col_ok                                   # the column-support pin catches it


def test_cholesky_index_slip_is_caught():
    rng = np.random.default_rng(3)
    Q, _ = np.linalg.qr(rng.standard_normal((6, 6)))
    G = (Q * np.geomspace(1, 100, 6)) @ Q.T

    def slipped(Gm):
        t = Gm.shape[0]
        R = np.zeros_like(Gm)
        for j in range(t):
            R[j, j] = np.sqrt(Gm[j, j] - R[:j, j] @ R[:j, j])
            for c in range(j + 1, t):
                R[j, c] = (Gm[j, c] - R[:j, j] @ R[:j, c]) / R[j, j] if j else Gm[j, c]
        return R

    with np.errstate(invalid="ignore"):
        R = slipped(G)
    assert not (np.abs(R.T @ R - G).max() <= 1e-12 * np.abs(G).max())
    Rg = O.chol_upper(G)
    assert np.abs(Rg.T @ Rg - G).max() <= 1e-12 * np.abs(G).max()


def test_skipped_second_block_update_changes_iteration_count(c1, monkeypatch):
    # updating x with the first block of V only (s-step update truncated):
    # the Poisson2D count leaves the paper's band
    p = P.poisson2d(rhs="unit", tol=1e-6)
    A = p.scipy()
    dom = O.partition_grid(p.shape, (2, 4, 1))
    orig_hstack = np.hstack

    def first_block_only(blocks, *a, **k):
        return orig_hstack(blocks[:1], *a, **k)

    monkeypatch.setattr(E.np, "hstack", first_block_only)
    try:
        it = O.sstep_srecg(A, dom, 8, 4, p.b, tol=1e-6, maxit=200).iters
    finally:
        monkeypatch.setattr(E.np, "hstack", orig_hstack)
    want = pinlib.read_poisson_table()[("sre-cg", 8)][pinlib.SVALS.index(4)]
    assert abs(it - want) > max(2, 0.10 * want)


# ---------------------------------------------------------------------------
# The binary32-basis precision form: each plausible slip fails a pin
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def lu_small():
    shape = (30, 30, 1)
    p = P.make_problem("lu", shape, P.kappa_loguniform(shape, 4, -2, 2), seed=4, t=4, s=2,
                       parts=(2, 2, 1))
    return p, p.scipy(), O.partition_grid(shape, (2, 2, 1))


def _mixed(lu_small, maxit=6, tol=1e-8):
    p, A, dom = lu_small
    trace = []
    r = O.sstep_srecg(A, dom, 4, 2, p.b, tol=tol, maxit=maxit, basis_dtype=np.float32,
                      inner_tol=1e-5, trace=trace)
    return r, trace


def _a32(lu_small):
    return lu_small[1].toarray().astype(np.float32).astype(np.float64)


def test_clean_binary32_form_passes(lu_small):
    r, trace = _mixed(lu_small)
    assert pinlib.binary32_representability_violation(trace) == 0
    assert pinlib.basis_product_rounding_violation(trace, _a32(lu_small)) <= 0.5 + 1e-6
    assert pinlib.gram_accuracy_violation(trace) <= 1.0


def test_unrounded_cgs_output_is_caught(lu_small, monkeypatch):
    # CGS2 result left in binary64 instead of stored as a binary32 block
    def cgs2_no_round(Z, Wp, AWp, dtype=np.float64):
        if Wp is None or Wp.shape[1] == 0:
            return Z
        Z = np.asarray(Z, dtype=np.float64)
        for _ in range(2):
            Z = Z - np.asarray(Wp, np.float64) @ (np.asarray(AWp, np.float64).T @ Z)
        return Z

    monkeypatch.setattr(E, "cgs2_a", cgs2_no_round)
    r, trace = _mixed(lu_small)
    assert pinlib.binary32_representability_violation(trace) > 0


def test_binary64_matrix_in_basis_product_is_caught(lu_small, monkeypatch):
    monkeypatch.setattr(E, "basis_matrix", lambda A, dtype: A)
    r, trace = _mixed(lu_small)
    assert pinlib.basis_product_rounding_violation(trace, _a32(lu_small)) > 0.5 + 1e-6


def test_binary32_matrix_in_residual_replacement_is_caught(lu_small, monkeypatch):
    p, A, dom = lu_small
    orig = E.basis_matrix
    monkeypatch.setattr(E, "true_residual",
                        lambda A_, b, x: b - orig(A_, np.float32) @ x)
    r = O.sstep_srecg(A, dom, 4, 2, p.b, tol=1e-11, maxit=500, basis_dtype=np.float32,
                      inner_tol=1e-5)
    true = np.linalg.norm(p.b - A @ r.x) / np.linalg.norm(p.b)
    assert true > 1e-11             # the refinement pin fails


def test_binary32_gram_accumulation_is_caught(lu_small, monkeypatch):
    # A-CholQR with the Gram summed in binary32 (and factorised from that)
    import scipy.linalg as sla

    def acholqr_gram32(Ab, Z, dtype=np.float64, trace=None):
        AZ = E._spmm(Ab, Z, dtype)
        G = (np.asarray(Z, np.float32).T @ np.asarray(AZ, np.float32)).astype(np.float64)
        G = np.triu(G) + np.triu(G, 1).T
        if trace is not None:
            trace.update(Z=Z, AZ=AZ, G=G)
        R = O.chol_upper(G)
        W = E._store(sla.solve_triangular(R, E._f64(Z).T, trans="T").T, dtype)
        AW = E._store(sla.solve_triangular(R, E._f64(AZ).T, trans="T").T, dtype)
        if trace is not None:
            trace.update(R=R, W=W, AW=AW)
        return W, AW, R

    monkeypatch.setattr(E, "a_cholqr", acholqr_gram32)
    r, trace = _mixed(lu_small, maxit=3)
    assert pinlib.gram_accuracy_violation(trace) > 1.0
