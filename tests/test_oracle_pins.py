"""Pins of the CPU oracle against what the paper and the mathematics fix.

No GPU.  Each check here is something other than the oracle's own formula:
closed forms, dense factorisations, the paper's printed iteration counts,
identities the paper states, and invariants that follow from eqs (1)-(3).
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
import problems as P
from tests import pinlib


# ---------------------------------------------------------------------------
# Small-matrix building blocks
# ---------------------------------------------------------------------------

def _rand_spd(n, seed, cond=10.0):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    ev = np.geomspace(1.0, cond, n)
    return (Q * ev) @ Q.T


def test_chol_upper_closed_form():
    # [[4, 2], [2, 5]] = R^t R with R = [[2, 1], [0, 2]]
    R = O.chol_upper(np.array([[4.0, 2.0], [2.0, 5.0]]))
    assert np.array_equal(R, np.array([[2.0, 1.0], [0.0, 2.0]]))


@pytest.mark.parametrize("t", [1, 2, 3, 8, 16, 64])
def test_chol_upper_reconstructs(t):
    G = _rand_spd(t, t, cond=1e6)
    R = O.chol_upper(G)
    assert np.allclose(np.tril(R, -1), 0.0)
    assert (np.diag(R) > 0).all()
    assert np.abs(R.T @ R - G).max() <= 1e-12 * np.abs(G).max()


def test_chol_upper_breakdown():
    with pytest.raises(O.Breakdown):
        O.chol_upper(np.diag([1.0, -1.0, 2.0]))
    with pytest.raises(O.Breakdown):
        O.chol_upper(np.diag([1.0, 0.0]))           # zero column of T(r)
    with pytest.raises(O.Breakdown):
        O.chol_upper(np.array([[np.nan]]))


# ---------------------------------------------------------------------------
# Generators (inputs) -- pinned so that the oracle is fed the right matrices
# ---------------------------------------------------------------------------

def test_poisson_matches_kron_construction():
    p = P.poisson2d(12, t=1, parts=(1, 1, 1))
    m = 12
    T = sp.diags([-1.0, 2.0, -1.0], [-1, 0, 1], shape=(m, m))
    G = (sp.kron(sp.eye(m), T) + sp.kron(T, sp.eye(m))).toarray()
    assert np.array_equal(p.scipy().toarray(), G)


def test_poisson_spectrum_closed_form():
    m = 12
    A = P.poisson2d(m, t=1, parts=(1, 1, 1)).scipy().toarray()
    pq = np.arange(1, m + 1) * math.pi / (m + 1)
    ev = (4.0 - 2.0 * np.cos(pq)[:, None] - 2.0 * np.cos(pq)[None, :]).ravel()
    assert np.allclose(np.sort(np.linalg.eigvalsh(A)), np.sort(ev), atol=1e-12)


@pytest.mark.parametrize("shape", [(100, 100, 1), (128, 128, 128), (1000, 1000, 1), (256, 256, 256)])
def test_stencil_nnz(shape):
    # Table 1 gives 49,600 for Poisson2D
    want = {(100, 100, 1): 49600, (128, 128, 128): 14581760,
            (1000, 1000, 1): 4996000, (256, 256, 256): 117047296}[shape]
    assert P.stencil_nnz(shape) == want


def test_generated_nnz_and_symmetry():
    p = P.poisson2d()
    assert p.nnz == 49600 and p.n == 10000
    A = P.make_problem("h", (9, 7, 5), P.kappa_random_blocks((9, 7, 5), 5, block=3),
                       seed=5, t=1, s=1, parts=(1, 1, 1)).scipy()
    assert A.nnz == P.stencil_nnz((9, 7, 5))
    assert abs(A - A.T).max() == 0.0
    # weakly diagonally dominant with a positive diagonal -> SPD for Dirichlet
    d = A.diagonal()
    off = np.asarray(abs(A).sum(axis=1)).ravel() - d
    assert (d > 0).all() and (d >= off - 1e-9 * d).all()
    assert np.linalg.eigvalsh(A.toarray()).min() > 0


def test_uniform_stream_is_deterministic_and_bounded():
    a = P.uniform_pm1(3, 0, 1000)
    b = P.uniform_pm1(3, 0, 1000)
    assert np.array_equal(a, b)
    assert a.min() >= -1.0 and a.max() < 1.0
    assert not np.array_equal(a, P.uniform_pm1(3, 1, 1000))
    assert abs(a.mean()) < 0.1


# ---------------------------------------------------------------------------
# Partition and T(r)
# ---------------------------------------------------------------------------

def _interval_part(i, n, p):
    """Axis part containing coordinate i when [0, n) is cut at
    ceil(d*n/p), d = 0..p (an interval description of the same boxes)."""
    cuts = [-(-d * n // p) for d in range(p + 1)]
    for d in range(p):
        if cuts[d] <= i < cuts[d + 1]:
            return d
    raise AssertionError


@pytest.mark.parametrize("shape,parts", [((10, 7, 3), (3, 2, 2)), ((100, 100, 1), (2, 4, 1)),
                                         ((5, 5, 5), (1, 5, 2)), ((13, 1, 1), (4, 1, 1))])
def test_partition_is_the_box_decomposition(shape, parts):
    dom = O.partition_grid(shape, parts)
    nx, ny, nz = shape
    px, py, pz = parts
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                want = (_interval_part(i, nx, px)
                        + px * (_interval_part(j, ny, py) + py * _interval_part(k, nz, pz)))
                assert dom[i + nx * (j + ny * k)] == want


@pytest.mark.parametrize("cfg,size", [("C1", 1250), ("C2", 131072), ("C3", 65536),
                                      ("C4", 62500), ("C5", 262144)])
def test_partition_domain_sizes(cfg, size):
    shapes = {"C1": ((100, 100, 1), (2, 4, 1)), "C2": ((128,) * 3, (4, 4, 1)),
              "C3": ((128,) * 3, (2, 4, 4)), "C4": ((1000, 1000, 1), (4, 4, 1)),
              "C5": ((256,) * 3, (4, 4, 4))}
    shape, parts = shapes[cfg]
    dom = O.partition_grid(shape, parts)
    t = parts[0] * parts[1] * parts[2]
    assert dom.dtype == np.int32
    assert np.array_equal(np.bincount(dom, minlength=t), np.full(t, size))


def test_split_T():
    rng = np.random.default_rng(0)
    dom = O.partition_grid((10, 7, 3), (3, 2, 2))
    r = rng.standard_normal(dom.shape[0])
    Z = O.split_T(r, dom, 12)
    assert np.array_equal(Z.sum(axis=1), r)            # T(r) 1_t = r, bitwise
    assert np.array_equal((Z != 0).sum(axis=1), np.ones_like(dom))
    for d in range(12):                                 # column d lives on domain d
        assert np.array_equal(np.nonzero(Z[:, d])[0], np.nonzero(dom == d)[0])


# ---------------------------------------------------------------------------
# Dense references
# ---------------------------------------------------------------------------

def test_dense_cholesky_solve_recovers_xstar():
    A = _rand_spd(40, 1, cond=1e4)
    xs = np.random.default_rng(2).standard_normal(40)
    x = O.dense_cholesky_solve(A, A @ xs)
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) < 1e-10


# ---------------------------------------------------------------------------
# CG and the enlarged methods
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def c1():
    p = P.poisson2d()
    return p, p.scipy(), O.partition_grid(p.shape, p.parts)


@pytest.fixture(scope="module")
def c1_s2(c1):
    p, A, dom = c1
    return O.sstep_srecg(A, dom, 8, 2, p.b, tol=1e-8, record=True)


def test_cg_matches_dense_solve():
    p = P.poisson2d(16, t=1, parts=(1, 1, 1))
    A = p.scipy()
    r = O.cg(A, p.b, tol=1e-13)
    assert np.linalg.norm(r.x - O.dense_cholesky_solve(A.toarray(), p.b)) < 1e-10 * np.linalg.norm(r.x)


@pytest.mark.parametrize("variant", ["srecg", "srecg2"])
@pytest.mark.parametrize("t,s", [(1, 1), (2, 3), (4, 2), (8, 1)])
def test_sstep_matches_dense_solve(variant, t, s):
    A = sp.csr_matrix(_rand_spd(48, 7, cond=50.0))
    xs = np.random.default_rng(8).standard_normal(48)
    dom = O.partition_grid((48, 1, 1), (t, 1, 1))
    r = O.sstep_srecg(A, dom, t, s, A @ xs, tol=1e-13, maxit=200, variant=variant)
    assert r.status == O.OK
    assert np.linalg.norm(r.x - xs) / np.linalg.norm(xs) < 1e-10


@pytest.mark.parametrize("t,s", [(4, 3), (2, 4), (8, 2), (16, 1)])
def test_srecg2_finite_termination(t, s):
    # the enlarged Krylov subspace after k s-step iterations has dimension
    # <= k s t; when it reaches n the solution is exact
    n = 48
    A = sp.csr_matrix(_rand_spd(n, 11, cond=20.0))
    xs = np.random.default_rng(12).standard_normal(n)
    dom = O.partition_grid((n, 1, 1), (t, 1, 1))
    r = O.sstep_srecg(A, dom, t, s, A @ xs, tol=1e-11, maxit=100, variant="srecg2")
    assert r.status == O.OK
    assert r.iters <= math.ceil(n / (s * t))
    assert np.linalg.norm(r.x - xs) / np.linalg.norm(xs) < 1e-9


def test_cg_poisson_table2(c1):
    p = P.poisson2d(rhs="unit", tol=1e-6)
    r = O.cg(p.scipy(), p.b, tol=1e-6)
    want = pinlib.read_poisson_table()[("cg", 1)][0]
    assert abs(r.iters - want) <= 0.05 * want


def _band(got, want):
    # our domains are geometric boxes and x comes from another generator,
    # not Metis k-way domains and MATLAB's rand: a soft band
    return abs(got - want) <= max(2, 0.10 * want)


@pytest.mark.parametrize("t", [2, 8, 16])
def test_sstep_srecg_poisson_table2(t):
    p = P.poisson2d(rhs="unit", tol=1e-6)
    A = p.scipy()
    parts = {2: (2, 1, 1), 4: (2, 2, 1), 8: (2, 4, 1), 16: (4, 4, 1),
             32: (4, 8, 1), 64: (8, 8, 1)}[t]
    dom = O.partition_grid(p.shape, parts)
    row = pinlib.read_poisson_table()[("sre-cg", t)]
    svals = [1, 2, 4, 10]
    want = [row[pinlib.SVALS.index(s)] for s in svals]
    got = [O.sstep_srecg(A, dom, t, s, p.b, tol=1e-6).iters for s in svals]
    for s, g, w in zip(svals, got, want):
        assert _band(g, w), (t, s, g, w)
    # no loss of A-orthogonality on Poisson2D: k_s = ceil(k_1 / s) (Section 4)
    for s, g in zip(svals[1:], got[1:]):
        assert math.ceil(got[0] / s) <= g <= math.ceil(got[0] / s) + 1


def test_sstep_srecg_poisson_table2_t64():
    # the 64-domain row at s = 4 (the wide-block case)
    p = P.poisson2d(rhs="unit", tol=1e-6)
    A = p.scipy()
    dom = O.partition_grid(p.shape, (8, 8, 1))
    want = pinlib.read_poisson_table()[("sre-cg", 64)][pinlib.SVALS.index(4)]
    got = O.sstep_srecg(A, dom, 64, 4, p.b, tol=1e-6).iters
    assert _band(got, want), (got, want)


@pytest.mark.parametrize("t", [2, 8])
def test_sstep_srecg2_poisson_table3(t):
    p = P.poisson2d(rhs="unit", tol=1e-6)
    A = p.scipy()
    parts = {2: (2, 1, 1), 8: (2, 4, 1)}[t]
    dom = O.partition_grid(p.shape, parts)
    want = pinlib.read_poisson_table()[("sre-cg2", t)]
    for s, w in zip([2, 10], [want[1], want[6]]):
        g = O.sstep_srecg(A, dom, t, s, p.b, tol=1e-6, variant="srecg2").iters
        assert _band(g, w), (t, s, g, w)


def test_s1_is_sre_cg(c1):
    # for s = 1 the s-step algorithms reduce to SRE-CG / SRE-CG2 (Section 3.1)
    p, A, dom = c1
    for variant in ("srecg", "srecg2"):
        a = O.sstep_srecg(A, dom, 8, 1, p.b, tol=1e-8, variant=variant,
                          maxit=40 if variant == "srecg2" else 100000)
        b = O.srecg(A, dom, 8, p.b, tol=1e-8, variant=variant,
                    maxit=40 if variant == "srecg2" else 100000)
        assert a.iters == b.iters
        assert np.linalg.norm(a.x - b.x) <= 1e-12 * np.linalg.norm(b.x)


def test_t1_s1_is_cg(c1):
    # t = s = 1: the enlarged Krylov subspace is the Krylov subspace
    p, A, _ = c1
    d1 = np.zeros(p.n, dtype=np.int32)
    a = O.sstep_srecg(A, d1, 1, 1, p.b, tol=1e-8, record=True)
    c = O.cg(A, p.b, tol=1e-8, record=True)
    assert abs(a.iters - c.iters) <= 2
    for k in range(1, c.iters):
        if c.hist[k] <= 1e-6 * c.hist[0]:
            break
        xc = c.extra["xs"][k]
        assert np.linalg.norm(a.extra["xs"][k] - xc) <= 1e-8 * np.linalg.norm(xc)


def test_sstep_is_s_sre_cg_steps(c1, c1_s2):
    # without loss of A-orthogonality one s-step iteration equals s SRE-CG
    # iterations (Section 3.1)
    p, A, dom = c1
    r1 = O.sstep_srecg(A, dom, 8, 1, p.b, tol=1e-8, record=True)
    r2 = c1_s2
    assert math.ceil(r1.iters / 2) <= r2.iters <= math.ceil(r1.iters / 2) + 1
    for k in range(1, r2.iters):
        xa, xb = r2.extra["xs"][k], r1.extra["xs"][2 * k]
        assert np.linalg.norm(xa - xb) <= 1e-8 * np.linalg.norm(xb)


def test_a_orthonormal_basis(c1, c1_s2):
    p, A, _ = c1
    assert pinlib.orthonormality_violation(c1_s2, A) <= 1e-10
    assert pinlib.cross_block_violation(c1_s2, A) <= 1e-10


def test_petrov_galerkin(c1_s2):
    assert pinlib.petrov_galerkin_violation(c1_s2) <= 1e-10


def test_error_drop_identity_and_monotone_energy(c1, c1_s2):
    p, A, _ = c1
    assert pinlib.error_drop_violation(c1_s2, A, p.xstar) <= 1e-8
    assert pinlib.monotone_energy_violation(c1_s2, A, p.xstar) <= 0.0


def test_basis_choice_invariance(c1, c1_s2):
    # x_k depends only on the span of the basis: A-CholQR, Pre-CholQR and a
    # fresh A W_{j-1} give the same iterates
    p, A, dom = c1
    for kw in ({"orth": "precholqr"}, {"aimage": "fresh"}):
        r = O.sstep_srecg(A, dom, 8, 2, p.b, tol=1e-8, record=True, **kw)
        assert r.iters == c1_s2.iters
        for k in range(1, 25):
            xa, xb = r.extra["xs"][k], c1_s2.extra["xs"][k]
            assert np.linalg.norm(xa - xb) <= 1e-10 * np.linalg.norm(xb)


def test_zero_rhs_and_maxit(c1):
    p, A, dom = c1
    r = O.sstep_srecg(A, dom, 8, 2, np.zeros(p.n), tol=1e-8)
    assert r.status == O.OK and r.iters == 0 and not r.x.any()
    r = O.sstep_srecg(A, dom, 8, 2, p.b, tol=1e-8, maxit=3)
    assert r.status == O.MAXIT and r.iters == 3 and len(r.hist) == 4


def test_breakdown_on_zero_domain(c1):
    # b zero on a whole domain -> zero column of T(r_0) -> singular Gram
    p, A, dom = c1
    b = p.b.copy()
    b[dom == 3] = 0.0
    x0 = np.zeros(p.n)
    r = O.sstep_srecg(A, dom, 8, 2, b - A @ x0 * 0, tol=1e-8)
    assert r.status == O.BREAKDOWN and r.iters == 0


def test_breakdown_on_indefinite_matrix():
    p = P.poisson2d(10, t=2, parts=(2, 1, 1))
    vals = p.vals.copy()
    diag = np.repeat(np.arange(p.n), np.diff(p.rowptr)) == p.colind
    vals[np.nonzero(diag)[0][:50]] *= -1.0
    A = O.csr(p.rowptr, p.colind, vals)
    dom = O.partition_grid(p.shape, p.parts)
    r = O.sstep_srecg(A, dom, 2, 2, p.b, tol=1e-8, maxit=100)
    assert r.status == O.BREAKDOWN


def test_mixed_precision_form_reaches_tolerance(c1, c1_s2):
    p, A, dom = c1
    r = O.sstep_srecg(A, dom, 8, 2, p.b, tol=1e-8, basis_dtype=np.float32, inner_tol=1e-5)
    assert r.status == O.OK and r.true_relres <= 1e-8 and r.restarts >= 1
    assert np.linalg.norm(r.x - c1_s2.x) <= 1e-6 * np.linalg.norm(c1_s2.x)


def test_srecg2_restart_at_capacity():
    p = P.poisson2d(40, t=8, parts=(2, 4, 1))
    A = p.scipy()
    dom = O.partition_grid(p.shape, p.parts)
    r = O.sstep_srecg(A, dom, 8, 2, p.b, tol=1e-8, variant="srecg2", q_cap_blocks=10)
    assert r.status == O.OK and r.restarts >= 1 and r.true_relres <= 1e-8


# ---------------------------------------------------------------------------
# Gradient of a loss through the solve
# ---------------------------------------------------------------------------

def test_adjoint_gradient_matches_finite_differences():
    shape = (6, 5, 1)
    p = P.make_problem("g", shape, P.kappa_loguniform(shape, 4, -1, 1), seed=4, t=1, s=1,
                       parts=(1, 1, 1))
    A = p.scipy().toarray()
    x_tgt = P.uniform_pm1(4, 2, p.n)
    x, lam, gA = O.dense_gradient(A, p.b, x_tgt)
    gv = O.sddmm(p.rowptr, p.colind, lam, x)
    rows = np.repeat(np.arange(p.n), np.diff(p.rowptr))

    def loss(Am, bv):
        xv = O.dense_cholesky_solve(Am, bv)
        return float(np.sum((xv - x_tgt) ** 2))

    for q in range(0, p.nnz, 7):
        i, j = rows[q], p.colind[q]
        h = 1e-6 * abs(A[i, j])
        Ap, Am = A.copy(), A.copy()
        Ap[i, j] += h
        Am[i, j] -= h
        if i != j:                                  # keep A symmetric
            Ap[j, i] += h
            Am[j, i] -= h
        fd = (loss(Ap, p.b) - loss(Am, p.b)) / (2 * h)
        q_t = np.nonzero((rows == j) & (p.colind == i))[0][0]
        an = gv[q] + (gv[q_t] if i != j else 0.0)
        assert abs(fd - an) <= 1e-5 * max(1.0, abs(an)), (q, fd, an)
    # dL/db by finite differences
    for i in range(0, p.n, 5):
        h = 1e-6
        bp, bm = p.b.copy(), p.b.copy()
        bp[i] += h
        bm[i] -= h
        fd = (loss(A, bp) - loss(A, bm)) / (2 * h)
        assert abs(fd - lam[i]) <= 1e-5 * max(1.0, abs(lam[i]))


# ---------------------------------------------------------------------------
# The binary32-basis precision form: what "binary32 basis, binary64 Grams
# and binary64 residual replacement" fixes, checked independently
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def lu_small():
    """30 x 30 log-uniform diffusion (harmonic-mean values, not binary32
    numbers), t = 4, s = 2."""
    shape = (30, 30, 1)
    p = P.make_problem("lu", shape, P.kappa_loguniform(shape, 4, -2, 2), seed=4, t=4, s=2,
                       parts=(2, 2, 1))
    return p, p.scipy(), O.partition_grid(shape, (2, 2, 1))


def _mixed_trace(lu_small, **kw):
    p, A, dom = lu_small
    trace = []
    args = dict(tol=1e-8, maxit=12, basis_dtype=np.float32, inner_tol=1e-5)
    args.update(kw)
    r = O.sstep_srecg(A, dom, 4, 2, p.b, trace=trace, **args)
    return r, trace


def test_binary32_blocks_are_binary32(lu_small):
    r, trace = _mixed_trace(lu_small)
    assert len(pinlib._blocks(trace)) == 24
    assert pinlib.binary32_representability_violation(trace) == 0
    # the same pin has teeth: the binary64 form's blocks are not binary32
    p, A, dom = lu_small
    t64 = []
    O.sstep_srecg(A, dom, 4, 2, p.b, tol=1e-8, maxit=2, trace=t64)
    assert pinlib.binary32_representability_violation(t64) > 1000


def test_binary32_basis_product_uses_rounded_matrix(lu_small):
    p, A, dom = lu_small
    # the matrix values are not binary32 numbers, so the two products differ
    assert np.count_nonzero(A.data.astype(np.float32).astype(np.float64) != A.data) > 0.9 * A.nnz
    r, trace = _mixed_trace(lu_small)
    A32 = A.toarray().astype(np.float32).astype(np.float64)
    assert pinlib.basis_product_rounding_violation(trace, A32) <= 0.5 + 1e-6


def test_binary32_grams_are_binary64_sums(lu_small):
    r, trace = _mixed_trace(lu_small, maxit=4)
    assert pinlib.gram_accuracy_violation(trace) <= 1.0


def test_binary32_form_refines_to_binary64_accuracy(lu_small):
    # iterative refinement with binary64 residuals reaches a true residual
    # (recomputed here with the binary64 matrix) far below binary32
    # resolution: the residual replacement uses the binary64 matrix
    p, A, dom = lu_small
    r = O.sstep_srecg(A, dom, 4, 2, p.b, tol=1e-11, maxit=500, basis_dtype=np.float32,
                      inner_tol=1e-5)
    true = np.linalg.norm(p.b - A @ r.x) / np.linalg.norm(p.b)
    assert r.status == O.OK and r.restarts >= 2
    assert true <= 1e-11


def test_parity_criterion_bounds_hold_for_oracle_ensembles():
    # the sensitive-regime criterion of tests/parity.py: the oracle's own
    # spread on the GPU tests' 16^3 skyscraper problem stays inside the
    # stated bounds, and the oracle passes the criterion against itself
    from tests.parity import SPREAD_2, SPREAD_A, check_parity, ensemble_spreads, oracle_ensemble
    shape = (16, 16, 16)
    p = P.make_problem("sky", shape, P.kappa_skyscraper(shape, 2, tile=4), seed=2, t=16, s=4,
                       parts=(4, 4, 1))
    A = p.scipy()
    dom = O.partition_grid(shape, (4, 4, 1))
    runs = oracle_ensemble(A, dom, 16, 4, p.b, k=3, variant="srecg2")
    _, s2, sa = ensemble_spreads(runs, A)
    assert sa <= SPREAD_A and s2 <= SPREAD_2
    check_parity(runs[-1].iters, runs[-1].x, runs[:-1], A)


def test_domain_order_brute_force():
    # the definition written out: sort by (domain, row)
    rng = np.random.default_rng(7)
    for n, t in ((1, 1), (17, 3), (200, 8)):
        dom = rng.integers(0, t, n).astype(np.int32)
        want = sorted(range(n), key=lambda i: (int(dom[i]), i))
        got = O.domain_order(dom)
        assert got.dtype == np.int32 and got.tolist() == want
    # with keys (small range, so that ties occur): sort by (domain, key, row)
    for n, t in ((1, 1), (17, 3), (300, 8)):
        dom = rng.integers(0, t, n).astype(np.int32)
        key = rng.integers(-5, 5, n).astype(np.int64)
        want = sorted(range(n), key=lambda i: (int(dom[i]), int(key[i]), i))
        assert O.domain_order(dom, key).tolist() == want
    p = P.poisson2d(12, t=8, parts=(2, 4, 1))
    dom = O.partition_grid(p.shape, p.parts)
    order = O.domain_order(dom)
    assert sorted(order.tolist()) == list(range(p.n))
    assert (np.diff(dom[order]) >= 0).all()
