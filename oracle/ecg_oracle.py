"""Plain float64 oracle of CG, enlarged CG (SRE-CG / SRE-CG2) and their
s-step versions (Moufawad, arXiv 1804.10629).

TEST INFRASTRUCTURE ONLY -- see ``oracle/__init__.py``.

The algorithms are written in the paper's order and notation: a block of t
vectors ``W_j`` is built from ``T(r_0)`` (first block) or from ``A W_{j-1}``,
A-orthonormalized against earlier blocks with block classical Gram-Schmidt
applied twice (CGS2), then against itself with A-CholQR (or Pre-CholQR); s
such blocks form ``V``; the solution is updated once per s-step iteration
with ``alpha = V^t r``.  Library primitives used as single steps: the sparse
matrix product (scipy CSR), dense matrix products (numpy), triangular solves
(scipy).  The small Cholesky factorisation is written out so that its
breakdown rule is explicit.

Readings of points the paper leaves open are marked READING in the code.

Pins (see tests/test_oracle_*.py): dense Cholesky solves on small systems,
closed-form Poisson spectra, the identities s=1 => SRE-CG and t=s=1 => CG,
A-orthonormality, the Petrov-Galerkin condition, the A-norm error drop
identity implied by eqs (1)-(3), finite termination in at most ceil(n/(st))
iterations for SRE-CG2, the Poisson2D iteration counts of Tables 2-3 (soft
band), and planted-mistake checks that each of these catches.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

__all__ = [
    "OK", "MAXIT", "BREAKDOWN", "STAGNATED",
    "csr", "partition_grid", "domain_order", "split_T", "chol_upper", "cgs2_a", "a_cholqr",
    "pre_cholqr", "cg", "srecg", "sstep_srecg", "SolveResult", "basis_matrix", "true_residual",
    "dense_cholesky_solve", "sddmm", "dense_gradient", "Breakdown",
    "ic0", "block_jacobi_ic0", "block_jacobi_cholesky", "apply_llt_inverse", "pcg",
]

OK, MAXIT, BREAKDOWN, STAGNATED = 0, 1, 2, 3


class Breakdown(Exception):
    """A Cholesky pivot was <= 0 or not finite."""


def csr(rowptr, colind, vals, n=None) -> sp.csr_matrix:
    n = len(rowptr) - 1 if n is None else n
    return sp.csr_matrix((np.asarray(vals), np.asarray(colind), np.asarray(rowptr)),
                         shape=(n, n))


# ---------------------------------------------------------------------------
# Domain decomposition and the split operator T (Section 2; Section 3.1)
# ---------------------------------------------------------------------------

def partition_grid(shape, parts) -> np.ndarray:
    """Geometric domain decomposition of an nx x ny x nz grid into px*py*pz
    boxes.  READING: the paper partitions with Metis k-way (Section 4);
    Metis is not available, so domains are axis-aligned boxes: cell
    (i, j, k), row ``i + nx*(j + ny*k)``, belongs to domain
    ``floor(i*px/nx) + px*(floor(j*py/ny) + py*floor(k*pz/nz))``.
    Parity: bit-exact (integers)."""
    nx, ny, nz = (int(v) for v in shape)
    px, py, pz = (int(v) for v in parts)
    n = nx * ny * nz
    dom = np.empty(n, dtype=np.int32)
    row = 0
    for k in range(nz):
        dk = (k * pz) // nz
        for j in range(ny):
            dj = (j * py) // ny
            base = px * (dj + py * dk)
            i = np.arange(nx, dtype=np.int64)
            dom[row:row + nx] = base + (i * px) // nx
            row += nx
    return dom


def domain_order(dom: np.ndarray, key: np.ndarray | None = None) -> np.ndarray:
    """Domain-contiguous row order: the rows of domain 0 in increasing index
    order, then those of domain 1, and so on (Section 4 reorders the matrix
    by its Metis domains; READING: rows keep the caller's order within a
    domain, or, when a per-row key is given, are sorted by key within a
    domain with ties in index order -- the paper leaves the order inside a
    domain open).  order[i] is the original row placed at position i.
    Parity: bit-exact (integers)."""
    dom = np.asarray(dom)
    if key is None:
        return np.argsort(dom, kind="stable").astype(np.int32)
    idx = np.arange(dom.shape[0])
    return np.lexsort((idx, np.asarray(key), dom)).astype(np.int32)


def split_T(r: np.ndarray, dom: np.ndarray, t: int) -> np.ndarray:
    """T(r): the n x t matrix whose column d is r restricted to domain d
    (Section 2: the operator that splits r into t vectors by domain;
    Theorem 1's proof uses T(r) 1_t = r).  Parity: bit-exact."""
    n = r.shape[0]
    Z = np.zeros((n, t), dtype=r.dtype)
    Z[np.arange(n), dom] = r
    return Z


# ---------------------------------------------------------------------------
# A-orthonormalization: CGS2 against earlier blocks, then A-CholQR or
# Pre-CholQR against itself (Section 4, the orthonormalization paragraph)
# ---------------------------------------------------------------------------

def chol_upper(G: np.ndarray) -> np.ndarray:
    """Upper triangular R with positive diagonal and R^t R = G, by the
    textbook column-by-column Cholesky recurrence.  READING (breakdown
    rule): the factorisation fails, raising Breakdown, iff a pivot is <= 0
    or not finite; no relative threshold is applied."""
    t = G.shape[0]
    R = np.zeros_like(G, dtype=np.float64)
    for j in range(t):
        piv = G[j, j] - R[:j, j] @ R[:j, j]
        if not np.isfinite(piv) or piv <= 0.0:
            raise Breakdown(f"pivot {j}: {piv}")
        R[j, j] = math.sqrt(piv)
        for c in range(j + 1, t):
            R[j, c] = (G[j, c] - R[:j, j] @ R[:j, c]) / R[j, j]
    return R


def _store(M: np.ndarray, dtype) -> np.ndarray:
    """Round a float64 result to the basis storage type."""
    return M if dtype == np.float64 else M.astype(dtype)


def _f64(M: np.ndarray) -> np.ndarray:
    return np.asarray(M, dtype=np.float64)


def _spmm(Ab: sp.csr_matrix, Z: np.ndarray, dtype) -> np.ndarray:
    """A Z with float64 accumulation, rounded to the storage type.  In the
    float32 form both the matrix values and Z are float32; their products
    are exact in float64."""
    return _store(Ab @ _f64(Z), dtype)


def cgs2_a(Z: np.ndarray, Wp: Optional[np.ndarray], AWp: Optional[np.ndarray],
           dtype=np.float64):
    """A-orthonormalize Z against the columns of Wp (earlier blocks side by
    side, Wp^t A Wp = I, with their A-images AWp) by block classical
    Gram-Schmidt in the A inner product, applied twice (the paper's CGS2).
    READING: the thesis' CGS2 is not reproduced in the paper; each pass
    computes H = (A Wp)^t Z from the stored A-images and then subtracts
    Wp H, with no normalisation in between.
    """
    if Wp is None or Wp.shape[1] == 0:
        return Z
    Wd, AWd = _f64(Wp), _f64(AWp)
    for _ in range(2):
        H = AWd.T @ _f64(Z)
        Z = _store(_f64(Z) - Wd @ H, dtype)
    return Z


class _BlockStore:
    """Earlier blocks W_i (and A W_i) kept side by side in one n x m array,
    grown by doubling, so that CGS2 against all of them is one product."""

    def __init__(self, n, dtype, keep_last=None):
        self.n, self.dtype, self.keep_last = n, dtype, keep_last
        self.W = np.zeros((n, 0), dtype=dtype)
        self.AW = np.zeros((n, 0), dtype=dtype)
        self.widths = []
        self.m = 0

    def __len__(self):
        return len(self.widths)

    def add(self, W, AW):
        w = W.shape[1]
        if self.keep_last is not None:
            self.widths = (self.widths + [w])[-self.keep_last:]
            cols = sum(self.widths)
            self.W = np.concatenate([self.W[:, self.m - (cols - w):self.m], W], axis=1)
            self.AW = np.concatenate([self.AW[:, self.m - (cols - w):self.m], AW], axis=1)
            self.m = cols
            return
        if self.m + w > self.W.shape[1]:
            cap = max(2 * self.W.shape[1], self.m + w)
            for name in ("W", "AW"):
                grown = np.zeros((self.n, cap), dtype=self.dtype)
                grown[:, :self.m] = getattr(self, name)[:, :self.m]
                setattr(self, name, grown)
        self.W[:, self.m:self.m + w] = W
        self.AW[:, self.m:self.m + w] = AW
        self.m += w
        self.widths.append(w)

    def last(self):
        w = self.widths[-1]
        return self.W[:, self.m - w:self.m], self.AW[:, self.m - w:self.m]

    def all(self):
        return self.W[:, :self.m], self.AW[:, :self.m]


def a_cholqr(Ab: sp.csr_matrix, Z: np.ndarray, dtype=np.float64, trace=None):
    """A-CholQR: G = Z^t A Z = R^t R, W = Z R^{-1}, A W = (A Z) R^{-1}.
    READING: G is formed from its upper triangle (i <= j) and mirrored.
    `trace` (a dict, optional) receives Z, A Z, G and R."""
    AZ = _spmm(Ab, Z, dtype)
    G = _f64(Z).T @ _f64(AZ)
    G = np.triu(G) + np.triu(G, 1).T
    if trace is not None:
        trace.update(Z=Z, AZ=AZ, G=G)
    R = chol_upper(G)
    W = _store(sla.solve_triangular(R, _f64(Z).T, trans="T", lower=False).T, dtype)
    AW = _store(sla.solve_triangular(R, _f64(AZ).T, trans="T", lower=False).T, dtype)
    if trace is not None:
        trace.update(R=R, W=W, AW=AW)
    return W, AW, R


def pre_cholqr(Ab: sp.csr_matrix, Z: np.ndarray, dtype=np.float64, trace=None):
    """Pre-CholQR: a Euclidean CholQR of Z (Z^t Z = Re^t Re, Z <- Z Re^{-1})
    followed by A-CholQR of the result."""
    Zd = _f64(Z)
    Ge = Zd.T @ Zd
    Ge = np.triu(Ge) + np.triu(Ge, 1).T
    Re = chol_upper(Ge)
    Z = _store(sla.solve_triangular(Re, Zd.T, trans="T", lower=False).T, dtype)
    if trace is None:
        return a_cholqr(Ab, Z, dtype)
    trace["Z_pre"] = Zd
    return a_cholqr(Ab, Z, dtype, trace=trace)


def basis_matrix(A: sp.csr_matrix, dtype) -> sp.csr_matrix:
    """The matrix the basis is built with: A itself, or in the binary32
    precision form A with its values rounded to binary32 (held as float64,
    so that products with binary32 blocks are exact before the sum)."""
    if dtype == np.float64:
        return A
    return csr(A.indptr, A.indices, A.data.astype(np.float32).astype(np.float64), A.shape[0])


def true_residual(A: sp.csr_matrix, b: np.ndarray, x: np.ndarray) -> np.ndarray:
    """b - A x with the binary64 matrix (initial residual and every residual
    replacement, in both precision forms)."""
    return b - A @ x


# ---------------------------------------------------------------------------
# Classical CG (Section 2; the preconditioned CG algorithm of Section 6 with
# M = I)
# ---------------------------------------------------------------------------

@dataclass
class SolveResult:
    x: np.ndarray
    iters: int
    hist: List[float]
    status: int
    restarts: int = 0
    true_relres: float = float("nan")
    blocks: int = 0
    extra: dict = field(default_factory=dict)


def cg(A: sp.csr_matrix, b: np.ndarray, x0=None, tol=1e-8, maxit=100000,
       record=False) -> SolveResult:
    """Hestenes-Stiefel CG: p_1 = r_0, alpha_k = ||r_{k-1}||^2 / ||p_k||_A^2,
    beta = ||r_{k-1}||^2/||r_{k-2}||^2, stopping when ||r_k|| <= tol ||r_0||
    (the same test as the s-step algorithms).  `iters` counts matrix-vector
    products in the loop."""
    x = np.zeros_like(b) if x0 is None else x0.astype(np.float64).copy()
    r = b - A @ x
    rho0 = float(np.linalg.norm(r))
    hist = [rho0]
    xs = [x.copy()] if record else None
    if rho0 == 0.0:
        return SolveResult(x, 0, hist, OK, extra={"xs": xs})
    p = r.copy()
    rr = float(r @ r)
    k = 0
    while math.sqrt(rr) > tol * rho0 and k < maxit:
        Ap = A @ p
        alpha = rr / float(p @ Ap)
        x = x + alpha * p
        r = r - alpha * Ap
        rr_new = float(r @ r)
        p = r + (rr_new / rr) * p
        rr = rr_new
        k += 1
        hist.append(math.sqrt(rr))
        if record:
            xs.append(x.copy())
    status = OK if math.sqrt(rr) <= tol * rho0 else MAXIT
    tr = float(np.linalg.norm(b - A @ x)) / rho0
    return SolveResult(x, k, hist, status, true_relres=tr, extra={"xs": xs})


# ---------------------------------------------------------------------------
# Enlarged CG, s = 1 (SRE-CG / SRE-CG2, Section 3.1 first paragraphs)
# ---------------------------------------------------------------------------

def srecg(A: sp.csr_matrix, dom: np.ndarray, t: int, b: np.ndarray, x0=None,
          tol=1e-8, maxit=100000, variant="srecg") -> SolveResult:
    """SRE-CG (variant='srecg') or SRE-CG2 ('srecg2') as described before
    the s-step algorithms: W_1 = T(r_0) A-orthonormalized; for k >= 2,
    W_k = A W_{k-1} (a fresh product) A-orthonormalized against W_{k-1} and
    W_{k-2} (SRE-CG) or against every earlier block (SRE-CG2), then against
    itself; alpha_k = W_k^t r_{k-1}, x_k = x_{k-1} + W_k alpha_k,
    r_k = r_{k-1} - A W_k alpha_k."""
    x = np.zeros_like(b) if x0 is None else x0.astype(np.float64).copy()
    r = b - A @ x
    rho0 = float(np.linalg.norm(r))
    hist = [rho0]
    if rho0 == 0.0:
        return SolveResult(x, 0, hist, OK)
    blocks = _BlockStore(b.shape[0], np.float64, 2 if variant == "srecg" else None)
    k = 0
    rho = rho0
    while rho > tol * rho0 and k < maxit:
        if k == 0:
            Z = split_T(r, dom, t)
        else:
            Z = A @ blocks.last()[0]
        Z = cgs2_a(Z, *blocks.all())
        try:
            W, AW, _ = a_cholqr(A, Z)
        except Breakdown:
            return SolveResult(x, k, hist, BREAKDOWN)
        blocks.add(W, AW)
        alpha = W.T @ r
        x = x + W @ alpha
        r = r - AW @ alpha
        rho = float(np.linalg.norm(r))
        k += 1
        hist.append(rho)
    status = OK if rho <= tol * rho0 else MAXIT
    tr = float(np.linalg.norm(b - A @ x)) / rho0
    return SolveResult(x, k, hist, status, true_relres=tr)


def _ca_arnoldi(Ab, blocks, r, dom, t, s, dtype, orthonormalize, *, split, aimage, precond,
                plain=False):
    """One iteration's basis by the modified CA-Arnoldi A-orthonormalization
    (Section 4, algorithm "Modified CA-Arnoldi A-orthonormalization"), or
    with plain=True by the CA-Arnoldi A-orthonormalization of Section 3.1
    (algorithm "CA-Arnoldi A-orthonormalization"), which skips the first
    block's own A-orthonormalization and takes the powers of the raw block.
    `blocks` holds Q and receives the s new blocks.  Returns the lists of
    the s blocks of V and of A V."""
    Q, AQ = blocks.all()
    if split:
        Z = split_T(r, dom, t)
    elif aimage == "stored":
        Z = blocks.last()[1].copy()
    else:
        Z = _spmm(Ab, blocks.last()[0], dtype)
    if precond is not None:
        Z = precond(_f64(Z))
    Z = _store(Z, dtype)
    if plain:
        # W_j is the raw block (A W_{j-1}, or T(r) at a (re)start)
        W, AW = Z, None
    else:
        # W_j: against Q, then against itself
        Z = cgs2_a(Z, Q, AQ, dtype)
        W, AW, _ = orthonormalize(Ab, Z, dtype)
    # the monomial powers of W_j
    powers = [W]
    P = W
    for i in range(1, s):
        if i == 1 and aimage == "stored" and AW is not None:
            P = AW.copy()
        else:
            P = _spmm(Ab, P, dtype)
        if precond is not None:
            P = _store(precond(_f64(P)), dtype)
        powers.append(P)
    Vraw = np.hstack(powers)
    # V: against Q, then against itself as one s t-column block
    Vraw = cgs2_a(Vraw, Q, AQ, dtype)
    V, AV, _ = orthonormalize(Ab, Vraw, dtype)
    Vb = [V[:, i * t:(i + 1) * t] for i in range(s)]
    AVb = [AV[:, i * t:(i + 1) * t] for i in range(s)]
    for Wb, AWb in zip(Vb, AVb):
        blocks.add(Wb, AWb)
    return Vb, AVb


# ---------------------------------------------------------------------------
# s-step SRE-CG (Algorithm "s-step SRE-CG") and s-step SRE-CG2 (Algorithm
# "s-step SRE-CG2"), with eqs (1)-(3) for the update
# ---------------------------------------------------------------------------

def sstep_srecg(A: sp.csr_matrix, dom: np.ndarray, t: int, s: int, b: np.ndarray,
                x0=None, tol=1e-8, maxit=100000, *, variant="srecg",
                orth="acholqr", aimage="stored", basis_dtype=np.float64,
                inner_tol=0.0, max_restarts=20, q_cap_blocks=0,
                record=False, stop_after_blocks: Optional[int] = None,
                trace: Optional[list] = None, precond=None,
                restart_on_breakdown=True, ca=False) -> SolveResult:
    """s-step SRE-CG (variant='srecg') / s-step SRE-CG2 ('srecg2') / s-step
    MSDO-CG ('msdo', Section 3.2, algorithm "s-step MSDO-CG").

    One s-step iteration builds blocks W_j .. W_{j+s-1} (t columns each),
    where the first block after a (re)start is T(r) and every later block
    starts from A W_{j-1}; each is A-orthonormalized against W_{j-2}, W_{j-1}
    (SRE-CG) or against all blocks since the (re)start (SRE-CG2) with CGS2,
    then against itself (A-CholQR, or Pre-CholQR with orth='precholqr').
    s-step MSDO-CG is SRE-CG2 with the first block of every iteration split
    from the current residual, T(r_{k-1}): the basis spans the modified
    enlarged Krylov subspace {T(r_i), A T(r_i), .., A^{s-1} T(r_i)}.
    With V = [W_j .. W_{j+s-1}]: alpha = V^t r_{k-1}, x_k = x_{k-1} + V alpha,
    r_k = r_{k-1} - (AV) alpha, rho = ||r_k||_2; stop when rho <= tol*rho_0.

    READINGS (where the paper is silent):
      * block indices run on across s-step iterations; the first block after
        a (re)start has no CGS step, the second is orthogonalized against the
        first only;
      * aimage='stored' starts block j from the stored A-image
        A W_{j-1} = (A Z) R^{-1} (equal in exact arithmetic to a fresh
        product); aimage='fresh' forms A W_{j-1} with a new product;
      * `maxit` bounds the number of s-step iterations executed;
      * when the recursive residual meets the tolerance, the true residual
        b - A x is formed; if it does not meet the tolerance the solve
        restarts from x (r <- b - A x, next block T(r)), at most
        `max_restarts` times;
      * precision form: basis_dtype=float32 stores W, AW, Z, AZ and the
        matrix values used for the basis in float32, keeps every Gram,
        Cholesky factor, alpha, x and r in float64, and restarts (an
        iterative-refinement step) whenever rho <= inner_tol * rho_restart;
      * SRE-CG2 and MSDO-CG keep all blocks since the last restart; when
        q_cap_blocks > 0 and another s blocks would exceed it, the solve
        restarts from x;
      * a Cholesky breakdown in a block after the first one since the last
        (re)start (a numerically rank-deficient block: the new directions
        already lie in the basis, which a strong preconditioner makes
        common near convergence) discards the iteration and restarts from
        the last completed iterate (restart_on_breakdown, counted in
        `restarts`, at most max_restarts); a breakdown in the first block
        ends the solve with status BREAKDOWN.

    `precond` (optional) applies M^{-1} of a preconditioner M = L L^t to an
    n x t float64 block: the split preconditioned s-step methods of Section 5
    ("Split preconditioned s-step SRE-CG", "... SRE-CG2", "... MSDO-CG"),
    which A-orthonormalize V = L^{-t} V-hat instead of L^{-1} A L^{-t}-
    orthonormalizing V-hat: the first block after a (re)start is
    M^{-1} T(r) (for a block-diagonal M whose blocks lie inside the
    domains, L^{-t} T(L^{-1} r) = M^{-1} T(r)), every later one
    M^{-1} A W_{j-1}; alpha, x and r are updated with V and A V exactly as
    without a preconditioner.

    ca=True (or "modified") builds each iteration's basis with the modified
    CA-Arnoldi
    A-orthonormalization (Section 3.1 with Section 4, algorithm "Modified
    CA-Arnoldi A-orthonormalization"): the CA SRE-CG, CA SRE-CG2 and (with
    variant='msdo') CA MSDO-CG methods.  Per iteration, with Q the blocks
    kept (the last s+1 for SRE-CG, all since the (re)start otherwise):
    W_j is T(r) after a (re)start (and every iteration for MSDO-CG), else
    A W_{j-1} of the last block; W_j is A-orthonormalized against Q (CGS2)
    and itself (A-CholQR); the monomial powers A W_j, .., A^{s-1} W_j follow
    (the matrix powers kernel); V = [W_j, A W_j, .., A^{s-1} W_j] is
    A-orthonormalized against Q (CGS2) and then against itself as one
    st-column block (A-CholQR of V, or Pre-CholQR).  READING: A W_j is the
    stored A-image of W_j, A^i W_j (i >= 2) fresh products; with a
    preconditioner every power is M^{-1} A times the previous one (Section
    5).  The s blocks of V enter Q as s blocks of t columns.  ca="plain"
    uses the CA-Arnoldi of Section 3.1 instead: W_j is not A-orthonormalized
    on its own, V = [W_j, A W_j, ..] holds the powers of the raw block.  In
    the CA forms a breakdown during the first iteration after a (re)start
    ends the solve (a restart would repeat it).

    `trace` (a list, optional) receives one dict per block (the CGS2 output
    Z, A Z, the Gram G, R, W and A W) and one per true-residual check (x
    and its residual norm), for the precision pins.
    """
    if s < 1 or t < 1:
        raise ValueError("s and t must be >= 1")
    if ca not in (False, True, "modified", "plain"):
        raise ValueError("ca must be False, True / 'modified' or 'plain'")
    if variant not in ("srecg", "srecg2", "msdo"):
        raise ValueError("variant must be 'srecg', 'srecg2' or 'msdo'")
    dtype = np.dtype(basis_dtype).type
    Ab = basis_matrix(A, dtype)
    x = np.zeros_like(b) if x0 is None else x0.astype(np.float64).copy()
    r = true_residual(A, b, x)
    rho0 = float(np.linalg.norm(r))
    hist = [rho0]
    res = SolveResult(x, 0, hist, OK)
    if rho0 == 0.0:
        res.true_relres = 0.0
        return res
    thr_final = tol * rho0
    rho = rho0
    rho_restart = rho0
    k = 0
    restarts = 0
    nblocks = 0
    keep = (s + 1 if ca else 2) if variant == "srecg" else None

    def new_store():
        return _BlockStore(b.shape[0], dtype, keep)

    blocks = new_store()
    fresh_start = True
    m_since = 0             # blocks completed since the last (re)start
    xs = [x.copy()] if record else None
    rs = [r.copy()] if record else None
    Vs, alphas = [], []
    status = OK
    orthonormalize = a_cholqr if orth == "acholqr" else pre_cholqr
    while True:
        thr = max(inner_tol * rho_restart, thr_final)
        while rho > thr and k < maxit:
            if (variant != "srecg" and q_cap_blocks and not fresh_start
                    and len(blocks) + s > q_cap_blocks):
                r = true_residual(A, b, x)
                rho = float(np.linalg.norm(r))
                hist.append(rho)
                restarts += 1
                rho_restart = rho
                fresh_start = True
                blocks = new_store()
                m_since = 0
                continue
            V, AV = [], []
            try:
                if ca:
                    V, AV = _ca_arnoldi(Ab, blocks, r, dom, t, s, dtype, orthonormalize,
                                        split=fresh_start or variant == "msdo",
                                        aimage=aimage, precond=precond, plain=ca == "plain")
                    fresh_start = False
                    nblocks += s
                    m_since += s
                    if stop_after_blocks is not None and nblocks >= stop_after_blocks:
                        res.extra["last_blocks"] = (V, AV)
                        res.x, res.iters, res.blocks = x, k, nblocks
                        return res
                for i in range(0 if not ca else s, s):
                    if fresh_start or (variant == "msdo" and i == 0):
                        Z = split_T(r, dom, t)
                        fresh_start = False
                    elif aimage == "stored":
                        Z = blocks.last()[1].copy()
                    else:
                        Z = _spmm(Ab, blocks.last()[0], dtype)
                    if precond is not None:
                        # split preconditioning (Section 5): W = M^{-1} T(r)
                        # for a first block, W = M^{-1} A W_{j-1} after it
                        Z = precond(_f64(Z))
                    Z = _store(Z, dtype)
                    Z = cgs2_a(Z, *blocks.all(), dtype)
                    if trace is None:
                        W, AW, _ = orthonormalize(Ab, Z, dtype)
                    else:
                        tr = {"block": nblocks + 1, "iteration": k + 1}
                        trace.append(tr)
                        W, AW, _ = orthonormalize(Ab, Z, dtype, trace=tr)
                    blocks.add(W, AW)
                    V.append(W)
                    AV.append(AW)
                    nblocks += 1
                    m_since += 1
                    if stop_after_blocks is not None and nblocks >= stop_after_blocks:
                        res.extra["last_blocks"] = (V, AV)
                        res.x, res.iters, res.blocks = x, k, nblocks
                        return res
            except Breakdown as e:
                res.extra["breakdown"] = str(e)
                # READING: a breakdown after the first block since the last
                # (re)start restarts from the last completed iterate
                if restart_on_breakdown and m_since >= 1 and restarts < max_restarts:
                    r = true_residual(A, b, x)
                    rho = float(np.linalg.norm(r))
                    hist.append(rho)
                    restarts += 1
                    rho_restart = rho
                    fresh_start = True
                    blocks = new_store()
                    m_since = 0
                    continue
                status = BREAKDOWN
                break
            Vm = _f64(np.hstack(V))
            AVm = _f64(np.hstack(AV))
            alpha = Vm.T @ r
            x = x + Vm @ alpha
            r = r - AVm @ alpha
            rho = float(np.linalg.norm(r))
            k += 1
            hist.append(rho)
            if record:
                xs.append(x.copy())
                rs.append(r.copy())
                Vs.append((Vm, AVm))
                alphas.append(alpha)
        if status == BREAKDOWN:
            break
        if rho > thr:             # iteration budget exhausted
            status = MAXIT
            break
        rt = true_residual(A, b, x)
        tau = float(np.linalg.norm(rt))
        if trace is not None:
            trace.append({"replacement": restarts + 1, "x": x.copy(), "tau": tau})
        if tau <= thr_final:
            status = OK
            break
        if restarts >= max_restarts or k >= maxit:
            status = STAGNATED if k < maxit else MAXIT
            break
        r = rt
        rho = tau
        hist.append(tau)
        restarts += 1
        rho_restart = tau
        fresh_start = True
        blocks = new_store()
        m_since = 0
    res.x, res.iters, res.hist, res.status = x, k, hist, status
    res.restarts, res.blocks = restarts, nblocks
    res.true_relres = float(np.linalg.norm(b - A @ x)) / rho0
    if record:
        res.extra.update(xs=xs, rs=rs, V=Vs, alpha=alphas)
    return res


# ---------------------------------------------------------------------------
# Block Jacobi preconditioner with incomplete Cholesky blocks (Section 5,
# convergence experiments) and preconditioned CG
# ---------------------------------------------------------------------------

def ic0(A: sp.csr_matrix) -> sp.csr_matrix:
    """Incomplete Cholesky with zero fill-in: the lower triangular L with
    the sparsity pattern of the lower triangle of A such that (L L^t)_ij =
    A_ij for every (i, j) in that pattern, computed row by row:
      L_ij = (A_ij - sum_{k < j} L_ik L_jk) / L_jj   for j < i in the pattern,
      L_ii = sqrt(A_ii - sum_{k < i} L_ik^2),
    the sums running over the pattern.  Raises Breakdown if a pivot is <= 0
    or not finite.  Pure Python: small matrices only."""
    A = sp.csr_matrix(A)
    A.sort_indices()
    n = A.shape[0]
    rows: List[dict] = []
    for i in range(n):
        lo, hi = A.indptr[i], A.indptr[i + 1]
        row = {}
        aii = 0.0
        for p in range(lo, hi):
            j = int(A.indices[p])
            if j > i:
                break
            if j == i:
                aii = float(A.data[p])
                break
            rj = rows[j]
            acc = float(A.data[p])
            for k, v in row.items():
                if k < j and k in rj:
                    acc -= v * rj[k]
            row[j] = acc / rj[j]
        d = aii - sum(v * v for v in row.values())
        if not np.isfinite(d) or d <= 0.0:
            raise Breakdown(f"IC(0) pivot {i}: {d}")
        row[i] = math.sqrt(d)
        rows.append(row)
    indptr = np.zeros(n + 1, dtype=np.int64)
    cols, vals = [], []
    for i, row in enumerate(rows):
        ks = sorted(row)
        cols += ks
        vals += [row[k] for k in ks]
        indptr[i + 1] = len(cols)
    return sp.csr_matrix((np.array(vals), np.array(cols, dtype=np.int64), indptr), shape=(n, n))


def block_jacobi_ic0(A: sp.csr_matrix, blocks: np.ndarray) -> sp.csr_matrix:
    """L of the block Jacobi preconditioner M = L L^t whose diagonal blocks
    A(B_i, B_i) (rows with equal blocks[]) are factorised by IC(0)
    (Section 5: 64 blocks, incomplete Cholesky with zero fill-in).  Entries
    of A between different blocks are dropped first, so L is block
    diagonal, in the original row numbering."""
    A = sp.coo_matrix(A)
    blocks = np.asarray(blocks)
    keep = blocks[A.row] == blocks[A.col]
    Abd = sp.csr_matrix((A.data[keep], (A.row[keep], A.col[keep])), shape=A.shape)
    return ic0(Abd)


def block_jacobi_cholesky(A: sp.csr_matrix, blocks: np.ndarray) -> sp.csr_matrix:
    """L of the block Jacobi preconditioner M = L L^t whose diagonal blocks
    A(B_i, B_i) are factorised by complete Cholesky (Section 5, the
    complete-Cholesky table): per block, the dense Cholesky factor of the
    block (numpy), placed at the block's rows and columns.  L L^t equals the
    block-diagonal part of A."""
    A = sp.csr_matrix(A)
    blocks = np.asarray(blocks)
    rows, cols, vals = [], [], []
    for b in np.unique(blocks):
        idx = np.flatnonzero(blocks == b)
        Ab = A[idx][:, idx].toarray()
        Lb = np.linalg.cholesky(Ab)
        r, c = np.nonzero(np.tril(Lb))
        rows.append(idx[r])
        cols.append(idx[c])
        vals.append(Lb[r, c])
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=A.shape)


def apply_llt_inverse(L: sp.csr_matrix):
    """The map Z -> M^{-1} Z = L^{-t} (L^{-1} Z) for M = L L^t (two sparse
    triangular solves, the library routine as a step)."""
    from scipy.sparse.linalg import spsolve_triangular
    Lc = sp.csr_matrix(L)
    Ut = sp.csr_matrix(L.T)

    def minv(Z):
        Z = np.asarray(Z, dtype=np.float64)
        Y = spsolve_triangular(Lc, Z, lower=True)
        return spsolve_triangular(Ut, Y, lower=False)
    return minv


def pcg(A: sp.csr_matrix, b: np.ndarray, minv, x0=None, tol=1e-8, maxit=100000,
        record=False) -> SolveResult:
    """Preconditioned CG (the paper's preconditioned CG algorithm in
    Section 6, M = L L^t): z = M^{-1} r, p_1 = z_0, alpha = r^t z / p^t A p,
    beta = r_new^t z_new / r^t z, stopping on ||r_k|| <= tol ||r_0||.
    `minv` maps a vector (or n x 1 block) r to M^{-1} r."""
    def mv(v):
        return np.asarray(minv(v.reshape(-1, 1)), dtype=np.float64).reshape(-1)
    x = np.zeros_like(b) if x0 is None else x0.astype(np.float64).copy()
    r = b - A @ x
    rho0 = float(np.linalg.norm(r))
    hist = [rho0]
    xs = [x.copy()] if record else None
    if rho0 == 0.0:
        return SolveResult(x, 0, hist, OK, extra={"xs": xs})
    z = mv(r)
    p = z.copy()
    rz = float(r @ z)
    k = 0
    rho = rho0
    while rho > tol * rho0 and k < maxit:
        Ap = A @ p
        alpha = rz / float(p @ Ap)
        x = x + alpha * p
        r = r - alpha * Ap
        z = mv(r)
        rz_new = float(r @ z)
        p = z + (rz_new / rz) * p
        rz = rz_new
        rho = float(np.linalg.norm(r))
        k += 1
        hist.append(rho)
        if record:
            xs.append(x.copy())
    status = OK if rho <= tol * rho0 else MAXIT
    tr = float(np.linalg.norm(b - A @ x)) / rho0
    return SolveResult(x, k, hist, status, true_relres=tr, extra={"xs": xs})


# ---------------------------------------------------------------------------
# Dense references (small systems only)
# ---------------------------------------------------------------------------

def dense_cholesky_solve(Ad: np.ndarray, b: np.ndarray) -> np.ndarray:
    """x = A^{-1} b via A = L L^t and two triangular solves (A SPD, the
    paper's problem statement)."""
    L = np.linalg.cholesky(Ad)
    y = sla.solve_triangular(L, b, lower=True)
    return sla.solve_triangular(L.T, y, lower=False)


def sddmm(rowptr, colind, lam: np.ndarray, x: np.ndarray) -> np.ndarray:
    """Gradient of a loss through x = A^{-1} b with respect to the stored
    nonzeros of A: dL/dA_ij = -lambda_i x_j with A lambda = dL/dx, evaluated
    on the sparsity pattern (general-matrix convention; one value per stored
    entry, in storage order)."""
    rowptr = np.asarray(rowptr)
    rows = np.repeat(np.arange(rowptr.shape[0] - 1), np.diff(rowptr))
    return -lam[rows] * x[np.asarray(colind)]


def dense_gradient(Ad: np.ndarray, b: np.ndarray, x_tgt: np.ndarray):
    """Loss L = ||x - x_tgt||^2 with x = A^{-1} b: returns (x, dL/db, dL/dA)
    with dL/db = lambda = A^{-1} (2 (x - x_tgt)) and dL/dA = -lambda x^t
    (dense, every entry)."""
    x = dense_cholesky_solve(Ad, b)
    g = 2.0 * (x - x_tgt)
    lam = dense_cholesky_solve(Ad, g)
    return x, lam, -np.outer(lam, x)
