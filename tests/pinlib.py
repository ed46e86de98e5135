"""Checks that pin the oracle to facts the paper and the mathematics fix.

Each function returns the largest violation it finds, so that a test can
assert both that the oracle passes and that a planted mistake does not.
"""
from __future__ import annotations

import math
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def read_poisson_table():
    """Rows of tests/golden/poisson2d_iterations.txt as {(table, t): [counts]}."""
    out = {}
    with open(os.path.join(GOLDEN, "poisson2d_iterations.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            parts = line.split()
            out[(parts[0], int(parts[1]))] = [int(v) for v in parts[2:]]
    return out


SVALS = [1, 2, 3, 4, 5, 8, 10]


def orthonormality_violation(res, A) -> float:
    """max_k ||V_k^t A V_k - I||_max over the recorded iterations, using a
    fresh product A V_k (not the stored A-images)."""
    worst = 0.0
    for V, _ in res.extra["V"]:
        G = V.T @ (A @ V)
        worst = max(worst, float(np.abs(G - np.eye(G.shape[0])).max()))
    return worst


def cross_block_violation(res, A) -> float:
    """max_k ||V_k^t A V_{k-1}||_max: consecutive s-step bases are
    A-orthogonal (SRE-CG keeps the last 2t vectors, which in exact
    arithmetic suffices for A-orthogonality to all earlier blocks)."""
    worst = 0.0
    Vs = res.extra["V"]
    for k in range(1, len(Vs)):
        worst = max(worst, float(np.abs(Vs[k][0].T @ (A @ Vs[k - 1][0])).max()))
    return worst


def petrov_galerkin_violation(res) -> float:
    """max_k ||V_k^t r_k|| / ||r_{k-1}|| with r the method's residual:
    r_k is orthogonal to the enlarged Krylov subspace (eqs (1)-(3))."""
    worst = 0.0
    rs = res.extra["rs"]
    for k, (V, _) in enumerate(res.extra["V"]):
        worst = max(worst, float(np.linalg.norm(V.T @ rs[k + 1]) / np.linalg.norm(rs[k])))
    return worst


def error_drop_violation(res, A, xstar, floor=1e-4) -> float:
    """With V^t A V = I and alpha = V^t r_{k-1} (eqs (1)-(3)),
    ||e_k||_A^2 = ||e_{k-1}||_A^2 - ||alpha_k||^2 for e = x* - x.  Returns
    the largest relative violation over iterations whose starting residual
    is above `floor` times the initial one (below that, cancellation in the
    energy difference dominates)."""
    worst = 0.0
    xs, rs = res.extra["xs"], res.extra["rs"]
    for k, a in enumerate(res.extra["alpha"]):
        if np.linalg.norm(rs[k]) < floor * np.linalg.norm(rs[0]):
            break
        e0 = xstar - xs[k]
        e1 = xstar - xs[k + 1]
        E0 = float(e0 @ (A @ e0))
        E1 = float(e1 @ (A @ e1))
        worst = max(worst, abs(E1 - (E0 - float(a @ a))) / E0)
    return worst


def monotone_energy_violation(res, A, xstar) -> float:
    """Largest increase of ||x* - x_k||_A relative to its predecessor."""
    worst = 0.0
    prev = None
    for x in res.extra["xs"]:
        e = xstar - x
        E = math.sqrt(float(e @ (A @ e)))
        if prev is not None:
            worst = max(worst, (E - prev) / prev)
        prev = E
    return worst


MSDO_SVALS = [1, 2, 3, 4, 5, 6, 7, 8, 10]


def read_msdo_table():
    """Rows of tests/golden/poisson2d_msdo_iterations.txt as
    {t: (msdo_cg, [s-step counts for MSDO_SVALS])}."""
    out = {}
    with open(os.path.join(GOLDEN, "poisson2d_msdo_iterations.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            v = [int(x) for x in line.split()]
            out[v[0]] = (v[1], v[2:])
    return out


CA_SVALS = [2, 3, 4, 5, 6, 7]


def read_ca_table():
    """Rows of tests/golden/poisson2d_ca_iterations.txt as
    {(table, t): [counts for CA_SVALS, as far as printed]}."""
    out = {}
    with open(os.path.join(GOLDEN, "poisson2d_ca_iterations.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            parts = line.split()
            out[(parts[0], int(parts[1]))] = [int(v) for v in parts[2:]]
    return out


# ---------------------------------------------------------------------------
# The binary32-basis precision form
# ---------------------------------------------------------------------------

def _blocks(trace):
    return [tr for tr in trace if "AZ" in tr]


def binary32_representability_violation(trace) -> int:
    """Number of entries of the recorded blocks (the CGS2 output Z handed to
    A-CholQR, A Z, W and A W) that are not binary32 values: in the precision
    form every stored block is a binary32 block."""
    bad = 0
    for tr in _blocks(trace):
        for key in ("Z", "AZ", "W", "AW"):
            v = np.asarray(tr[key], dtype=np.float64)
            bad += int(np.count_nonzero(v.astype(np.float32).astype(np.float64) != v))
    return bad


def basis_product_rounding_violation(trace, A32_dense) -> float:
    """max |A Z - P| / ulp32(P) over the recorded blocks, where P is the
    product of the binary32-rounded matrix with Z formed as a dense product
    (products of binary32 values are exact in binary64; the binary64 sum is
    far more accurate than a binary32 ulp).  A Z rounded to nearest from
    that product gives at most 0.5."""
    worst = 0.0
    for tr in _blocks(trace):
        P = A32_dense @ np.asarray(tr["Z"], dtype=np.float64)
        got = np.asarray(tr["AZ"], dtype=np.float64)
        ulp = np.spacing(np.abs(P).astype(np.float32)).astype(np.float64)
        worst = max(worst, float((np.abs(got - P) / ulp).max()))
    return worst


def gram_accuracy_violation(trace) -> float:
    """max over the recorded Grams G = Z^t (A Z) of |G - G_exact| in units of
    the binary64 summation bound n * 2^-53 * (|Z|^t |A Z|), with G_exact the
    correctly rounded exact sum (math.fsum of products that are exact, both
    factors being binary32 values).  A Gram accumulated in binary64 gives at
    most 1; one accumulated in binary32 gives about 2^29 / n."""
    worst = 0.0
    for tr in _blocks(trace):
        Z = np.asarray(tr["Z"], dtype=np.float64)
        AZ = np.asarray(tr["AZ"], dtype=np.float64)
        G = np.asarray(tr["G"], dtype=np.float64)
        n, t = Z.shape
        absb = np.abs(Z).T @ np.abs(AZ)
        for i in range(t):
            for j in range(i, t):
                exact = math.fsum(Z[:, i] * AZ[:, j])
                bound = n * 2.0 ** -53 * absb[i, j]
                if bound > 0:
                    worst = max(worst, abs(G[i, j] - exact) / bound)
                elif G[i, j] != exact:
                    worst = float("inf")
    return worst
