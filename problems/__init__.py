"""Seeded synthetic SPD test problems (inputs only).

This module builds the sparse symmetric positive definite systems the solver
is exercised on, and the seeded vectors that go with them.  It holds none of
the solver's arithmetic: no split operator, no basis construction, no
orthonormalization, no update.  Both the CPU oracle (through the tests) and
the GPU path (through the tests and the benchmark) consume what it produces,
byte for byte.

Matrices are cell-centred finite-difference / finite-volume diffusion
operators with homogeneous Dirichlet boundaries on an nx x ny (x nz) grid,
rows numbered ``i + nx*(j + ny*k)`` (x fastest).  For an interior face
between cells p and q along axis a the off-diagonal entry is ``-kf`` with
``kf`` the harmonic mean of the two cells' axis-a coefficients; a boundary
face contributes the cell's own coefficient to the diagonal.  With all
coefficients equal to one this is exactly MATLAB's ``gallery('poisson', m)``
used for the paper's Poisson2D matrix (Section 4, Table 1): diagonal 4 (2D)
or 6 (3D), off-diagonals -1.

Random numbers come from SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014) used as a counter-based
generator: value ``i`` of stream ``(seed, stream)`` is the SplitMix64 output
for state ``key + (i+1)*gamma`` where ``key`` is itself a SplitMix64 output
keyed by seed and stream.  Uniform doubles take the top 53 bits.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional, Tuple

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def _mix64(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output function (variant 13 finaliser), elementwise on uint64."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def splitmix64(seed: int, stream: int, idx: np.ndarray) -> np.ndarray:
    """Counter-based SplitMix64: 64-bit value number ``idx`` of stream (seed, stream)."""
    with np.errstate(over="ignore"):
        key = _mix64(np.uint64(seed) * GAMMA + np.uint64(stream))
        state = key + (np.asarray(idx, dtype=np.uint64) + np.uint64(1)) * GAMMA
    return _mix64(state)


def uniform01(seed: int, stream: int, n: int) -> np.ndarray:
    """n doubles in [0, 1): top 53 bits of the SplitMix64 stream times 2^-53."""
    h = splitmix64(seed, stream, np.arange(n, dtype=np.uint64))
    return (h >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def uniform_pm1(seed: int, stream: int, n: int) -> np.ndarray:
    """n doubles uniform in [-1, 1): 2u - 1."""
    return 2.0 * uniform01(seed, stream, n) - 1.0


# ---------------------------------------------------------------------------
# Coefficient fields
# ---------------------------------------------------------------------------

def kappa_constant(shape: Tuple[int, int, int], value: float = 1.0) -> np.ndarray:
    nx, ny, nz = shape
    return np.full(nx * ny * nz, value, dtype=np.float64)


def kappa_skyscraper(shape, seed: int, tile: int = 8, high: float = 1e5,
                     prob: float = 0.25) -> np.ndarray:
    """kappa = 1 except full-height columns of kappa = `high` on tile x tile
    cells of the xy plane; each xy tile is chosen with probability `prob`
    (stream 1 of `seed`)."""
    nx, ny, nz = shape
    tx, ty = -(-nx // tile), -(-ny // tile)
    u = uniform01(seed, 1, tx * ty).reshape(ty, tx)
    chosen = u < prob                                   # [ty, tx]
    i = np.arange(nx) // tile
    j = np.arange(ny) // tile
    plane = np.where(chosen[j][:, i], high, 1.0)        # [ny, nx]
    return np.broadcast_to(plane, (nz, ny, nx)).reshape(-1).astype(np.float64)


def kappa_loguniform(shape, seed: int, lo_exp: float = -3.0,
                     hi_exp: float = 3.0) -> np.ndarray:
    """kappa = 10^U(lo_exp, hi_exp) per cell (stream 1 of `seed`)."""
    nx, ny, nz = shape
    u = uniform01(seed, 1, nx * ny * nz)
    return 10.0 ** (lo_exp + (hi_exp - lo_exp) * u)


def kappa_random_blocks(shape, seed: int, block: int = 32,
                        max_exp: int = 6) -> np.ndarray:
    """block^3-cell blocks, kappa = 10^e with e uniform in {0..max_exp}
    (stream 1 of `seed`)."""
    nx, ny, nz = shape
    bx, by, bz = -(-nx // block), -(-ny // block), -(-nz // block)
    u = uniform01(seed, 1, bx * by * bz).reshape(bz, by, bx)
    e = np.minimum(np.floor(u * (max_exp + 1)), max_exp)
    i = np.arange(nx) // block
    j = np.arange(ny) // block
    k = np.arange(nz) // block
    ee = e[k][:, j][:, :, i]
    return (10.0 ** ee).reshape(-1)


# ---------------------------------------------------------------------------
# Stencil assembly
# ---------------------------------------------------------------------------

@dataclass
class Problem:
    name: str
    shape: Tuple[int, int, int]      # (nx, ny, nz); nz == 1 for 2D
    rowptr: np.ndarray               # int32 [n+1]
    colind: np.ndarray               # int32 [nnz]
    vals: np.ndarray                 # float64 [nnz]
    xstar: np.ndarray                # float64 [n]
    b: np.ndarray                    # float64 [n]  (= A @ xstar, row order)
    t: int = 1
    s: int = 1
    parts: Tuple[int, int, int] = (1, 1, 1)   # geometric domain counts (px, py, pz)
    tol: float = 1e-8
    seed: int = 0
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.rowptr.shape[0] - 1)

    @property
    def nnz(self) -> int:
        return int(self.colind.shape[0])

    def scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.vals, self.colind, self.rowptr), shape=(self.n, self.n))


def _harmonic(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    return 2.0 * a * b / (a + b)


def diffusion_csr(shape, kx: np.ndarray, ky: Optional[np.ndarray] = None,
                  kz: Optional[np.ndarray] = None):
    """Assemble the 5-point (nz == 1) or 7-point diffusion matrix in CSR with
    ascending column indices per row.  kx/ky/kz are per-cell coefficients
    along each axis (ky, kz default to kx)."""
    nx, ny, nz = shape
    n = nx * ny * nz
    ky = kx if ky is None else ky
    kz = kx if kz is None else kz
    dims = 3 if nz > 1 else 2
    K = {0: kx.reshape(nz, ny, nx), 1: ky.reshape(nz, ny, nx), 2: kz.reshape(nz, ny, nx)}
    idx = np.arange(n, dtype=np.int64).reshape(nz, ny, nx)
    diag = np.zeros((nz, ny, nx))
    # off-diagonal entries: lists of (row, col, value)
    rows, cols, vals = [], [], []
    for axis in range(dims):
        ax = 2 - axis                 # numpy axis: x -> 2, y -> 1, z -> 0
        k = K[axis]
        m = k.shape[ax]
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[ax] = slice(0, m - 1)
        hi[ax] = slice(1, m)
        kf = _harmonic(k[tuple(lo)], k[tuple(hi)])
        # interior faces: both cells get kf on the diagonal
        diag[tuple(lo)] += kf
        diag[tuple(hi)] += kf
        a, b = idx[tuple(lo)].ravel(), idx[tuple(hi)].ravel()
        rows += [a, b]
        cols += [b, a]
        vals += [-kf.ravel(), -kf.ravel()]
        # boundary faces (Dirichlet): the cell's own coefficient
        first = [slice(None)] * 3
        last = [slice(None)] * 3
        first[ax] = slice(0, 1)
        last[ax] = slice(m - 1, m)
        diag[tuple(first)] += k[tuple(first)]
        diag[tuple(last)] += k[tuple(last)]
    rows.append(idx.ravel())
    cols.append(idx.ravel())
    vals.append(diag.ravel())
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    v = np.concatenate(vals)
    order = np.lexsort((c, r))
    r, c, v = r[order], c[order], v[order]
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rowptr, r + 1, 1)
    rowptr = np.cumsum(rowptr)
    return rowptr.astype(np.int32), c.astype(np.int32), v.astype(np.float64)


def csr_matvec_rows(rowptr, colind, vals, x) -> np.ndarray:
    """b_i = sum_p vals[p] * x[colind[p]] over row i, products summed in
    storage order (used once per problem to form the right-hand side)."""
    prod = vals * x[colind]
    lens = np.diff(rowptr)
    out = np.zeros(rowptr.shape[0] - 1)
    # rows of a stencil have at most 7 entries: sum position by position so
    # the order within a row is the storage order
    start = rowptr[:-1].astype(np.int64)
    for q in range(int(lens.max()) if lens.size else 0):
        m = lens > q
        out[m] += prod[start[m] + q]
    return out


def make_problem(name: str, shape, kx, ky=None, kz=None, *, seed: int,
                 t: int, s: int, parts, tol: float = 1e-8,
                 rhs: str = "pm1") -> Problem:
    rowptr, colind, vals = diffusion_csr(shape, kx, ky, kz)
    n = rowptr.shape[0] - 1
    if rhs == "pm1":
        xstar = uniform_pm1(seed, 0, n)
    elif rhs == "unit":            # MATLAB-style rand in [0, 1)
        xstar = uniform01(seed, 0, n)
    else:
        raise ValueError(rhs)
    b = csr_matvec_rows(rowptr, colind, vals, xstar)
    return Problem(name, tuple(shape), rowptr, colind, vals, xstar, b, t=t, s=s,
                   parts=tuple(parts), tol=tol, seed=seed)


# ---------------------------------------------------------------------------
# The named workloads
# ---------------------------------------------------------------------------

def poisson2d(m: int = 100, *, seed: int = 1, t: int = 8, s: int = 2,
              parts=(2, 4, 1), tol: float = 1e-8, rhs: str = "pm1") -> Problem:
    """Poisson2D: gallery('poisson', m), the paper's Table 1 matrix for m = 100."""
    shape = (m, m, 1)
    return make_problem("poisson2d", shape, kappa_constant(shape), seed=seed, t=t,
                        s=s, parts=parts, tol=tol, rhs=rhs)


def skyscraper3d(m: int = 128, *, seed: int = 2, t: int = 16, s: int = 4,
                 parts=(4, 4, 1), tol: float = 1e-8) -> Problem:
    shape = (m, m, m)
    return make_problem("skyscraper3d", shape, kappa_skyscraper(shape, seed), seed=seed,
                        t=t, s=s, parts=parts, tol=tol)


def anisotropic3d(m: int = 128, *, seed: int = 3, t: int = 32, s: int = 4,
                  parts=(2, 4, 4), tol: float = 1e-8,
                  kappas=(1.0, 1e-2, 1e-4)) -> Problem:
    shape = (m, m, m)
    n = m ** 3
    kx = np.full(n, kappas[0])
    ky = np.full(n, kappas[1])
    kz = np.full(n, kappas[2])
    return make_problem("anisotropic3d", shape, kx, ky, kz, seed=seed, t=t, s=s,
                        parts=parts, tol=tol)


def loguniform2d(m: int = 1000, *, seed: int = 4, t: int = 16, s: int = 3,
                 parts=(4, 4, 1), tol: float = 1e-8) -> Problem:
    shape = (m, m, 1)
    p = make_problem("loguniform2d", shape, kappa_loguniform(shape, seed), seed=seed,
                     t=t, s=s, parts=parts, tol=tol)
    p.extra["x_tgt"] = uniform_pm1(seed, 2, p.n)
    return p


def randomblocks3d(m: int = 256, *, seed: int = 5, t: int = 64, s: int = 2,
                   parts=(4, 4, 4), tol: float = 1e-8, block: int = 32) -> Problem:
    shape = (m, m, m)
    return make_problem("randomblocks3d", shape, kappa_random_blocks(shape, seed, block),
                        seed=seed, t=t, s=s, parts=parts, tol=tol)


CONFIGS = {
    "C1": poisson2d,
    "C2": skyscraper3d,
    "C3": anisotropic3d,
    "C4": loguniform2d,
    "C5": randomblocks3d,
}


def stencil_nnz(shape) -> int:
    """Closed-form nonzero count of the 5/7-point stencil on `shape`."""
    nx, ny, nz = shape
    n = nx * ny * nz
    edges = (nx - 1) * ny * nz + nx * (ny - 1) * nz + (nx * ny * (nz - 1) if nz > 1 else 0)
    return n + 2 * edges
