"""MI355X-native s-step enlarged Conjugate Gradient (SRE-CG family).

Thin Python binding over the C ABI of ``libecg.so`` (declared in
``include/ecg.h``).  Every step of the solve runs in the library's HIP
kernels; this module only marshals arguments: it hands the library device
pointers of torch tensors (torch is used for device memory and streams) or
host numpy arrays.  If the library has not been built the import fails.

Method: Moufawad, "Numerical Stability of s-step Enlarged Krylov Subspace
Conjugate Gradient methods", arXiv 1804.10629, Section 3.1.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

# torch first: its libraries bring their own libamdhip64; loading libecg.so
# after it binds the library to that same HIP runtime instead of a second
# copy (two runtimes in one process do not share the device)
import torch  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
# always the in-tree build (paper_1804_10629_amd/build.py)
LIB_PATH = os.path.join(_HERE, "libecg.so")

OK, MAXIT, BREAKDOWN, STAGNATED = 0, 1, 2, 3
EINVAL, ENOMEM, EDEVICE, ENOTSUP = -1, -2, -3, -4
SRECG, SRECG2, MSDO = 0, 1, 2
ACHOLQR, PRECHOLQR = 0, 1
FP64, MIXED = 0, 1
KCLASSES = ["resid", "tsplit", "cgs_gram", "cgs_update", "spmm", "xr_update", "gram",
            "update", "small", "precond"]
PREC_NONE, PREC_BJ_IC0, PREC_BJ_CHOL = 0, 1, 2
CA_NONE, CA_MODIFIED, CA_PLAIN = 0, 1, 2   # opts.ca: s-step, modified / plain CA-Arnoldi
SPMM_NOALLOC_MAX = 4194304   # n x padded width limit of ecg_spmm_noalloc


class EcgError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"ecg error {code}: {msg}")
        self.code = code


class _Opts(ctypes.Structure):
    _fields_ = [
        ("variant", ctypes.c_int32), ("orth", ctypes.c_int32),
        ("precision", ctypes.c_int32), ("device_ptrs", ctypes.c_int32),
        ("inner_tol", ctypes.c_double), ("max_restarts", ctypes.c_int32),
        ("q_cap_blocks", ctypes.c_int32), ("ws_cap_bytes", ctypes.c_int64),
        ("hip_stream", ctypes.c_void_p), ("collect_stats", ctypes.c_int32),
        ("grid", ctypes.c_int32), ("progress_every", ctypes.c_int32),
        ("permute_domains", ctypes.c_int32), ("ca", ctypes.c_int32),
        ("reserved", ctypes.c_int32 * 1), ("row_key", ctypes.c_void_p),
    ]


class _Result(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int32), ("iters", ctypes.c_int32),
        ("hist_len", ctypes.c_int32), ("restarts", ctypes.c_int32),
        ("blocks", ctypes.c_int32), ("reserved", ctypes.c_int32),
        ("rho0", ctypes.c_double), ("relres", ctypes.c_double),
        ("true_relres", ctypes.c_double), ("solve_ms", ctypes.c_double),
    ]


class _Stats(ctypes.Structure):
    _fields_ = [
        ("launches", ctypes.c_int64 * 10), ("ms", ctypes.c_double * 10),
        ("bytes", ctypes.c_double * 10), ("flops", ctypes.c_double * 10),
    ]


_P = ctypes.c_void_p
_SIGS = {
    "ecg_opts_default": (None, [ctypes.POINTER(_Opts)]),
    "ecg_version": (ctypes.c_char_p, []),
    "ecg_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "ecg_last_error": (ctypes.c_char_p, []),
    "ecg_kclass_name": (ctypes.c_char_p, [ctypes.c_int]),
    "ecg_partition_grid": (ctypes.c_int, [ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                                          ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _P, _P]),
    "ecg_grid_morton_keys": (ctypes.c_int, [ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, _P]),
    "ecg_setup": (ctypes.c_int, [ctypes.POINTER(_P), ctypes.c_int64, _P, _P, _P, _P,
                                 ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(_Opts)]),
    "ecg_solve": (ctypes.c_int, [_P, _P, _P, ctypes.c_double, ctypes.c_int32, _P, _P, _P,
                                 _P]),
    "ecg_solve_ex": (ctypes.c_int, [_P, _P, _P, ctypes.c_double, ctypes.c_int32, _P,
                                    ctypes.c_int32, ctypes.POINTER(_Result)]),
    "ecg_sddmm": (ctypes.c_int, [_P, _P, _P, _P]),
    "ecg_spmm": (ctypes.c_int, [_P, _P, _P, ctypes.c_int32]),
    "ecg_spmm_noalloc": (ctypes.c_int, [_P, _P, _P, ctypes.c_int32]),
    "ecg_tsplit": (ctypes.c_int, [_P, _P, _P]),
    "ecg_get_basis": (ctypes.c_int, [_P, _P, _P]),
    "ecg_last_stats": (ctypes.c_int, [_P, ctypes.POINTER(_Stats)]),
    "ecg_domain_order": (ctypes.c_int, [_P, _P]),
    "ecg_set_preconditioner": (ctypes.c_int, [_P, ctypes.c_int32, _P]),
    "ecg_destroy": (None, [_P]),
}

_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libecg.so (once).  Raises ImportError if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(
            f"{path} is missing: build it with `python -m paper_1804_10629_amd.build` "
            "(there is no fallback implementation)")
    lib = ctypes.CDLL(path)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


lib = load_library()


def version() -> str:
    return lib.ecg_version().decode()


def strerror(code: int) -> str:
    return lib.ecg_strerror(code).decode()


def _check(code: int) -> int:
    if code < 0:
        raise EcgError(code, f"{strerror(code)}: {lib.ecg_last_error().decode()}")
    return code


# ---------------------------------------------------------------------------
# argument marshalling
# ---------------------------------------------------------------------------

def _torch():
    import torch
    return torch


def _is_tensor(a) -> bool:
    try:
        import torch
        return isinstance(a, torch.Tensor)
    except ImportError:
        return False


def _dev_tensor(a, dtype):
    """A contiguous CUDA tensor of `dtype` holding `a` (no copy if it already is one)."""
    torch = _torch()
    if isinstance(a, torch.Tensor):
        t = a.detach()
        if t.device.type != "cuda" or t.dtype != dtype or not t.is_contiguous():
            t = t.to(device="cuda", dtype=dtype).contiguous()
        return t
    return torch.as_tensor(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def _stream_ptr() -> int:
    torch = _torch()
    return int(torch.cuda.current_stream().cuda_stream)


def partition_grid(shape: Sequence[int], parts: Sequence[int]):
    """Geometric box decomposition of a grid (GPU kernel); int32 CUDA tensor."""
    torch = _torch()
    nx, ny, nz = (int(v) for v in shape)
    px, py, pz = (int(v) for v in parts)
    dom = torch.empty(nx * ny * nz, dtype=torch.int32, device="cuda")
    _check(lib.ecg_partition_grid(nx, ny, nz, px, py, pz, dom.data_ptr(), _stream_ptr()))
    return dom


def grid_morton_keys(shape: Sequence[int]) -> np.ndarray:
    """Morton keys of a grid's cells (host int64 array), for Solver(row_key=)."""
    nx, ny, nz = (int(v) for v in shape)
    keys = np.empty(nx * ny * nz, dtype=np.int64)
    _check(lib.ecg_grid_morton_keys(nx, ny, nz, keys.ctypes.data))
    return keys


@dataclass
class SolveInfo:
    status: int
    iters: int
    restarts: int
    blocks: int
    rho0: float
    relres: float
    true_relres: float
    solve_ms: float
    hist: np.ndarray

    @property
    def converged(self) -> bool:
        return self.status == OK


class Solver:
    """s-step SRE-CG / SRE-CG2 / MSDO-CG solver (ca=True: their CA forms)
    for one sparse SPD matrix on the GPU.

    rowptr/colind/vals: CSR (int32, int32, float64), numpy arrays or torch
    tensors; partition: int32 domain index per row in [0, t).  Inputs are
    copied to the device by the library (as CUDA tensors, device_ptrs=1).
    row_key: optional int64 per row; the rows of each domain are then stored
    by ascending key (grid_morton_keys gives the Morton order of a grid).
    """

    def __init__(self, rowptr, colind, vals, partition, t: int, s: int, *,
                 variant: int = SRECG, orth: int = ACHOLQR, precision: int = FP64,
                 inner_tol: float = 1e-4, max_restarts: int = 20, q_cap_blocks: int = 0,
                 ws_cap_bytes: int = 0, collect_stats: bool = False, grid: int = 0,
                 progress_every: int = 0, permute_domains: bool = True,
                 ca: int = CA_NONE, precond_blocks=None, row_key=None):
        torch = _torch()
        self._ctx = _P()
        o = _Opts()
        lib.ecg_opts_default(ctypes.byref(o))
        o.variant, o.orth, o.precision = variant, orth, precision
        o.device_ptrs = 1
        o.inner_tol, o.max_restarts, o.q_cap_blocks = inner_tol, max_restarts, q_cap_blocks
        o.ws_cap_bytes, o.collect_stats, o.grid = ws_cap_bytes, int(collect_stats), grid
        o.progress_every = progress_every
        o.permute_domains = int(permute_domains)
        o.ca = int(ca)
        o.hip_stream = _stream_ptr()
        self.opts = o
        rp = _dev_tensor(rowptr, torch.int32)
        ci = _dev_tensor(colind, torch.int32)
        va = _dev_tensor(vals, torch.float64)
        pd = _dev_tensor(partition, torch.int32)
        rk = _dev_tensor(row_key, torch.int64) if row_key is not None else None
        o.row_key = rk.data_ptr() if rk is not None else None
        self.n = int(rp.numel() - 1)
        self.nnz = int(ci.numel())
        self.t, self.s = int(t), int(s)
        _check(lib.ecg_setup(ctypes.byref(self._ctx), self.n, rp.data_ptr(), ci.data_ptr(),
                             va.data_ptr(), pd.data_ptr(), self.t, self.s, ctypes.byref(o)))
        o.row_key = None   # the library keeps its own order; the key tensor may go
        if precond_blocks is not None:
            self.set_preconditioner(PREC_BJ_IC0, precond_blocks)

    def set_preconditioner(self, kind: int, blocks=None):
        """Block Jacobi IC(0) preconditioner with blocks[i] the block of row i
        (kind PREC_BJ_IC0), or none (PREC_NONE)."""
        torch = _torch()
        bd = _dev_tensor(blocks, torch.int32) if blocks is not None else None
        _check(lib.ecg_set_preconditioner(self._ctx, int(kind),
                                          bd.data_ptr() if bd is not None else None))

    def close(self):
        if getattr(self, "_ctx", None) and self._ctx.value:
            lib.ecg_destroy(self._ctx)
            self._ctx = _P()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve(self, b, x0=None, tol: float = 1e-8, maxit: int = 10000):
        """Returns (x as a float64 CUDA tensor, SolveInfo)."""
        torch = _torch()
        bd = _dev_tensor(b, torch.float64)
        if x0 is None:
            x = torch.zeros(self.n, dtype=torch.float64, device="cuda")
        else:
            x = _dev_tensor(x0, torch.float64).clone()
        # rho_0, one norm per iteration, one per restart (residual replacements
        # are bounded by max_restarts, SRE-CG2 block-cap restarts by maxit)
        cap = 2 * maxit + self.opts.max_restarts + 4
        hist = np.zeros(cap, dtype=np.float64)
        res = _Result()
        code = lib.ecg_solve_ex(self._ctx, bd.data_ptr(), x.data_ptr(), float(tol), int(maxit),
                             hist.ctypes.data, cap, ctypes.byref(res))
        _check(code)
        info = SolveInfo(code, res.iters, res.restarts, res.blocks, res.rho0, res.relres,
                         res.true_relres, res.solve_ms, hist[:res.hist_len].copy())
        return x, info

    def sddmm(self, lam, x):
        """-lambda[row(p)] * x[col(p)] for every stored entry p (CUDA tensor)."""
        torch = _torch()
        ld = _dev_tensor(lam, torch.float64)
        xd = _dev_tensor(x, torch.float64)
        out = torch.empty(self.nnz, dtype=torch.float64, device="cuda")
        _check(lib.ecg_sddmm(self._ctx, ld.data_ptr(), xd.data_ptr(), out.data_ptr()))
        return out

    def spmm(self, X):
        """A X for an n x k float64 block (k <= 64)."""
        torch = _torch()
        Xd = _dev_tensor(X, torch.float64)
        k = 1 if Xd.dim() == 1 else int(Xd.shape[1])
        Y = torch.empty_like(Xd)
        _check(lib.ecg_spmm(self._ctx, Xd.data_ptr(), Y.data_ptr(), k))
        return Y

    def spmm_noalloc(self, X, out):
        """A X into the preallocated n x k float64 CUDA tensor `out`, through
        ecg_spmm_noalloc (no device allocation inside the call; n times the
        padded width of k must not exceed SPMM_NOALLOC_MAX)."""
        torch = _torch()
        if not (X.is_cuda and X.dtype == torch.float64 and X.is_contiguous()):
            raise ValueError("X must be a contiguous float64 CUDA tensor")
        if not (out.is_cuda and out.dtype == torch.float64 and out.is_contiguous()
                and out.shape == X.shape):
            raise ValueError("out must be a contiguous float64 CUDA tensor shaped like X")
        k = 1 if X.dim() == 1 else int(X.shape[1])
        _check(lib.ecg_spmm_noalloc(self._ctx, X.data_ptr(), out.data_ptr(), k))
        return out

    def tsplit(self, r):
        """T(r) as an n x t float64 CUDA tensor."""
        torch = _torch()
        rd = _dev_tensor(r, torch.float64)
        Z = torch.empty((self.n, self.t), dtype=torch.float64, device="cuda")
        _check(lib.ecg_tsplit(self._ctx, rd.data_ptr(), Z.data_ptr()))
        return Z

    def basis(self):
        """(V, AV) of the last completed s-step iteration, n x (s t) each."""
        torch = _torch()
        V = torch.empty((self.n, self.s * self.t), dtype=torch.float64, device="cuda")
        AV = torch.empty_like(V)
        _check(lib.ecg_get_basis(self._ctx, V.data_ptr(), AV.data_ptr()))
        return V, AV

    def domain_order(self):
        """order[i]: the caller's row stored as solver row i (int32 CUDA tensor)."""
        torch = _torch()
        out = torch.empty(self.n, dtype=torch.int32, device="cuda")
        _check(lib.ecg_domain_order(self._ctx, out.data_ptr()))
        return out

    def stats(self) -> dict:
        st = _Stats()
        _check(lib.ecg_last_stats(self._ctx, ctypes.byref(st)))
        return {name: {"launches": st.launches[i], "ms": st.ms[i], "bytes": st.bytes[i],
                       "flops": st.flops[i]} for i, name in enumerate(KCLASSES)}


from .autograd import ECGSolve, solve_with_grad  # noqa: E402,F401
