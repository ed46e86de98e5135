"""Writes the full-size oracle references used by tests/test_gpu_fullsize.py.

Calls only oracle/ and problems/ (no GPU code).  For a configuration it runs
the float64 oracle of s-step SRE-CG on the exact problem the GPU tests
solve, and stores: iteration count, status, restarts, the residual history,
the true relative residual, the 2-norm of x, and x at SAMPLES seeded row
indices (the tests compare the GPU solution there: a sampled estimate of
||x - x_oracle|| / ||x_oracle||).  Ensemble members solve b perturbed by
about one part in 1e15 (tests/parity.py); their counts and sampled spreads
bound the criterion in the rounding-sensitive regime.

Usage: python tests/golden/make_fullsize.py CFG [--member K]
       python tests/golden/make_fullsize.py CFG --merge
Member 0 is the unperturbed solve.  The merged file is
tests/golden/fullsize_<cfg>.npz.
"""
from __future__ import annotations

import argparse
import glob
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402
import problems as P  # noqa: E402

SAMPLES = 1 << 16


def sample_rows(n: int) -> np.ndarray:
    """SAMPLES distinct row indices from a seeded generator (sorted)."""
    rng = np.random.default_rng(20260101)
    return np.sort(rng.choice(n, size=min(SAMPLES, n), replace=False)).astype(np.int64)


def member(cfg: str, k: int) -> str:
    p = P.CONFIGS[cfg]()
    A = p.scipy()
    dom = O.partition_grid(p.shape, p.parts)
    b = p.b
    if k > 0:
        rng = np.random.default_rng(k)
        b = b * (1.0 + 1e-15 * rng.standard_normal(b.shape[0]))
    t0 = time.time()
    r = O.sstep_srecg(A, dom, p.t, p.s, b, tol=p.tol, maxit=30000)
    idx = sample_rows(p.n)
    out = os.path.join(HERE, f"_fullsize_{cfg}_m{k}.npz")
    np.savez(out, iters=r.iters, status=r.status, restarts=r.restarts,
             hist=np.asarray(r.hist), true_relres=r.true_relres,
             xnorm=np.linalg.norm(r.x), idx=idx, xs=r.x[idx], seconds=time.time() - t0)
    print(f"{cfg} member {k}: {r.iters} iterations, status {r.status}, "
          f"true relres {r.true_relres:.2e}, {time.time() - t0:.0f} s", flush=True)
    return out


def merge(cfg: str) -> str:
    files = sorted(glob.glob(os.path.join(HERE, f"_fullsize_{cfg}_m*.npz")),
                   key=lambda f: int(f.rsplit("_m", 1)[1][:-4]))
    ms = [dict(np.load(f)) for f in files]
    ref = ms[0]
    iters = np.array([int(m["iters"]) for m in ms])
    xs = np.array([m["xs"] for m in ms])
    spread = max(float(np.linalg.norm(x - ref["xs"]) / np.linalg.norm(ref["xs"])) for x in xs)
    # each member's sampled error against the exact solution x* of b = A x*
    xstar = P.CONFIGS[cfg]().xstar[ref["idx"]]
    err = np.array([float(np.linalg.norm(x - xstar) / np.linalg.norm(xstar)) for x in xs])
    out = os.path.join(HERE, f"fullsize_{cfg}.npz")
    np.savez_compressed(out, iters=ref["iters"], status=ref["status"], restarts=ref["restarts"],
                        hist=ref["hist"], true_relres=ref["true_relres"], xnorm=ref["xnorm"],
                        idx=ref["idx"], xs=ref["xs"], ens_iters=iters, ens_spread2=spread,
                        ens_err_xstar=err, seconds=np.array([float(m["seconds"]) for m in ms]))
    print(f"{cfg}: members {iters.tolist()}, sampled 2-norm spread {spread:.2e}, "
          f"sampled error vs x* {err.min():.2e} .. {err.max():.2e} -> {out}")
    return out


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("cfg")
    ap.add_argument("--member", type=int, default=0)
    ap.add_argument("--merge", action="store_true")
    a = ap.parse_args()
    if a.merge:
        merge(a.cfg)
    else:
        member(a.cfg, a.member)
