"""Benchmark of the s-step enlarged CG hot path on one MI355X (gfx950).

Workload (default, --config C5): heterogeneous 3D diffusion, 7-point stencil
on a 256^3 grid (n = 16,777,216, nnz = 117,047,296), kappa = 10^e on 32^3-cell
blocks with e uniform in {0..6}, t = 64 box domains (4 x 4 x 4), s = 2,
s-step SRE-CG (the short-recurrence variant), x* uniform in [-1, 1],
b = A x*, x0 = 0, tolerance 1e-8 on the relative residual.  Inputs are
resident in HBM before any timed region starts.

One step = one s-step iteration of the solve: s blocks (CGS2 against the two
previous blocks, the sparse product with its Gram epilogue, A-CholQR), the
x/r update and the residual norm.  W untimed steps (a solve stopped after W
iterations), then K timed steps (a solve from x0 stopped after K iterations,
bracketed by device synchronisations), with per-kernel timing switched off.
value = HBM GB/s of those K iterations: the algorithmic bytes of every kernel
they launch (operand bytes per launch, counted by the library) over the
measured wall time.  The same is measured for the binary32-basis precision
form.

Time-to-1e-8 of the full solve: at 256^3 the unpreconditioned solve takes
about ten thousand s-step iterations (712 s FP64, 547 s mixed), so it is
measured by `python bench.py --full --form fp64|mixed` (progress on stderr)
and committed under profiles/; every run measures the full time-to-1e-8 of the same 256^3 system
with the split preconditioned method of Section 5 (block Jacobi, IC(0)
blocks = the 64 domains; about sixty iterations) in both forms, and of the
128^3 skyscraper problem (t = 16, s = 4; seconds) in both forms as the
`skyscraper_128` key.

Extra keys: the kernel table and roofline of the dominant kernel (from a
separate solve with per-kernel HIP events on the solver's stream), and the
CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "time-to-1e-8 rel-residual + SpMM/block HBM GB/s; FP32-mixed vs FP64 solve"
PEAK_HBM_GBS = 8000.0          # MI355X HBM3E
PEAK_F64_MFMA_TFS = 78.6       # MI355X dense FP64 matrix
KERNEL_SOURCE = os.path.join(ROOT, "paper_1804_10629_amd", "csrc", "ecg_kernels.hip")
PROFILES = os.path.join(ROOT, "profiles")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def build_problem(cfg: str):
    import problems as P
    return P.CONFIGS[cfg]()


def describe(p) -> str:
    nx, ny, nz = p.shape
    grid = f"{nx}x{ny}" if nz == 1 else f"{nx}x{ny}x{nz}"
    return (f"{p.name} {grid} (n={p.n}, nnz={p.nnz}), s-step SRE-CG t={p.t} s={p.s}, "
            f"tol {p.tol:g}")


def kernel_table(stats):
    out = {}
    for name, v in stats.items():
        if v["launches"] == 0:
            continue
        ms = v["ms"]
        out[name] = {
            "launches": int(v["launches"]),
            "ms_total": round(ms, 3),
            "us_per_launch": round(1e3 * ms / v["launches"], 2),
            "gb_per_launch": round(v["bytes"] / v["launches"] / 1e9, 4),
            "gflop_per_launch": round(v.get("flops", 0.0) / v["launches"] / 1e9, 3),
            "gbs": round(v["bytes"] / (ms * 1e-3) / 1e9, 1) if ms > 0 else None,
        }
    return out


def kernel_source_hash():
    with open(KERNEL_SOURCE, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic(kclass, workload, form="fp64", row_order="domain"):
    """HBM bytes per launch of a kernel class from a committed rocprofv3
    --pmc summary (FETCH_SIZE and WRITE_SIZE, scaled against a plain copy),
    or None when no summary matches this workload, form, row order and
    kernel source."""
    src = kernel_source_hash()
    if not os.path.isdir(PROFILES):
        return None
    for name in sorted(os.listdir(PROFILES)):
        if not name.endswith(".md"):
            continue
        with open(os.path.join(PROFILES, name)) as f:
            for line in f:
                m = re.match(r"^traffic_json: (\{.*\})\s*$", line)
                if not m:
                    continue
                d = json.loads(m.group(1))
                if (d.get("kclass") == kclass and d.get("workload") == workload
                        and d.get("form", "fp64") == form
                        and d.get("row_order", "domain") == row_order
                        and d.get("kernel_source_sha256_16") == src):
                    return d
    return None


def roofline(ktab, workload, form, row_order="domain"):
    """The dominant kernel class (device time) against its binding peak:
    FP64 matrix cores when its flops at 78.6 TFLOP/s take longer than its
    bytes at 8 TB/s, HBM otherwise."""
    name = max(ktab, key=lambda k: ktab[k]["ms_total"])
    k = ktab[name]
    sec = k["us_per_launch"] * 1e-6
    t_mem = k["gb_per_launch"] / PEAK_HBM_GBS
    t_mfma = k["gflop_per_launch"] / (PEAK_F64_MFMA_TFS * 1e3)
    tr = measured_traffic(name, workload, form, row_order)
    common = {"kernel": name, "algorithmic_gb_per_launch": k["gb_per_launch"],
              "gflop_per_launch": k["gflop_per_launch"],
              "traffic": tr["hbm_gb_per_launch"] if tr else None,
              "traffic_unit": "GB per launch (FETCH_SIZE + WRITE_SIZE, copy-scaled)",
              "traffic_vs_algorithmic": (round(tr["hbm_gb_per_launch"] / k["gb_per_launch"], 3)
                                         if tr else None),
              "traffic_source": tr["file"] if tr else None}
    if t_mfma > t_mem:
        ach = k["gflop_per_launch"] / sec / 1e3
        return {"bound": "mfma", "achieved": round(ach, 2), "peak": PEAK_F64_MFMA_TFS,
                "unit": "TFLOP/s", "frac": round(ach / PEAK_F64_MFMA_TFS, 4),
                "hbm_gbs": round(k["gb_per_launch"] / sec, 1), **common}
    ach = k["gb_per_launch"] / sec
    return {"bound": "hbm", "achieved": round(ach, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": round(ach / PEAK_HBM_GBS, 4),
            "tflops": round(k["gflop_per_launch"] / sec / 1e3, 2), **common}


def host_info():
    info = {"nproc": os.cpu_count()}
    try:
        info["nproc"] = int(subprocess.run(["nproc"], capture_output=True, text=True,
                                           timeout=10).stdout.strip())
    except Exception:
        pass
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        m = re.search(r"Model name:\s*(.+)", out)
        if m:
            info["cpu_model"] = m.group(1).strip()
    except Exception:
        pass
    try:
        with open("/proc/meminfo") as f:
            m = re.search(r"MemTotal:\s*(\d+) kB", f.read())
            if m:
                info["mem_total_gb"] = round(int(m.group(1)) / 1e6, 1)
    except Exception:
        pass
    return info


def blas_threads():
    try:
        from threadpoolctl import threadpool_info
        return max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    except Exception:
        return int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))


def cpu_baseline(p, gpu_bytes_per_iter):
    """The CPU oracle (as it stands) on the same problem, stopped after its
    first basis block, timed; extrapolated to an s-step iteration (s blocks)
    and expressed in the metric's unit with the GPU's bytes per iteration.
    The first block has no CGS2 step, so this underestimates the oracle's
    time per iteration."""
    import oracle as O
    A = p.scipy()
    dom = O.partition_grid(p.shape, p.parts)
    t0 = time.perf_counter()
    r = O.sstep_srecg(A, dom, p.t, p.s, p.b, tol=p.tol, maxit=1, stop_after_blocks=1)
    dt = time.perf_counter() - t0
    per_iter = dt * p.s / max(r.blocks, 1)
    hi = host_info()
    one_core = None
    try:
        from threadpoolctl import threadpool_limits
        with threadpool_limits(limits=1):
            t1 = time.perf_counter()
            O.sstep_srecg(A, dom, p.t, p.s, p.b, tol=p.tol, maxit=1, stop_after_blocks=1)
            dt1 = time.perf_counter() - t1
        per1 = dt1 * p.s / max(r.blocks, 1)
        one_core = {"value": round(gpu_bytes_per_iter / per1 / 1e9, 3), "unit": "GB/s",
                    "cores": 1, "s_per_iteration": round(per1, 2),
                    "sample": "the same first block with the BLAS pool limited to one thread"}
    except ImportError:
        pass
    return {
        "value": round(gpu_bytes_per_iter / per_iter / 1e9, 3),
        "unit": "GB/s",
        "cores": blas_threads(),
        "kind": "oracle",
        "sample": (f"oracle (numpy/scipy, float64) on the same {'x'.join(map(str, p.shape))} problem stopped "
                   f"after its first basis block ({dt:.1f} s: T(r), the sparse product, the "
                   f"Gram, Cholesky, two triangular solves); x {p.s} blocks = {per_iter:.1f} s "
                   f"per s-step iteration (an underestimate: later blocks add CGS2), over the "
                   f"GPU's algorithmic bytes per iteration; BLAS threads as 'cores', the "
                   f"sparse product single-threaded"),
        "s_per_iteration": round(per_iter, 2),
        "one_core": one_core,
        "host": hi,
    }


def c1_full_solves(E):
    """Time-to-1e-8 of the 100^2 Poisson problem (t = 8, s = 2) by the CPU
    oracle on all BLAS threads and on one, and by the GPU (FP64)."""
    import torch
    import oracle as O
    p = build_problem("C1")
    A = p.scipy()
    dom = O.partition_grid(p.shape, p.parts)
    out = {"workload": describe(p)}
    t0 = time.perf_counter()
    r = O.sstep_srecg(A, dom, p.t, p.s, p.b, tol=p.tol)
    out["oracle_all_threads"] = {"time_s": round(time.perf_counter() - t0, 3), "iters": r.iters,
                                 "threads": blas_threads()}
    try:
        from threadpoolctl import threadpool_limits
        with threadpool_limits(limits=1):
            t0 = time.perf_counter()
            r1 = O.sstep_srecg(A, dom, p.t, p.s, p.b, tol=p.tol)
            out["oracle_one_thread"] = {"time_s": round(time.perf_counter() - t0, 3),
                                        "iters": r1.iters, "threads": 1}
    except ImportError:
        pass
    _, g = full_solve(E, p, device_arrays(E, p), E.FP64, 10000, "C1 fp64")
    out["gpu_fp64"] = g
    torch.cuda.empty_cache()
    return out


def device_arrays(E, p):
    import torch
    dom = E.partition_grid(p.shape, p.parts)
    rp = torch.as_tensor(p.rowptr).cuda()
    ci = torch.as_tensor(p.colind).cuda()
    va = torch.as_tensor(p.vals).cuda()
    bd = torch.as_tensor(p.b).cuda()
    return rp, ci, va, dom, bd


def iteration_form(E, p, arrs, precision, steps, warmup, form, **opts):
    """W untimed and K timed s-step iterations, then a separate K-iteration
    solve with per-kernel events for the kernel table (`opts`: further
    Solver options, e.g. the row order)."""
    import torch
    rp, ci, va, dom, bd = arrs
    t0 = time.perf_counter()
    sol = E.Solver(rp, ci, va, dom, p.t, p.s, precision=precision, **opts)
    torch.cuda.synchronize()
    log(f"[{form}] setup {time.perf_counter() - t0:.1f} s")
    if warmup > 0:
        _, wi = sol.solve(bd, tol=p.tol, maxit=warmup)
        log(f"[{form}] warmup: {wi.iters} iterations, rho/rho0 {wi.relres:.2e}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x, info = sol.solve(bd, tol=p.tol, maxit=steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    log(f"[{form}] timed: {info.iters} iterations in {wall * 1e3:.1f} ms, "
        f"rho/rho0 {info.relres:.2e}")
    sol.close()
    st = E.Solver(rp, ci, va, dom, p.t, p.s, precision=precision, collect_stats=True, **opts)
    _, si = st.solve(bd, tol=p.tol, maxit=steps)
    stats = st.stats()
    st.close()
    total_bytes = sum(v["bytes"] for v in stats.values())
    return {"iters": info.iters, "wall_s": wall, "ms_per_step": wall * 1e3 / max(info.iters, 1),
            "relres": info.relres, "bytes": total_bytes,
            "gbs": total_bytes / wall / 1e9, "kernels": kernel_table(stats)}


def full_solve(E, p, arrs, precision, maxit, form, progress_every=0, **opts):
    """One warm-up solve of two iterations, then the full solve to the
    tolerance, bracketed by device synchronisations (`opts`: further
    Solver options, e.g. the variant)."""
    import torch
    rp, ci, va, dom, bd = arrs
    sol = E.Solver(rp, ci, va, dom, p.t, p.s, precision=precision,
                   progress_every=progress_every, **opts)
    sol.solve(bd, tol=p.tol, maxit=2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x, info = sol.solve(bd, tol=p.tol, maxit=maxit)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    sol.close()
    xs = x.cpu().numpy()
    log(f"[{form}] full solve: status {info.status}, {info.iters} iterations, "
        f"{info.restarts} restarts, true relres {info.true_relres:.2e}, {wall:.2f} s")
    return xs, {"time_s": round(wall, 4), "status": info.status, "iters": info.iters,
                "restarts": info.restarts, "true_relres": info.true_relres,
                "rel_err_vs_xstar": float(np.linalg.norm(xs - p.xstar) / np.linalg.norm(p.xstar))}


def precond_solve(E, p, arrs, precision, maxit, form, **opts):
    """Time-to-tolerance of the split preconditioned s-step SRE-CG with the
    block Jacobi IC(0) preconditioner whose blocks are the t domains; the
    host factorisation is timed separately."""
    import torch
    rp, ci, va, dom, bd = arrs
    sol = E.Solver(rp, ci, va, dom, p.t, p.s, precision=precision, **opts)
    t0 = time.perf_counter()
    sol.set_preconditioner(E.PREC_BJ_IC0, dom)
    torch.cuda.synchronize()
    t_fact = time.perf_counter() - t0
    sol.solve(bd, tol=p.tol, maxit=2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x, info = sol.solve(bd, tol=p.tol, maxit=maxit)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    sol.close()
    xs = x.cpu().numpy()
    log(f"[{form} + block Jacobi IC(0)] status {info.status}, {info.iters} iterations, "
        f"{info.restarts} restarts, true relres {info.true_relres:.2e}, {wall:.2f} s "
        f"(factorisation {t_fact:.2f} s)")
    return {"time_s": round(wall, 4), "factorisation_s": round(t_fact, 3), "status": info.status,
            "iters": info.iters, "restarts": info.restarts, "true_relres": info.true_relres,
            "ms_per_iteration": round(wall * 1e3 / max(info.iters, 1), 2),
            "rel_err_vs_xstar": float(np.linalg.norm(xs - p.xstar) / np.linalg.norm(p.xstar))}


def both_forms_to_tolerance(E, p, maxit, progress_every=0):
    arrs = device_arrays(E, p)
    x64, f64 = full_solve(E, p, arrs, E.FP64, maxit, "fp64", progress_every)
    x32, mx = full_solve(E, p, arrs, E.MIXED, maxit, "mixed", progress_every)
    mx["speedup_vs_fp64"] = round(f64["time_s"] / mx["time_s"], 3)
    mx["rel_diff_vs_fp64_x"] = float(np.linalg.norm(x32 - x64) / np.linalg.norm(x64))
    return {"workload": describe(p), "fp64": f64, "mixed": mx}


def variant_solves(E, cfgs, maxit, cap=64, only=None):
    """Time-to-1e-8 of the variants the paper compares (Section 4; Tables
    2-3), both forms: s-step SRE-CG, s-step SRE-CG2 with a cap of `cap`
    blocks, Pre-CholQR, s-step MSDO-CG with the same cap, and the CA forms
    of SRE-CG and SRE-CG2 (modified CA-Arnoldi)."""
    import torch
    table = [("sstep_srecg", {}),
             ("sstep_srecg2_cap", {"variant": E.SRECG2, "q_cap_blocks": cap}),
             ("sstep_srecg_precholqr", {"orth": E.PRECHOLQR}),
             ("sstep_msdo_cap", {"variant": E.MSDO, "q_cap_blocks": cap}),
             ("ca_srecg", {"ca": True}),
             ("ca_srecg2_cap", {"variant": E.SRECG2, "ca": True, "q_cap_blocks": cap})]
    out = {}
    for cfg in cfgs:
        p = build_problem(cfg)
        log(f"problem {describe(p)}")
        arrs = device_arrays(E, p)
        rows = {"workload": describe(p), "block_cap": cap}
        for name, kw in table:
            if only and name not in only:
                continue
            rows[name] = {}
            for form, prec in (("fp64", E.FP64), ("mixed", E.MIXED)):
                log(f"[{cfg} {name} {form}]")
                _, r = full_solve(E, p, arrs, prec, maxit, form, progress_every=50, **kw)
                rows[name][form] = r
        out[cfg] = rows
        del arrs
        torch.cuda.empty_cache()
    return out


def calibrate(torch):
    """Plain device copy of 256 MiB: the practical streaming ceiling, and the
    known-size kernel against which FETCH_SIZE / WRITE_SIZE are scaled."""
    n = 1 << 25
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    reps = 20
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    print(json.dumps({"calibration": "copy", "bytes_read": 8 * n, "bytes_written": 8 * n,
                      "us_per_copy": round(ms * 1e3, 1),
                      "gbs": round(16 * n / (ms * 1e-3) / 1e9, 1)}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed s-step iterations")
    ap.add_argument("--warmup", type=int, default=5, help="untimed s-step iterations")
    ap.add_argument("--config", default="C5", help="workload of the main line (C1..C5)")
    ap.add_argument("--maxit", type=int, default=30000, help="bound for full solves")
    ap.add_argument("--full", action="store_true",
                    help="only the time-to-1e-8 of the main workload (forms: --form)")
    ap.add_argument("--form", choices=("both", "fp64", "mixed"), default="both",
                    help="with --full: which form(s) to solve")
    ap.add_argument("--variants", default="",
                    help="comma-separated configs (e.g. C2,C3): only the time-to-1e-8 of the "
                         "s-step, SRE-CG2, Pre-CholQR, MSDO-CG and CA variants there")
    ap.add_argument("--cap", type=int, default=64,
                    help="with --variants: blocks kept by SRE-CG2 / MSDO-CG before a restart")
    ap.add_argument("--only", default="",
                    help="with --variants: comma-separated variant names to run")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-solve", action="store_true",
                    help="skip the full 128^3 skyscraper solves")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--row-order", choices=("domain", "morton"), default="domain",
                    help="rows of each domain in the caller's order or in Morton order")
    ap.add_argument("--calibrate", action="store_true",
                    help="time a plain 256 MiB device copy (the reference for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}): every box has one GPU, "
              "and the multi-GPU sharding is a design, not a build.", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1804_10629_amd as E

    torch.cuda.set_device(0)
    if args.calibrate:
        calibrate(torch)
        return
    if args.variants:
        res = variant_solves(E, args.variants.split(","), args.maxit, args.cap,
                             [v for v in args.only.split(",") if v])
        print(json.dumps({"variants_time_to_tolerance": res}), flush=True)
        return

    t0 = time.perf_counter()
    p = build_problem(args.config)
    log(f"problem {describe(p)} ({time.perf_counter() - t0:.1f} s)")
    if args.full:
        if args.form == "both":
            res = both_forms_to_tolerance(E, p, args.maxit, progress_every=100)
        else:
            prec = E.FP64 if args.form == "fp64" else E.MIXED
            _, one = full_solve(E, p, device_arrays(E, p), prec, args.maxit, args.form,
                                progress_every=100)
            res = {"workload": describe(p), args.form: one}
        print(json.dumps({"time_to_tolerance": res}), flush=True)
        return

    arrs = device_arrays(E, p)
    ro = {"row_key": E.grid_morton_keys(p.shape)} if args.row_order == "morton" else {}
    main_f = iteration_form(E, p, arrs, E.FP64, args.steps, args.warmup, "fp64", **ro)
    mixed = None
    if not args.no_mixed:
        mixed = iteration_form(E, p, arrs, E.MIXED, args.steps, args.warmup, "mixed", **ro)
    prec = None
    if not args.no_solve:
        prec = {"preconditioner": "block Jacobi, IC(0) blocks = the t domains (Section 5)",
                "workload": describe(p),
                "fp64": precond_solve(E, p, arrs, E.FP64, args.maxit, "fp64", **ro)}
        if not args.no_mixed:
            prec["mixed"] = precond_solve(E, p, arrs, E.MIXED, args.maxit, "mixed", **ro)
            prec["mixed"]["speedup_vs_fp64"] = round(prec["fp64"]["time_s"] / prec["mixed"]["time_s"], 3)
    del arrs
    torch.cuda.empty_cache()

    sky = None
    if not args.no_solve:
        ps = build_problem("C2")
        log(f"problem {describe(ps)}")
        sky = both_forms_to_tolerance(E, ps, args.maxit)

    cpu = None
    bytes_per_iter = main_f["bytes"] / max(main_f["iters"], 1)
    if not args.no_cpu_baseline:
        log("CPU oracle sample")
        cpu = cpu_baseline(p, bytes_per_iter)
        log("C1 full solves: oracle and GPU")
        cpu["c1_full_solves"] = c1_full_solves(E)

    out = {
        "metric": METRIC,
        "value": round(main_f["gbs"], 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": main_f["iters"],
        "warmup": args.warmup,
        "ms_per_step": round(main_f["ms_per_step"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": describe(p), "n": p.n, "nnz": p.nnz, "t": p.t, "s": p.s,
                   "tol": p.tol, "variant": "s-step SRE-CG", "parallelism": "single GPU",
                   "step": "one s-step iteration", "row_order": args.row_order},
        "value_definition": ("algorithmic HBM bytes of the kernels of the timed s-step "
                             "iterations over their wall time (binary64)"),
        "gb_per_step": round(bytes_per_iter / 1e9, 3),
        "kernels": main_f["kernels"],
        "roofline": roofline(main_f["kernels"], p.name, "fp64", args.row_order),
        "mixed": None if mixed is None else {
            "value": round(mixed["gbs"], 1), "unit": "GB/s",
            "ms_per_step": round(mixed["ms_per_step"], 3),
            "speedup_per_step_vs_fp64": round(main_f["ms_per_step"] / mixed["ms_per_step"], 3),
            "gb_per_step": round(mixed["bytes"] / max(mixed["iters"], 1) / 1e9, 3),
            "kernels": mixed["kernels"],
            "roofline": roofline(mixed["kernels"], p.name, "mixed", args.row_order),
        },
        "time_to_1e8": {"unpreconditioned": ("python bench.py --full --form fp64|mixed; "
                                             "profiles/randomblocks3d_256_time_to_1e8.md"),
                        "block_jacobi_ic0": prec},
        "skyscraper_128": sky,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
