"""GPU parity at the full problem sizes, in the launch configuration the
benchmark uses (default grid, stream and options).

* 128^3 skyscraper (t = 16, s = 4) and 128^3 anisotropic (t = 32, s = 4):
  the first s-step iteration is compared element by element with the
  oracle's (x_1 over all 2.1M rows; at 16 columns also the basis it built),
  in the FP64 and the mixed form.
* 128^3 skyscraper with the rows of each domain in Morton order: the first
  iterate against the oracle.
* 128^3 anisotropic, CA SRE-CG: the first two iterates against the oracle.
* 1000^2 log-uniform (t = 16, s = 3): x_1 and x_4 over all 1M rows and the
  residual history against the oracle's.
* 128^3 skyscraper: a full solve, its true residual recomputed on the CPU,
  and two 60-iteration solves in each form that agree bit for bit.
* 256^3 random blocks (t = 64, s = 2, 16.8M rows): too large for the oracle;
  the first iteration is checked against properties that hold at any size
  (eqs (1)-(3) with an A-orthonormal basis): V^t A V = I, V^t r_1 = 0, and the
  A-norm error drop ||e_0||_A^2 - ||e_1||_A^2 = ||alpha||^2.
"""
import numpy as np
import pytest

import oracle as O
import problems as P

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def E():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    import paper_1804_10629_amd as E
    return E


def _device_solver(E, p, **kw):
    import torch
    dom = E.partition_grid(p.shape, p.parts)
    rp, ci, va = (torch.as_tensor(a).cuda() for a in (p.rowptr, p.colind, p.vals))
    return E.Solver(rp, ci, va, dom, p.t, p.s, **kw), dom


@pytest.fixture(scope="module")
def sky():
    p = P.CONFIGS["C2"]()
    return p, p.scipy(), O.partition_grid(p.shape, p.parts)


@pytest.mark.parametrize("mixed", [False, True])
def test_skyscraper_first_iteration(E, sky, mixed):
    p, A, dom = sky
    kw = {"basis_dtype": np.float32, "inner_tol": 1e-4} if mixed else {}
    ref = O.sstep_srecg(A, dom, p.t, p.s, p.b, tol=p.tol, maxit=1, record=True, **kw)
    sol, _ = _device_solver(E, p, precision=E.MIXED if mixed else E.FP64)
    x, info = sol.solve(p.b, tol=p.tol, maxit=1)
    assert info.iters == 1
    x = x.cpu().numpy()
    xr = ref.extra["xs"][1]
    # binary32 blocks round differently on the two sides (the device keeps
    # them unnormalised): the mixed bound allows some binary32 ulps
    bound = 1e-6 if mixed else 1e-10
    rel = np.linalg.norm(x - xr) / np.linalg.norm(xr)
    print(f"x_1 relative difference {rel:.2e}")
    assert rel <= bound
    assert abs(info.hist[1] - ref.hist[1]) <= bound * ref.hist[1]
    if not mixed:
        V, AV = (a.cpu().numpy() for a in sol.basis())
        Vr, AVr = ref.extra["V"][0]
        assert np.abs(V - Vr).max() <= 1e-10 * np.abs(Vr).max()
        assert np.abs(AV - AVr).max() <= 1e-10 * np.abs(AVr).max()
    sol.close()


def test_skyscraper_first_iteration_morton_order(E, sky):
    # the rows of each domain stored in Morton order (the grid's keys): the
    # first iterate, in the caller's order, against the oracle's
    p, A, dom = sky
    ref = O.sstep_srecg(A, dom, p.t, p.s, p.b, tol=p.tol, maxit=1, record=True)
    sol, _ = _device_solver(E, p, row_key=E.grid_morton_keys(p.shape))
    x, info = sol.solve(p.b, tol=p.tol, maxit=1)
    assert info.iters == 1
    xr = ref.extra["xs"][1]
    rel = float(np.linalg.norm(x.cpu().numpy() - xr) / np.linalg.norm(xr))
    print(f"Morton order x_1 relative difference {rel:.2e}")
    assert rel <= 1e-10
    assert abs(info.hist[1] - ref.hist[1]) <= 1e-10 * ref.hist[1]
    sol.close()


def test_skyscraper_full_solve(E, sky):
    p, A, _ = sky
    sol, _ = _device_solver(E, p)
    x, info = sol.solve(p.b, tol=p.tol, maxit=5000)
    assert info.status == E.OK and info.true_relres <= p.tol
    x = x.cpu().numpy()
    # the true residual again, on the CPU in binary64
    assert np.linalg.norm(p.b - A @ x) <= p.tol * np.linalg.norm(p.b)
    assert np.linalg.norm(x - p.xstar) <= 1e-2 * np.linalg.norm(p.xstar)
    sol.close()


@pytest.mark.parametrize("mixed", [False, True])
def test_skyscraper_bitwise_reproducible(E, sky, mixed):
    # fixed-order reductions: two solves of the same system give the same
    # bits (x, every residual norm, the true residual)
    p, _, _ = sky
    sol, _ = _device_solver(E, p, precision=E.MIXED if mixed else E.FP64)
    x1, i1 = sol.solve(p.b, tol=p.tol, maxit=60)
    x1 = x1.cpu().numpy()
    x2, i2 = sol.solve(p.b, tol=p.tol, maxit=60)
    x2 = x2.cpu().numpy()
    assert i1.iters == i2.iters == 60 and i1.restarts == i2.restarts
    assert np.array_equal(x1, x2)
    assert np.array_equal(np.asarray(i1.hist), np.asarray(i2.hist))
    assert i1.true_relres == i2.true_relres
    sol.close()


def test_ca_first_iterations_full_size(E):
    # CA SRE-CG (modified CA-Arnoldi) at 128^3, t = 32, s = 4: the first two
    # iterates over all 2.1M rows against the oracle (the second one
    # A-orthonormalizes against the kept blocks)
    p = P.CONFIGS["C3"]()
    A = p.scipy()
    dom = O.partition_grid(p.shape, p.parts)
    ref = O.sstep_srecg(A, dom, p.t, p.s, p.b, tol=p.tol, maxit=2, ca=True, record=True)
    sol, _ = _device_solver(E, p, ca=True)
    for k in (1, 2):
        x, info = sol.solve(p.b, tol=p.tol, maxit=k)
        assert info.iters == k and info.blocks == k * p.s
        xr = ref.extra["xs"][k]
        rel = float(np.linalg.norm(x.cpu().numpy() - xr) / np.linalg.norm(xr))
        print(f"CA SRE-CG 128^3 x_{k}: rel {rel:.2e}")
        assert rel <= 1e-9
    sol.close()


@pytest.mark.parametrize("mixed", [False, True])
def test_anisotropic_first_iteration(E, mixed):
    p = P.CONFIGS["C3"]()
    A = p.scipy()
    dom = O.partition_grid(p.shape, p.parts)
    kw = {"basis_dtype": np.float32, "inner_tol": 1e-4} if mixed else {}
    ref = O.sstep_srecg(A, dom, p.t, p.s, p.b, tol=p.tol, maxit=1, record=True, **kw)
    sol, _ = _device_solver(E, p, precision=E.MIXED if mixed else E.FP64)
    x, info = sol.solve(p.b, tol=p.tol, maxit=1)
    xr = ref.extra["xs"][1]
    rel = np.linalg.norm(x.cpu().numpy() - xr) / np.linalg.norm(xr)
    print(f"x_1 relative difference {rel:.2e}")
    assert rel <= (1e-6 if mixed else 1e-10)
    sol.close()


def test_log_uniform_first_iterations(E):
    # 1000^2 log-uniform (t = 16, s = 3): the full solve is rounding-sensitive
    # (its count moves with ulp-level changes), the first iterates are not
    # (perturbing b by one part in 1e15 moves the oracle's x_4 by 7e-15), so
    # x_1 and x_4 over all 1M rows and the residual history are compared with
    # the oracle's
    p = P.CONFIGS["C4"]()
    A = p.scipy()
    dom = O.partition_grid(p.shape, p.parts)
    ref = O.sstep_srecg(A, dom, p.t, p.s, p.b, tol=p.tol, maxit=4, record=True)
    sol, _ = _device_solver(E, p)
    for k in (1, 4):
        x, info = sol.solve(p.b, tol=p.tol, maxit=k)
        assert info.iters == k
        xr = ref.extra["xs"][k]
        rel = float(np.linalg.norm(x.cpu().numpy() - xr) / np.linalg.norm(xr))
        h_gpu, h_or = np.asarray(info.hist[:k + 1]), np.asarray(ref.hist[:k + 1])
        hrel = float(np.max(np.abs(h_gpu - h_or) / h_or))
        print(f"log-uniform 1000^2 x_{k}: rel {rel:.2e}, history {hrel:.2e}")
        assert rel <= 1e-9 and hrel <= 1e-9
    sol.close()


def test_random_blocks_first_iteration_properties(E):
    import torch
    p = P.CONFIGS["C5"]()
    sol, _ = _device_solver(E, p)
    b = torch.as_tensor(p.b).cuda()
    xs = torch.as_tensor(p.xstar).cuda()
    x, info = sol.solve(b, tol=p.tol, maxit=1)
    assert info.iters == 1
    V, AV = sol.basis()                       # n x (s t), binary64
    G = V.T @ AV                              # V^t A V
    eye = torch.eye(G.shape[0], dtype=G.dtype, device=G.device)
    dev = float((G - eye).abs().max())
    print(f"max |V^t A V - I| = {dev:.2e}")
    assert dev <= 1e-10
    # AV is A V: compare with a fresh product of the solver's own kernel on a
    # few columns
    AVc = sol.spmm(V[:, :8].contiguous())
    assert float((AVc - AV[:, :8]).abs().max()) <= 1e-10 * float(AV[:, :8].abs().max())
    # r_1 = b - A x_1 is orthogonal to V (Petrov-Galerkin)
    r1 = b - sol.spmm(x)
    pg = float((V.T @ r1).abs().max()) / float(b.norm())
    print(f"max |V^t r_1| / ||b|| = {pg:.2e}")
    assert pg <= 1e-12
    # A-norm error drop: alpha = V^t r_0 with r_0 = b (x_0 = 0)
    alpha = V.T @ b
    e0, e1 = xs, xs - x
    E0 = float(e0 @ sol.spmm(e0))
    E1 = float(e1 @ sol.spmm(e1))
    drop = abs((E0 - E1) - float(alpha @ alpha)) / E0
    print(f"error-drop identity residual {drop:.2e}")
    assert drop <= 1e-10
    del V, AV, G
    sol.close()


@pytest.mark.parametrize("cfg,mixed", [("C2", True), ("C5", False)])
def test_block_jacobi_preconditioned_full_size(E, cfg, mixed):
    # block Jacobi IC(0), blocks = the t domains: the full solve reaches the
    # tolerance (at 128^3 in the mixed form the basis turns rank-deficient
    # near convergence and the solve restarts from the last iterate); the
    # true residual recomputed on the CPU in binary64
    import torch
    p = P.CONFIGS[cfg]()
    sol, dom = _device_solver(E, p, precision=E.MIXED if mixed else E.FP64)
    sol.set_preconditioner(E.PREC_BJ_IC0, dom)
    x, info = sol.solve(torch.as_tensor(p.b).cuda(), tol=p.tol, maxit=1000)
    xs = x.cpu().numpy()
    true = float(np.linalg.norm(p.b - p.scipy() @ xs) / np.linalg.norm(p.b))
    print(f"{cfg} preconditioned ({'mixed' if mixed else 'fp64'}): {info.iters} iterations, "
          f"{info.restarts} restarts, true relres {true:.2e}")
    assert info.status == E.OK and info.true_relres <= p.tol and true <= p.tol
    assert info.iters <= (150 if cfg == "C5" else 100)
    sol.close()


def _golden(cfg):
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                        f"fullsize_{cfg}.npz")
    if not os.path.exists(path):
        pytest.skip(f"no oracle reference for {cfg} (tests/golden/make_fullsize.py)")
    return dict(np.load(path))


@pytest.mark.parametrize("cfg", ["C2", "C3", "C4"])
def test_full_solve_parity_against_oracle(E, cfg):
    # the full FP64 solve against the float64 oracle's (tests/golden): count
    # within 2 (within the ulp-perturbed ensemble's band + 2 where the
    # oracle's own count moves), x at 65536 seeded rows within 1e-6 of the
    # oracle's (relative 2-norm over the sample; the ensemble's sampled
    # spread, capped, where the count moves), the residual history, and the
    # true residual recomputed on the CPU
    import torch
    from tests.parity import CAP_2_FULL, SPREAD_2_FULL
    g = _golden(cfg)
    p = P.CONFIGS[cfg]()
    sol, _ = _device_solver(E, p)
    x, info = sol.solve(torch.as_tensor(p.b).cuda(), tol=p.tol, maxit=30000)
    xs = x.cpu().numpy()
    true = float(np.linalg.norm(p.b - p.scipy() @ xs) / np.linalg.norm(p.b))
    idx = g["idx"]
    rel = float(np.linalg.norm(xs[idx] - g["xs"]) / np.linalg.norm(g["xs"]))
    lo, hi = int(g["ens_iters"].min()), int(g["ens_iters"].max())
    spread = float(g["ens_spread2"])
    print(f"{cfg}: GPU {info.iters} iterations, oracle {int(g['iters'])} (ensemble {lo}..{hi}, "
          f"sampled spread {spread:.1e}); sampled |x - x_or|/|x_or| = {rel:.2e}; "
          f"true relres {true:.2e}")
    assert info.status == E.OK and true <= p.tol and int(g["status"]) == 0
    if hi - lo <= 2 and spread <= 1e-7:
        assert abs(info.iters - int(g["iters"])) <= 2
        assert rel <= 1e-6
        n = min(len(info.hist), len(g["hist"]))
        h_or, h_gpu = g["hist"][:n], info.hist[:n]
        assert np.all(np.abs(h_gpu - h_or) <= 1e-6 * h_or)
    else:
        assert spread <= SPREAD_2_FULL
        assert lo - 2 <= info.iters <= hi + 2
        assert rel <= min(CAP_2_FULL, max(1e-6, 2.0 * spread))
    if "ens_err_xstar" in g:
        # as accurate as the oracle: the sampled error against x* (b = A x*)
        # within 1.5x of the worst ensemble member's
        xst = p.xstar[idx]
        err = float(np.linalg.norm(xs[idx] - xst) / np.linalg.norm(xst))
        print(f"{cfg}: sampled error vs x* {err:.2e} (oracle ensemble up to "
              f"{float(np.max(g['ens_err_xstar'])):.2e})")
        assert err <= 1.5 * float(np.max(g["ens_err_xstar"]))
    sol.close()


def test_differentiation_full_size(E):
    # the differentiation form on the 1000^2 log-uniform problem: loss
    # ||x - x_tgt||^2, forward and adjoint solves on the GPU, SDDMM bit-exact
    # on all 4,996,000 stored entries and the adjoint residual recomputed on
    # the CPU (finite differences of single entries are checked on a 32 x 32
    # field of the same family, test_gpu_autograd.py: at 1000^2 the loss
    # differences they need lie below what a solve resolves)
    import time
    import torch
    p = P.CONFIGS["C4"]()
    A = p.scipy()
    sol, _ = _device_solver(E, p)
    b = torch.as_tensor(p.b).cuda()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x, fi = sol.solve(b, tol=p.tol, maxit=30000)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    gx = 2.0 * (x - torch.as_tensor(p.extra["x_tgt"]).cuda())
    lam, bi = sol.solve(gx, tol=p.tol, maxit=30000)
    gA = sol.sddmm(lam, x)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    print(f"forward {t1 - t0:.2f} s ({fi.iters} iterations), backward {t2 - t1:.2f} s "
          f"({bi.iters} iterations) incl. SDDMM")
    assert fi.status == E.OK and bi.status == E.OK
    xs, ls, gs = x.cpu().numpy(), lam.cpu().numpy(), gx.cpu().numpy()
    assert np.linalg.norm(A @ ls - gs) <= 1.01 * p.tol * np.linalg.norm(gs)
    assert np.array_equal(gA.cpu().numpy(), O.sddmm(p.rowptr, p.colind, ls, xs))
    sol.close()
