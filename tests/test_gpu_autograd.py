"""Differentiation form through the C ABI: x = A(vals)^{-1} b with the
torch.autograd.Function, its backward an adjoint solve on the GPU and the
SDDMM kernel.  Checked against a dense FP64 reference gradient (oracle) and
against central finite differences of the loss, both on a 32 x 32 instance
of the log-uniform 2D diffusion field."""
import numpy as np
import pytest
import scipy.sparse as sp

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


@pytest.fixture(scope="module")
def case():
    p = P.loguniform2d(32, t=16, parts=(4, 4, 1), s=3)
    dom = O.partition_grid(p.shape, p.parts)
    return p, dom


def _grad(E, p, dom, vals, b, tol=1e-12):
    import torch
    v = torch.tensor(vals, dtype=torch.float64, device="cuda", requires_grad=True)
    bt = torch.tensor(b, dtype=torch.float64, device="cuda", requires_grad=True)
    tgt = torch.tensor(p.extra["x_tgt"], dtype=torch.float64, device="cuda")
    x = E.solve_with_grad(p.rowptr, p.colind, v, dom, p.t, p.s, bt, tol=tol, maxit=5000)
    loss = ((x - tgt) ** 2).sum()
    loss.backward()
    return float(loss.detach()), x.detach().cpu().numpy(), v.grad.cpu().numpy(), bt.grad.cpu().numpy()


def test_gradient_matches_dense_reference(E, case):
    p, dom = case
    loss, x, gv, gb = _grad(E, p, dom, p.vals, p.b)
    A = p.scipy().toarray()
    xr, lam, _ = O.dense_gradient(A, p.b, p.extra["x_tgt"])
    gv_ref = O.sddmm(p.rowptr, p.colind, lam, xr)
    assert np.linalg.norm(x - xr) <= 1e-9 * np.linalg.norm(xr)
    assert np.linalg.norm(gb - lam) <= 1e-8 * np.linalg.norm(lam)
    assert np.linalg.norm(gv - gv_ref) <= 1e-8 * np.linalg.norm(gv_ref)


def test_gradient_matches_finite_differences(E, case):
    import torch
    p, dom = case
    loss0, x, gv, gb = _grad(E, p, dom, p.vals, p.b)
    rows = np.repeat(np.arange(p.n), np.diff(p.rowptr))
    tgt = p.extra["x_tgt"]

    def loss_at(vals, b):
        # the loss differences sit ~1e-9 below the loss, under what a solve
        # to 1e-12 resolves: one step of iterative refinement (residual in
        # binary64 on the host, correction by a second GPU solve) removes
        # that noise
        s = E.Solver(p.rowptr, p.colind, vals, dom, p.t, p.s)
        xx, info = s.solve(b, tol=1e-12, maxit=5000)
        assert info.status == E.OK
        xx = xx.cpu().numpy()
        A = sp.csr_matrix((vals, p.colind, p.rowptr), shape=(p.n, p.n))
        d, info = s.solve(b - A @ xx, tol=1e-12, maxit=5000)
        assert info.status == E.OK
        s.close()
        return float(np.sum((xx + d.cpu().numpy() - tgt) ** 2))

    # four-point central differences, O(h^4); the step is relative to the
    # entry's natural scale sqrt(A_ii A_jj), and entries whose scale is below 1
    # are skipped (their steps would sit at the loss's rounding level)
    diag = p.vals[rows == p.colind]
    scale = np.sqrt(diag[rows] * diag[p.colind])

    def fd4(f, h):
        return (8.0 * (f(h) - f(-h)) - (f(2 * h) - f(-2 * h))) / (12.0 * h)

    rng = np.random.default_rng(3)
    for q in rng.choice(np.nonzero(scale >= 1.0)[0], 6, replace=False):
        i, j = rows[q], p.colind[q]
        qt = np.nonzero((rows == j) & (p.colind == i))[0][0]

        def f(d):
            v = p.vals.copy()
            v[q] += d
            if qt != q:                          # symmetric pair keeps A SPD
                v[qt] += d
            return loss_at(v, p.b)

        fd = fd4(f, 1e-4 * scale[q])
        an = gv[q] + (gv[qt] if i != j else 0.0)
        assert abs(fd - an) <= 1e-5 * max(abs(an), 1e-3 * np.abs(gv).max()), (q, fd, an)
    for i in rng.choice(p.n, 4, replace=False):
        def fb(d):
            b = p.b.copy()
            b[i] += d
            return loss_at(p.vals, b)

        fd = fd4(fb, 1e-4 * max(abs(p.b[i]), 1.0))
        assert abs(fd - gb[i]) <= 1e-5 * max(abs(gb[i]), 1e-3 * np.abs(gb).max())
    del torch
