"""GPU parity of the hand-written adjoint (spx_values_grad and the autograd
function) against the oracle's adjoint, which is pinned by finite differences
(tests/test_oracle_adjoint.py).  Tolerance: the gradient entries are products
of two solutions with componentwise backward error <= 1e-14; the difference
between the two is bounded by a few kappa * 1e-14 relative to the largest
entry, and we gate at 1e-9 for kappa up to ~1e3."""
import numpy as np
import pytest

from gen import grid_laplacian, make_config, random_spd, rhs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


def _oracle_adjoint(orc, p, B, Xbar):
    sym = orc.analyze(p.n, p.colptr, p.rowind)
    P = orc.factor(sym, p.colptr, p.rowind, p.values)
    x, _ = orc.solve_refined(sym, P, p.colptr, p.rowind, p.values, B)
    db, g = orc.adjoint(sym, P, p.colptr, p.rowind, p.values, x, Xbar)
    return x, db, g


@pytest.mark.parametrize("case", ["c1", "rand", "grid3"])
def test_values_grad_matches_oracle(orc, torch, case):
    if case == "c1":
        p, nrhs = make_config(1), 1
    elif case == "rand":
        p, nrhs = random_spd(900, 0.005, 12), 3
    else:
        p, nrhs = grid_laplacian((14, 13, 12), shift=1e-3), 2
    print("adjoint case %s n=%d nrhs=%d" % (case, p.n, nrhs), flush=True)
    B = rhs(p.n, nrhs, 31)
    Xbar = rhs(p.n, nrhs, 32)
    xo, dbo, go = _oracle_adjoint(orc, p, B, Xbar)
    from paper_1405_2636_amd import Solver, solve_autograd
    s = Solver(p.n, p.colptr, p.rowind)
    vals = torch.tensor(p.values, device="cuda", requires_grad=True)
    b = torch.tensor(np.ascontiguousarray(B.T), device="cuda", requires_grad=True)
    x = solve_autograd(s, vals, b)
    xbar = torch.tensor(np.ascontiguousarray(Xbar.T), device="cuda")
    gv, gb = torch.autograd.grad(x, (vals, b), grad_outputs=xbar)
    assert np.max(np.abs(x.detach().cpu().numpy().T - xo)) <= 1e-10 * np.max(np.abs(xo))
    assert np.max(np.abs(gb.cpu().numpy().T - dbo)) <= 1e-10 * np.max(np.abs(dbo))
    g = gv.cpu().numpy()
    assert np.max(np.abs(g - go)) <= 1e-9 * np.max(np.abs(go))
    col = np.repeat(np.arange(p.n), np.diff(p.colptr))
    assert np.all(g[p.rowind < col] == 0.0)


def test_autograd_finite_differences(torch):
    # directional derivative of a scalar loss along a random value perturbation
    # (kept symmetric-definite), central differences of the GPU solve itself
    p = random_spd(200, 0.03, 4)
    from paper_1405_2636_amd import Solver, solve_autograd
    s = Solver(p.n, p.colptr, p.rowind)
    rng = np.random.default_rng(9)
    c = torch.tensor(rng.uniform(-1, 1, p.n), device="cuda")
    b = torch.tensor(rng.uniform(-1, 1, p.n), device="cuda")
    v0 = torch.tensor(p.values, device="cuda")
    dv = torch.tensor(rng.uniform(-1, 1, p.nnz) * 1e-2, device="cuda")
    v = v0.clone().requires_grad_(True)
    loss = (c * solve_autograd(s, v, b)).sum()
    (g,) = torch.autograd.grad(loss, v)
    analytic = float((g * dv).sum())
    h = 1e-4

    def L(vals):
        with torch.no_grad():
            return float((c * solve_autograd(s, vals, b)).sum())

    fd = (L(v0 + h * dv) - L(v0 - h * dv)) / (2 * h)
    assert abs(fd - analytic) <= 1e-7 * max(1.0, abs(fd))


def test_backward_after_refactorization(orc, torch):
    # two forward passes on one solver with different values before either
    # backward pass: each backward pass must use its own matrix
    from paper_1405_2636_amd import Solver, solve_autograd
    p = grid_laplacian((11, 10, 9), shift=1e-3)
    q = grid_laplacian((11, 10, 9), shift=0.5)          # same pattern, other values
    assert np.array_equal(p.rowind, q.rowind)
    print("adjoint after refactorization n=%d" % p.n, flush=True)
    B, Xbar = rhs(p.n, 1, 41), rhs(p.n, 1, 42)
    s = Solver(p.n, p.colptr, p.rowind)
    vp = torch.tensor(p.values, device="cuda", requires_grad=True)
    vq = torch.tensor(q.values, device="cuda", requires_grad=True)
    b = torch.tensor(np.ascontiguousarray(B[:, 0]), device="cuda")
    xp = solve_autograd(s, vp, b)
    xq = solve_autograd(s, vq, b)
    xbar = torch.tensor(np.ascontiguousarray(Xbar[:, 0]), device="cuda")
    (gq,) = torch.autograd.grad(xq, vq, grad_outputs=xbar)
    (gp,) = torch.autograd.grad(xp, vp, grad_outputs=xbar)
    for prob, x, g in ((p, xp, gp), (q, xq, gq)):
        xo, _, go = _oracle_adjoint(orc, prob, B, Xbar)
        assert np.max(np.abs(x.detach().cpu().numpy() - xo[:, 0])) <= 1e-10 * np.max(np.abs(xo))
        assert np.max(np.abs(g.cpu().numpy() - go)) <= 1e-9 * np.max(np.abs(go))
