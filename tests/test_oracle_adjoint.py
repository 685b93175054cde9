"""Pins of the oracle's adjoint (x = A^{-1} b, symmetric A given by its lower
triangle): central finite differences of the oracle's own refined solve, and
the backward solve against a dense library solve."""
import numpy as np
import scipy.sparse as sp

from gen import random_spd


def _loss_and_x(orc, p, values, b, c):
    sym = orc.analyze(p.n, p.colptr, p.rowind, leaf=4)
    P = orc.factor(sym, p.colptr, p.rowind, values)
    x, _ = orc.solve_refined(sym, P, p.colptr, p.rowind, values, b)
    return float(np.sum(c * x)), x, sym, P


def test_adjoint_matches_finite_differences(orc):
    # loss = sum(c * x); the gradient with respect to every stored value,
    # checked entry by entry against central differences of the loss
    p = random_spd(14, 0.3, 21)
    rng = np.random.default_rng(3)
    b = rng.uniform(-1, 1, (p.n, 2))
    c = rng.uniform(-1, 1, (p.n, 2))
    L0, x, sym, P = _loss_and_x(orc, p, p.values, b, c)
    db, g = orc.adjoint(sym, P, p.colptr, p.rowind, p.values, x, c)
    col = np.repeat(np.arange(p.n), np.diff(p.colptr))
    checked = 0
    for q in range(p.nnz):
        h = 1e-5 * max(1.0, abs(p.values[q]))
        vp, vm = p.values.copy(), p.values.copy()
        vp[q] += h
        vm[q] -= h
        fd = (_loss_and_x(orc, p, vp, b, c)[0] - _loss_and_x(orc, p, vm, b, c)[0]) / (2 * h)
        assert abs(fd - g[q]) <= 1e-6 * max(1.0, abs(fd)), (q, p.rowind[q], col[q], fd, g[q])
        checked += p.rowind[q] >= col[q]
    assert checked > p.n   # diagonal and off-diagonal entries were exercised


def test_adjoint_upper_entries_have_zero_gradient(orc):
    # with the full symmetric pattern given, only the lower entries are read
    p = random_spd(12, 0.3, 5)
    col = np.repeat(np.arange(p.n), np.diff(p.colptr))
    assert np.any(p.rowind < col)   # the generator gives both triangles
    rng = np.random.default_rng(1)
    x = rng.standard_normal((p.n, 3))
    db = rng.standard_normal((p.n, 3))
    g = orc.values_grad(p.n, p.colptr, p.rowind, x, db)
    assert np.all(g[p.rowind < col] == 0.0)
    assert np.all(g[p.rowind >= col] != 0.0)


def test_adjoint_backward_solve_is_dense_solve(orc):
    p = random_spd(30, 0.2, 8)
    A = sp.csc_matrix((p.values, p.rowind, p.colptr), shape=(p.n, p.n)).toarray()
    A = np.tril(A) + np.tril(A, -1).T   # the matrix the lower triangle defines
    rng = np.random.default_rng(2)
    b = rng.uniform(-1, 1, (p.n, 1))
    xbar = rng.uniform(-1, 1, (p.n, 1))
    sym = orc.analyze(p.n, p.colptr, p.rowind)
    P = orc.factor(sym, p.colptr, p.rowind, p.values)
    x, _ = orc.solve_refined(sym, P, p.colptr, p.rowind, p.values, b)
    db, _ = orc.adjoint(sym, P, p.colptr, p.rowind, p.values, x, xbar)
    ref = np.linalg.solve(A, xbar)
    assert np.max(np.abs(db - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_values_grad_entry_by_entry(orc):
    # the C routine against the definition written out entry by entry
    p = random_spd(40, 0.15, 13)
    rng = np.random.default_rng(4)
    x = rng.standard_normal((p.n, 3))
    db = rng.standard_normal((p.n, 3))
    g = orc.values_grad(p.n, p.colptr, p.rowind, x, db)
    col = np.repeat(np.arange(p.n), np.diff(p.colptr))
    for q in range(p.nnz):
        i, j = int(p.rowind[q]), int(col[q])
        if i > j:
            ref = -(db[i] @ x[j] + db[j] @ x[i])
        elif i == j:
            ref = -(db[i] @ x[i])
        else:
            ref = 0.0
        assert abs(g[q] - ref) <= 1e-14 * max(1.0, abs(ref))
