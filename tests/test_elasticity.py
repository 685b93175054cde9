"""The Q1 elasticity input (the L D L^T workload: 27-point, 3-dof, SPD once
clamped) pinned by what mechanics fixes, and the oracle's L D L^T and
adjoint on it.

Element: symmetric, rank 18, the six rigid-body motions in its null space;
a uniform strain field stores exactly eps^T D eps per unit volume (Q1
elements represent linear displacements exactly).  Assembly: symmetric,
positive definite, 81 entries in an interior row, and the entry count
9 (3m - 2)^3 for m free nodes per side (14,787,288 at m = 40)."""
import numpy as np
import pytest
import scipy.sparse as sp

from gen import elasticity3d, element_stiffness, material_matrix


def _corners():
    return np.array([[a & 1, (a >> 1) & 1, (a >> 2) & 1] for a in range(8)], float)


def test_element_rigid_modes_and_rank():
    K = element_stiffness()
    assert np.allclose(K, K.T, atol=1e-15)
    X = _corners()
    modes = []
    for d in range(3):                       # translations
        u = np.zeros((8, 3)); u[:, d] = 1.0
        modes.append(u.ravel())
    for (i, j) in [(0, 1), (1, 2), (0, 2)]:  # infinitesimal rotations
        u = np.zeros((8, 3)); u[:, i] = -X[:, j]; u[:, j] = X[:, i]
        modes.append(u.ravel())
    for u in modes:
        assert np.max(np.abs(K @ u)) <= 1e-13
    ev = np.linalg.eigvalsh(K)
    assert np.sum(ev > 1e-10) == 18 and np.min(ev) > -1e-13


def test_uniform_strain_energy():
    # u(x) = G x with G symmetric (no rotation): strain = G in Voigt form,
    # energy u^T K u = eps^T D eps over the unit volume
    rng = np.random.default_rng(1)
    K = element_stiffness(0.3)
    D = material_matrix(0.3)
    X = _corners()
    for _ in range(5):
        G = rng.uniform(-1, 1, (3, 3))
        G = 0.5 * (G + G.T)
        u = (X @ G.T).ravel()
        eps = np.array([G[0, 0], G[1, 1], G[2, 2], 2 * G[1, 2], 2 * G[0, 2], 2 * G[0, 1]])
        assert abs(u @ K @ u - eps @ D @ eps) <= 1e-13 * abs(eps @ D @ eps)


@pytest.mark.parametrize("n", [3, 5, 8])
def test_assembled_matrix(n):
    p = elasticity3d(n, seed=7)
    m = n - 2
    assert p.n == 3 * m ** 3
    assert p.nnz == 9 * (3 * m - 2) ** 3
    A = sp.csc_matrix((p.values, p.rowind, p.colptr), shape=(p.n, p.n))
    assert abs(A - A.T).max() == 0.0
    assert np.linalg.eigvalsh(A.toarray())[0] > 0
    if n >= 5:
        assert np.diff(p.colptr).max() == 81
    # the stated size of the 40^3 workload follows from the same count
    assert 9 * (3 * 40 - 2) ** 3 == 14787288 and 3 * 40 ** 3 == 192000


def test_ldlt_on_elasticity(orc):
    p = elasticity3d(7, seed=1005)
    sym = orc.analyze(p.n, p.colptr, p.rowind)
    P = orc.factor_ldlt(sym, p.colptr, p.rowind, p.values)
    ri, ci, v = orc.unpack(sym, P)
    dg = ri == ci
    D = np.zeros(p.n)
    D[ri[dg]] = v[dg]
    assert np.all(D > 0)
    Lu = sp.csc_matrix((v[~dg], (ri[~dg], ci[~dg])), shape=(p.n, p.n)) + sp.identity(p.n, format="csc")
    A = sp.csc_matrix((p.values, p.rowind, p.colptr), shape=(p.n, p.n))
    PA = A[sym.perm][:, sym.perm]
    assert sp.linalg.norm(PA - Lu @ sp.diags(D) @ Lu.T) / sp.linalg.norm(PA) <= 1e-13
    lad, nneg = orc.logabsdet_ldlt(sym, P)
    sign, ref = np.linalg.slogdet(A.toarray())
    assert nneg == 0 and sign == 1 and abs(lad - ref) <= 1e-10 * abs(ref)
    b = np.random.default_rng(5).uniform(-1, 1, (p.n, 8))
    x = orc.solve_ldlt(sym, P, b)
    r, s = orc.residual(p.n, p.colptr, p.rowind, p.values, x, b)
    assert orc.omega(r, s) <= 1e-14


def _ldlt_solve_refined(orc, sym, p, values, b):
    P = orc.factor_ldlt(sym, p.colptr, p.rowind, values)
    x = orc.solve_ldlt(sym, P, b)
    for _ in range(2):
        r, _ = orc.residual(p.n, p.colptr, p.rowind, values, x, b)
        x = x + orc.solve_ldlt(sym, P, r)
    return x


def test_ldlt_adjoint_finite_differences(orc):
    # loss = sum(c * x), x = A^{-1} b with A from its lower triangle, solved
    # by L D L^T; the value gradient -db x^T on the pattern (db = A^{-1} c)
    # against central differences of the loss, entry by entry
    p = elasticity3d(4, seed=3)
    sym = orc.analyze(p.n, p.colptr, p.rowind)
    rng = np.random.default_rng(2)
    b = rng.uniform(-1, 1, (p.n, 8))
    c = rng.uniform(-1, 1, (p.n, 8))
    x = _ldlt_solve_refined(orc, sym, p, p.values, b)
    db = _ldlt_solve_refined(orc, sym, p, p.values, c)
    g = orc.values_grad(p.n, p.colptr, p.rowind, x, db)
    col = np.repeat(np.arange(p.n), np.diff(p.colptr))
    lower = 0
    for q in range(p.nnz):
        h = 1e-5 * max(1.0, abs(p.values[q]))
        vp, vm = p.values.copy(), p.values.copy()
        vp[q] += h
        vm[q] -= h
        fd = (np.sum(c * _ldlt_solve_refined(orc, sym, p, vp, b))
              - np.sum(c * _ldlt_solve_refined(orc, sym, p, vm, b))) / (2 * h)
        assert abs(fd - g[q]) <= 1e-6 * max(1.0, abs(fd)), (q, fd, g[q])
        lower += p.rowind[q] >= col[q]
    assert lower > p.n
