"""The Q1 elasticity input (the L D L^T workload: 27-point, 3-dof, SPD once
clamped) pinned by what mechanics fixes, and the oracle's L D L^T and
adjoint on it.

Material: the inverse of the textbook compliance matrix.  Element:
symmetric, rank 18, the six rigid-body motions in its null space; a uniform
strain field stores exactly eps^T D eps per unit volume (Q1 elements
represent linear displacements exactly); a 3-point Gauss rule gives the same
matrix.  Assembly: equal to a brute-force element loop; symmetric,
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


def test_material_matrix_is_the_inverse_compliance():
    # Hooke's law in compliance form: strains from stresses with 1/E on the
    # normal diagonal, -nu/E between normal components, 1/G = 2 (1 + nu)/E
    # on the (engineering) shear diagonal
    for E, nu in [(1.0, 0.3), (2.5, 0.2), (0.7, 0.45)]:
        S = np.zeros((6, 6))
        S[:3, :3] = -nu / E
        S[[0, 1, 2], [0, 1, 2]] = 1.0 / E
        S[[3, 4, 5], [3, 4, 5]] = 2.0 * (1.0 + nu) / E
        assert np.allclose(material_matrix(nu, E) @ S, np.eye(6), atol=1e-12)


def test_element_quadrature_is_exact():
    # the integrand is of degree <= 2 in each coordinate, so a 3-point
    # Gauss-Legendre rule gives the same stiffness as the element's 2-point one
    from gen import strain_matrix
    t, w = np.polynomial.legendre.leggauss(3)
    t, w = 0.5 * (t + 1.0), 0.5 * w
    D = material_matrix(0.3)
    K3 = np.zeros((24, 24))
    for i in range(3):
        for j in range(3):
            for k in range(3):
                B = strain_matrix(t[i], t[j], t[k])
                K3 += w[i] * w[j] * w[k] * B.T @ D @ B
    assert np.max(np.abs(K3 - element_stiffness(0.3))) <= 1e-14 * np.max(np.abs(K3))


@pytest.mark.parametrize("n", [4, 5])
def test_assembly_brute_force(n):
    # element by element into a dense matrix, nodes addressed by their
    # coordinates: free node (x, y, z), 1 <= x, y, z <= n-2, has index
    # (x-1) + m (y-1) + m^2 (z-1); moduli drawn in element order, x fastest
    seed, sigma = 11, 0.5
    p = elasticity3d(n, seed=seed, sigma=sigma)
    m = n - 2
    E = np.random.default_rng(seed).lognormal(0.0, sigma, (n - 1) ** 3)
    Ke = element_stiffness(0.3)
    A = np.zeros((p.n, p.n))
    e = 0
    for z in range(n - 1):
        for y in range(n - 1):
            for x in range(n - 1):
                dofs = []
                for a in range(8):
                    cx, cy, cz = a & 1, (a >> 1) & 1, (a >> 2) & 1
                    X, Y, Z = x + cx, y + cy, z + cz
                    inner = all(1 <= c <= n - 2 for c in (X, Y, Z))
                    node = (X - 1) + m * (Y - 1) + m * m * (Z - 1)
                    dofs += [3 * node + comp if inner else -1 for comp in range(3)]
                for i, gi in enumerate(dofs):
                    for j, gj in enumerate(dofs):
                        if gi >= 0 and gj >= 0:
                            A[gi, gj] += E[e] * Ke[i, j]
                e += 1
    G = sp.csc_matrix((p.values, p.rowind, p.colptr), shape=(p.n, p.n)).toarray()
    assert np.max(np.abs(G - A)) <= 1e-14 * np.max(np.abs(A))
