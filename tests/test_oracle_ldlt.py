"""Pins of the oracle's L D L^T factorization (the symmetric-indefinite
variant of the method, static pivoting) against what the mathematics fixes:
the factorization without pivoting is unique when it exists, so rebuilding
P A P^T from L and D pins it; Sylvester's law of inertia fixes the number of
negative pivots; a dense library log-determinant fixes sum log |d|; on SPD
matrices d_j = l_jj^2 and L_ldl = L_chol diag(1/l_jj) relate it to the
separately pinned Cholesky factor."""
import numpy as np
import pytest
import scipy.sparse as sp

from gen import grid_laplacian, random_spd
from gen.stencils import Problem


def _unit_l_and_d(orc, sym, P, n):
    ri, ci, v = orc.unpack(sym, P)
    diag = ri == ci
    D = np.zeros(n)
    D[ri[diag]] = v[diag]
    Lu = sp.csc_matrix((v[~diag], (ri[~diag], ci[~diag])), shape=(n, n)) + sp.identity(n, format="csc")
    return Lu, D


def _quasi_definite(n1, n2, seed):
    # K = [[H, B^T], [B, -C]] with H, C SPD: quasi-definite, so every
    # symmetric permutation has an L D L^T; inertia (n1 positive, n2 negative)
    rng = np.random.default_rng(seed)
    H = random_spd(n1, 0.05, seed).values
    p1 = random_spd(n1, 0.05, seed)
    H = sp.csc_matrix((p1.values, p1.rowind, p1.colptr), shape=(n1, n1))
    p2 = random_spd(n2, 0.08, seed + 1)
    Cm = sp.csc_matrix((p2.values, p2.rowind, p2.colptr), shape=(n2, n2))
    B = sp.random(n2, n1, density=0.05, random_state=rng, format="csc") * 2.0
    K = sp.bmat([[H, B.T], [B, -Cm]], format="csc")
    K.sort_indices()
    return Problem(n1 + n2, K.indptr.astype(np.int64), K.indices.astype(np.int32), K.data.copy()), K


def _cases():
    yield "spd_rand", random_spd(300, 0.02, 3), None
    yield "grid3", grid_laplacian((7, 6, 5), shift=1e-3), None
    yield "qd", *_quasi_definite(120, 60, 5)


@pytest.mark.parametrize("split", [256, 8])
def test_ldlt_rebuilds_the_matrix(orc, split):
    for name, p, _ in _cases():
        sym = orc.analyze(p.n, p.colptr, p.rowind, split_width=split)
        P = orc.factor_ldlt(sym, p.colptr, p.rowind, p.values)
        Lu, D = _unit_l_and_d(orc, sym, P, p.n)
        A = sp.csc_matrix((p.values, p.rowind, p.colptr), shape=(p.n, p.n))
        PA = A[sym.perm][:, sym.perm]
        err = sp.linalg.norm(PA - Lu @ sp.diags(D) @ Lu.T) / sp.linalg.norm(PA)
        assert err <= 1e-13, (name, err)


def test_ldlt_inertia_and_log_abs_det(orc):
    p, K = _quasi_definite(120, 60, 11)
    sym = orc.analyze(p.n, p.colptr, p.rowind)
    P = orc.factor_ldlt(sym, p.colptr, p.rowind, p.values)
    lad, nneg = orc.logabsdet_ldlt(sym, P)
    ev = np.linalg.eigvalsh(K.toarray())
    assert nneg == int(np.sum(ev < 0)) == 60
    sign, ref = np.linalg.slogdet(K.toarray())
    assert abs(lad - ref) <= 1e-10 * abs(ref)


def test_ldlt_of_spd_is_scaled_cholesky(orc):
    p = grid_laplacian((9, 8, 7), shift=1e-3)
    sym = orc.analyze(p.n, p.colptr, p.rowind)
    Pc = orc.factor(sym, p.colptr, p.rowind, p.values)
    Pl = orc.factor_ldlt(sym, p.colptr, p.rowind, p.values)
    ri, ci, vc = orc.unpack(sym, Pc)
    _, _, vl = orc.unpack(sym, Pl)
    dc = np.zeros(p.n)
    dc[ri[ri == ci]] = vc[ri == ci]
    expect = np.where(ri == ci, vc ** 2, vc / dc[ci])
    assert np.max(np.abs(vl - expect) / np.maximum(np.abs(expect), 1e-300)) <= 1e-12


def test_ldlt_solve(orc):
    for name, p, _ in _cases():
        sym = orc.analyze(p.n, p.colptr, p.rowind)
        P = orc.factor_ldlt(sym, p.colptr, p.rowind, p.values)
        rng = np.random.default_rng(7)
        b = rng.uniform(-1, 1, (p.n, 2))
        x = orc.solve_ldlt(sym, P, b)
        r, s = orc.residual(p.n, p.colptr, p.rowind, p.values, x, b)
        assert orc.omega(r, s) <= 1e-12, name


def test_ldlt_zero_pivot(orc):
    # [[0, 1], [1, 0]]: the first pivot is zero in any order;
    # [[1, 1], [1, 1]]: the second pivot is exactly 1 - 1 = 0
    for vals, first in [(np.array([0.0, 1.0, 1.0, 0.0]), True), (np.array([1.0, 1.0, 1.0, 1.0]), False)]:
        colptr = np.array([0, 2, 4], np.int64)
        rowind = np.array([0, 1, 0, 1], np.int32)
        sym = orc.analyze(2, colptr, rowind)
        with pytest.raises(orc.ZeroPivot) as e:
            orc.factor_ldlt(sym, colptr, rowind, vals)
        assert e.value.col_new == (0 if first else 1)
        assert e.value.col_orig == int(sym.perm[e.value.col_new])
