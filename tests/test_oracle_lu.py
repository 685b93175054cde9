"""Pins of the oracle's L U factorization with static pivoting (the
non-symmetric variant of the method on the pattern of A + A^T) against what
the mathematics fixes: L U without pivoting (unit L) is unique when it
exists, so rebuilding P A P^T pins it; A^T = (U^T D^{-1}) (D L^T) with
D = diag(U) relates the factors of A and A^T; on SPD matrices L U is the
(separately pinned) L D L^T with U = D L^T; a dense library log-determinant
and sign fix prod u_jj."""
import numpy as np
import pytest
import scipy.sparse as sp

from gen import convection_diffusion, grid_laplacian
from gen.stencils import Problem


def _dense_lu(sym, PL, PU):
    """Dense unit-lower L and upper U of P A P^T from the two panel arrays."""
    a = sym.arrays
    n = sym.n
    L = np.eye(n)
    U = np.zeros((n, n))
    for k in range(len(a["fcol"])):
        f, l, ld, off = int(a["fcol"][k]), int(a["lcol"][k]), int(a["stride"][k]), int(a["panel_off"][k])
        wd = l - f + 1
        blk = PL[off:off + ld * wd].reshape(wd, ld).T   # [row, col] of the panel
        ublk = PU[off:off + ld * wd].reshape(wd, ld).T
        for c in range(wd):
            for r in range(wd):
                if r > c:
                    L[f + r, f + c] = blk[r, c]
                else:
                    U[f + r, f + c] = blk[r, c]
            for b in range(int(a["bptr"][k]) + 1, int(a["bptr"][k + 1])):
                for g in range(int(a["frow"][b]), int(a["lrow"][b]) + 1):
                    pr = int(a["coefind"][b]) + g - int(a["frow"][b])
                    L[g, f + c] = blk[pr, c]
                    U[f + c, g] = ublk[pr, c]
    return L, U


def _transpose(p):
    A = sp.csc_matrix((p.values, p.rowind, p.colptr), shape=(p.n, p.n)).T.tocsc()
    A.sort_indices()
    return Problem(p.n, A.indptr.astype(np.int64), A.indices.astype(np.int32), A.data.copy())


def _unsym_random(n, seed):
    rng = np.random.default_rng(seed)
    M = sp.random(n, n, density=0.03, random_state=rng, format="csc")
    M = M + M.T.multiply(rng.uniform(-1, 1)) + sp.identity(n) * 0.0
    A = M.tocsc()
    A = A + sp.diags(np.abs(A).sum(axis=1).A1 + 1.0)   # row diagonally dominant
    A = A.tocsc()
    A.sort_indices()
    return Problem(n, A.indptr.astype(np.int64), A.indices.astype(np.int32), A.data.copy())


def _cases():
    yield "convdiff3", convection_diffusion((6, 5, 4), seed=3)
    yield "convdiff2", convection_diffusion((15, 12), seed=4)
    yield "rand", _unsym_random(150, 5)


@pytest.mark.parametrize("split", [256, 8])
def test_lu_rebuilds_the_matrix(orc, split):
    for name, p in _cases():
        sym = orc.analyze(p.n, p.colptr, p.rowind, split_width=split)
        PL, PU = orc.factor_lu(sym, p.colptr, p.rowind, p.values)
        L, U = _dense_lu(sym, PL, PU)
        A = sp.csc_matrix((p.values, p.rowind, p.colptr), shape=(p.n, p.n)).toarray()
        PA = A[np.ix_(sym.perm, sym.perm)]
        err = np.linalg.norm(PA - L @ U) / np.linalg.norm(PA)
        assert err <= 1e-13, (name, err)
        assert np.allclose(np.triu(L, 1), 0) and np.allclose(np.tril(U, -1), 0)


def test_lu_of_transpose(orc):
    p = convection_diffusion((7, 6, 3), seed=8)
    q = _transpose(p)
    sym = orc.analyze(p.n, p.colptr, p.rowind)   # the pattern is symmetric: same analysis for A^T
    L, U = _dense_lu(sym, *orc.factor_lu(sym, p.colptr, p.rowind, p.values))
    Lt, Ut = _dense_lu(sym, *orc.factor_lu(sym, q.colptr, q.rowind, q.values))
    D = np.diag(U)
    assert np.allclose(Lt, U.T / D[None, :], rtol=1e-11, atol=1e-13)
    assert np.allclose(Ut, D[:, None] * L.T, rtol=1e-11, atol=1e-13)


def test_lu_of_spd_is_ldlt(orc):
    p = grid_laplacian((8, 7, 5), shift=1e-3)
    sym = orc.analyze(p.n, p.colptr, p.rowind)
    L, U = _dense_lu(sym, *orc.factor_lu(sym, p.colptr, p.rowind, p.values))
    P = orc.factor_ldlt(sym, p.colptr, p.rowind, p.values)
    ri, ci, v = orc.unpack(sym, P)
    Lldl = np.eye(p.n)
    D = np.zeros(p.n)
    for r, c, x in zip(ri, ci, v):
        if r == c:
            D[r] = x
        else:
            Lldl[r, c] = x
    assert np.allclose(L, Lldl, rtol=1e-12, atol=1e-14)
    assert np.allclose(U, D[:, None] * Lldl.T, rtol=1e-12, atol=1e-14)


def test_lu_log_abs_det_and_sign(orc):
    for name, p in _cases():
        sym = orc.analyze(p.n, p.colptr, p.rowind)
        PL, _ = orc.factor_lu(sym, p.colptr, p.rowind, p.values)
        lad, nneg = orc.logabsdet_lu(sym, PL)
        A = sp.csc_matrix((p.values, p.rowind, p.colptr), shape=(p.n, p.n)).toarray()
        sign, ref = np.linalg.slogdet(A)
        assert abs(lad - ref) <= 1e-10 * max(1.0, abs(ref)), name
        assert (-1) ** nneg == sign, name


def test_lu_solve(orc):
    for name, p in _cases():
        sym = orc.analyze(p.n, p.colptr, p.rowind)
        PL, PU = orc.factor_lu(sym, p.colptr, p.rowind, p.values)
        b = np.random.default_rng(9).uniform(-1, 1, (p.n, 3))
        x = orc.solve_lu(sym, PL, PU, b)
        A = sp.csc_matrix((p.values, p.rowind, p.colptr), shape=(p.n, p.n))
        r = b - A @ x
        den = abs(A) @ np.abs(x) + np.abs(b)
        assert np.max(np.abs(r) / den) <= 1e-13, name


def test_lu_zero_pivot(orc):
    colptr = np.array([0, 2, 4], np.int64)
    rowind = np.array([0, 1, 0, 1], np.int32)
    # [[0, 1], [1, 0]]: the first pivot is zero; [[1, 2], [3, 6]]: the second is 6 - 3 * 2 = 0
    for vals, col in [(np.array([0.0, 1.0, 1.0, 0.0]), 0), (np.array([1.0, 3.0, 2.0, 6.0]), 1)]:
        sym = orc.analyze(2, colptr, rowind)
        with pytest.raises(orc.ZeroPivot) as e:
            orc.factor_lu(sym, colptr, rowind, vals)
        assert e.value.col_new == col


def test_convection_diffusion_workload_size():
    # 7-point pattern: n + 2 * (sum over axes of the edges along that axis);
    # checked on a small grid by the generator, then the stated size of the
    # 80^3 workload (512,000 unknowns, 3,545,600 entries) from the same count
    def count(d):
        return d ** 3 + 2 * 3 * d * d * (d - 1)
    p = convection_diffusion((9, 9, 9), seed=1)
    assert p.n == 729 and p.nnz == count(9)
    assert count(80) == 3545600
    from gen import make_config, CONFIG_NAMES
    assert CONFIG_NAMES[3] == "convdiff3d_7pt_80^3"
