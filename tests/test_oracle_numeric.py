"""Pins of the oracle's numeric factorization and solve.

The supernodal method reaches, up to rounding order, the unique Cholesky
factor of P A P^T (Section III: the structure is fixed by the analysis,
static pivoting).  The pins below check it against a LAPACK dense Cholesky,
closed forms of constant-coefficient Laplacians, and backward-error
invariants of the solve.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from gen import grid_laplacian, make_config, random_spd, rhs


def _dense(p):
    return sp.csc_matrix((p.values, p.rowind, p.colptr), shape=(p.n, p.n)).toarray()


def _factor_dense(orc, s, P):
    ri, ci, v = orc.unpack(s, P)
    return sp.csc_matrix((v, (ri, ci)), shape=(s.n, s.n)).toarray()


@pytest.mark.parametrize("n,dens,seed", [(1, 0.0, 1), (5, 0.5, 2), (60, 0.05, 3), (150, 0.02, 4), (200, 0.1, 5)])
@pytest.mark.parametrize("split", [256, 7])
def test_factor_matches_dense_cholesky(orc, n, dens, seed, split):
    p = random_spd(n, dens, seed)
    s = orc.analyze(p.n, p.colptr, p.rowind, leaf=8, split_width=split)
    P = orc.factor(s, p.colptr, p.rowind, p.values)
    L = _factor_dense(orc, s, P)
    A = _dense(p)
    PA = A[np.ix_(s.perm, s.perm)]
    Lref = np.linalg.cholesky(PA)
    assert np.max(np.abs(L - Lref)) <= 1e-13 * np.max(np.abs(Lref))
    # explicit zeros added by amalgamation stay zero (within rounding) in the factor
    assert np.linalg.norm(PA - L @ L.T) <= 1e-14 * np.linalg.norm(PA) * max(1, np.sqrt(n))


def test_lower_triangle_input_is_enough(orc):
    p = random_spd(80, 0.06, 11)
    cols = np.repeat(np.arange(p.n), np.diff(p.colptr))
    keep = p.rowind >= cols
    cp = np.concatenate([[0], np.cumsum(np.bincount(cols[keep], minlength=p.n))]).astype(np.int64)
    s_full = orc.analyze(p.n, p.colptr, p.rowind)
    s_low = orc.analyze(p.n, cp, p.rowind[keep])
    assert np.array_equal(s_full.perm, s_low.perm)
    P1 = orc.factor(s_full, p.colptr, p.rowind, p.values)
    P2 = orc.factor(s_low, cp, p.rowind[keep], p.values[keep])
    assert np.array_equal(P1, P2)


def test_1d_laplacian_closed_form(orc):
    # tridiag(-1, 2, -1) in natural order: l_kk = sqrt((k+1)/k), l_{k+1,k} = -sqrt(k/(k+1)) (1-based k)
    n = 300
    p = grid_laplacian((n,))
    s = orc.analyze(p.n, p.colptr, p.rowind, user_perm=np.arange(n))
    assert np.array_equal(s.perm, np.arange(n))
    L = _factor_dense(orc, s, orc.factor(s, p.colptr, p.rowind, p.values))
    k = np.arange(1, n + 1, dtype=np.float64)
    assert np.allclose(np.diag(L), np.sqrt((k + 1) / k), rtol=1e-14, atol=0)
    assert np.allclose(np.diag(L, -1), -np.sqrt(k[:-1] / (k[:-1] + 1)), rtol=1e-13, atol=0)
    # log det of tridiag(-1,2,-1) of order n is log(n+1)
    assert abs(orc.logdet(s, orc.factor(s, p.colptr, p.rowind, p.values)) - np.log(n + 1)) < 1e-11


def _laplacian_logdet(dims, shift):
    lam = np.zeros(())
    for d in dims:
        ev = 2.0 - 2.0 * np.cos(np.arange(1, d + 1) * np.pi / (d + 1))
        lam = np.add.outer(lam, ev) if lam.ndim else ev
    return float(np.sum(np.log(lam + shift)))


@pytest.mark.parametrize("dims,shift", [((64, 64), 0.0), ((17, 9), 0.0), ((12, 10, 8), 1e-3), ((20, 20, 20), 1e-3)])
def test_logdet_closed_form(orc, dims, shift):
    p = grid_laplacian(dims, shift=shift)
    s = orc.analyze(p.n, p.colptr, p.rowind)
    P = orc.factor(s, p.colptr, p.rowind, p.values)
    ref = _laplacian_logdet(dims, shift)
    assert abs(orc.logdet(s, P) - ref) <= 1e-10 * abs(ref)


def test_config1_solve_backward_error(orc):
    p = make_config(1)
    s = orc.analyze(p.n, p.colptr, p.rowind)
    P = orc.factor(s, p.colptr, p.rowind, p.values)
    x, om = orc.solve_refined(s, P, p.colptr, p.rowind, p.values, p.b)
    assert om[-1] <= 1e-14
    # factor residual, exact on the full pattern
    L = _factor_dense(orc, s, P)
    A = _dense(p)
    PA = A[np.ix_(s.perm, s.perm)]
    assert np.linalg.norm(PA - L @ L.T) / np.linalg.norm(PA) <= 1e-13
    assert np.linalg.norm(A @ x - p.b) <= 1e-12 * np.linalg.norm(p.b) * np.linalg.cond(A)


def test_manufactured_solution(orc):
    p = grid_laplacian((15, 14, 13), shift=1e-3)
    s = orc.analyze(p.n, p.colptr, p.rowind)
    P = orc.factor(s, p.colptr, p.rowind, p.values)
    xs = rhs(p.n, 3, 5)
    b = np.asfortranarray(_dense(p) @ xs)
    x, om = orc.solve_refined(s, P, p.colptr, p.rowind, p.values, b)
    assert om[-1] <= 1e-14
    kappa = np.linalg.cond(_dense(p))
    assert np.max(np.abs(x - xs)) <= 10 * kappa * om[-1] * np.max(np.abs(xs)) + 1e-14


def _first_bad_pivot(A):
    """Plain Gaussian elimination without pivoting: first k with Schur pivot <= 0."""
    S = A.copy()
    for k in range(S.shape[0]):
        if not S[k, k] > 0:
            return k
        S[k + 1:, k + 1:] -= np.outer(S[k + 1:, k], S[k, k + 1:]) / S[k, k]
    return -1


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_not_positive_definite(orc, seed):
    p = grid_laplacian((9, 8))
    rng = np.random.default_rng(seed)
    vals = p.values.copy()
    cols = np.repeat(np.arange(p.n), np.diff(p.colptr))
    victim = int(rng.integers(0, p.n))
    vals[(p.rowind == victim) & (cols == victim)] = -0.5 - rng.uniform()
    s = orc.analyze(p.n, p.colptr, p.rowind, leaf=6)
    A = sp.csc_matrix((vals, p.rowind, p.colptr), shape=(p.n, p.n)).toarray()
    expect = _first_bad_pivot(A[np.ix_(s.perm, s.perm)])
    assert expect >= 0
    with pytest.raises(orc.NotPositiveDefinite) as ei:
        orc.factor(s, p.colptr, p.rowind, vals)
    assert ei.value.col_new == expect
    assert ei.value.col_orig == s.perm[expect]


def test_nan_is_a_breakdown(orc):
    p = grid_laplacian((6, 6))
    vals = p.values.copy()
    vals[0] = np.nan
    s = orc.analyze(p.n, p.colptr, p.rowind)
    with pytest.raises(orc.NotPositiveDefinite):
        orc.factor(s, p.colptr, p.rowind, vals)


def test_omega_conventions(orc):
    r = np.array([0.0, 0.0, 1e-3])
    s = np.array([0.0, 2.0, 1.0])
    assert orc.omega(r, s) == pytest.approx(1e-3)
    assert orc.omega(np.array([1.0]), np.array([0.0])) == np.inf


@pytest.mark.parametrize("dims", [(12, 12, 12), (40, 40)])
def test_subtree_factor_equals_full_factor(orc, dims):
    # the bounded CPU sample factors one subtree of the block elimination
    # tree: every update into its blocks comes from inside it (postorder), so
    # its panels equal those of the full factorization bit for bit, and the
    # subtrees' ranges nest as in a tree
    p = grid_laplacian(dims, shift=1e-3)
    s = orc.analyze(p.n, p.colptr, p.rowind, leaf=16)
    first = orc.subtree_first(s)
    nc = int(s.stats["ncblk"])
    for k in range(nc):
        c = int(s.cparent[k])
        assert first[k] <= k
        if c >= 0:
            assert first[c] <= first[k] and k < c
    P = orc.factor(s, p.colptr, p.rowind, p.values)
    sizes = np.arange(nc) - first
    for root in (int(np.argmax(np.where(sizes < nc // 3, sizes, -1))), nc - 1, 0):
        Ps, _, _ = orc.factor_subtree(s, p.colptr, p.rowind, p.values, root)
        lo, hi = int(s.panel_off[first[root]]), int(s.panel_off[root + 1])
        assert np.array_equal(Ps[lo:hi], P[lo:hi])
