"""Pins of the oracle's static pivot replacement (Section III: static
pivoting, no row or column exchange; a pivot below tau = eps * max |a_ij| in
magnitude is replaced by +-tau, +tau for a zero pivot, and counted).

The matrices are built exactly in integers from a chosen factor, on a
dense pattern with the identity ordering: A = L0 D0 L0^T (or L0 U0) where some pivots of D0 (U0) are
zero and the matching column of L0 (and row of U0) is zero beyond the
diagonal, so every step of the elimination is exact and the replaced factor
is known in closed form: L = L0 and D = D0 (U = U0) with tau in place of the
zero pivots.  A pivot of exactly 2 tau is kept.  eps is a power of two and
max |a_ij| an integer, so tau is exact."""
import numpy as np
import pytest

from planted import dense_problem, planted_ldlt, planted_lu, unpack

EPS = 2.0 ** -26
ZEROS = (10, 35)
N = 60


def test_ldlt_replaces_planted_zero_pivots(orc):
    A, L0, d0 = planted_ldlt(N, ZEROS, 3)
    amax = np.max(np.abs(np.tril(A)))
    tau = EPS * amax
    d0[5] = 2 * tau                 # exactly twice the threshold: kept
    A = L0 @ np.diag(d0) @ L0.T     # (changes only a_55; still integers elsewhere, amax unchanged)
    assert np.max(np.abs(np.tril(A))) == amax
    p = dense_problem(A)
    sym = orc.analyze(p.n, p.colptr, p.rowind, user_perm=np.arange(N))
    assert np.array_equal(sym.perm, np.arange(N))
    P, nrep = orc.factor_ldlt(sym, p.colptr, p.rowind, p.values, pivot_eps=EPS, return_nrep=True)
    assert nrep == len(ZEROS)
    F = unpack(sym, P, N)
    d = np.diag(F).copy()
    dref = d0.copy()
    for z in ZEROS:
        dref[z] = tau
    assert np.array_equal(d, dref)
    assert np.array_equal(np.tril(F, -1) + np.eye(N), L0)
    # the factor is that of A + tau at the replaced positions
    Apert = A + np.diag([tau if i in ZEROS else 0.0 for i in range(N)])
    assert np.allclose(L0 @ np.diag(d) @ L0.T, Apert, rtol=0, atol=1e-12)
    # eps = 0: the first zero pivot is a breakdown at its column
    with pytest.raises(orc.ZeroPivot) as e:
        orc.factor_ldlt(sym, p.colptr, p.rowind, p.values)
    assert e.value.col_new == ZEROS[0]


def test_lu_replaces_planted_zero_pivots(orc):
    A, L0, U0 = planted_lu(N, ZEROS, 4)
    u = np.diag(U0).copy()
    amax = np.max(np.abs(A))
    tau = EPS * amax
    p = dense_problem(A)
    sym = orc.analyze(p.n, p.colptr, p.rowind, user_perm=np.arange(N))
    assert np.array_equal(sym.perm, np.arange(N))
    PL, PU, nrep = orc.factor_lu(sym, p.colptr, p.rowind, p.values, pivot_eps=EPS, return_nrep=True)
    assert nrep == len(ZEROS)
    FL, FU = unpack(sym, PL, N), unpack(sym, PU, N)
    Lc = np.tril(FL, -1) + np.eye(N)
    Uc = np.triu(FL) + np.tril(FU, -1).T
    uref = u.copy()
    for z in ZEROS:
        uref[z] = tau
    assert np.array_equal(np.diag(Uc), uref)
    assert np.array_equal(Lc, L0)
    assert np.array_equal(np.triu(Uc, 1), np.triu(U0, 1))
    with pytest.raises(orc.ZeroPivot) as e:
        orc.factor_lu(sym, p.colptr, p.rowind, p.values)
    assert e.value.col_new == ZEROS[0]


def test_small_pivots_two_by_two(orc):
    # [[1, 1], [1, 1]]: d_2 = 0 -> tau = eps; [[1, 2], [3, 6]]: u_22 = 0 -> tau = 6 eps
    cp = np.array([0, 2, 4], np.int64)
    ri = np.array([0, 1, 0, 1], np.int32)
    sym = orc.analyze(2, cp, ri, user_perm=np.arange(2))
    P, nrep = orc.factor_ldlt(sym, cp, ri, np.array([1.0, 1.0, 1.0, 1.0]), pivot_eps=EPS, return_nrep=True)
    assert nrep == 1 and P[0] == 1.0 and P[1] == 1.0 and P[3] == EPS
    PL, PU, nrep = orc.factor_lu(sym, cp, ri, np.array([1.0, 3.0, 2.0, 6.0]), pivot_eps=EPS, return_nrep=True)
    assert nrep == 1 and PL[0] == 1.0 and PL[1] == 3.0 and PL[2] == 2.0 and PL[3] == 6.0 * EPS
    # a negative tiny pivot keeps its sign: [[1, 1], [1, 1 - 1e-12]]
    P, nrep = orc.factor_ldlt(sym, cp, ri, np.array([1.0, 1.0, 1.0, 1.0 - 2.0 ** -40]), pivot_eps=EPS,
                              return_nrep=True)
    assert nrep == 1 and P[3] == -EPS
