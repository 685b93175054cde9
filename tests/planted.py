"""Matrices with planted zero pivots for the static pivoting tests, built
exactly in integers from a chosen factor on a dense pattern (zeros kept as
entries) so that the identity ordering is the final order: A = L0 D0 L0^T
or A = L0 U0, where the planted zero pivots' columns of L0 (and rows of U0)
are zero beyond the diagonal.  Every step of the elimination is then exact,
and the factor with the zero pivots replaced by tau is L0 with D0 (U0)
holding tau at those positions."""
import numpy as np

from gen.stencils import Problem


def dense_problem(A):
    """A dense pattern: the elimination tree is a path, so with the identity
    ordering the final order is the identity."""
    n = A.shape[0]
    colptr = np.arange(0, n * n + 1, n, dtype=np.int64)
    rowind = np.tile(np.arange(n, dtype=np.int32), n)
    return Problem(n, colptr, rowind, np.asfortranarray(A).ravel(order="F").copy())


def unit_lower(rng, n, zero_cols, per_col=3):
    """Unit lower triangular with up to per_col entries in {-2..2} below the
    diagonal of each column, none in the columns zero_cols."""
    L0 = np.eye(n)
    for c in range(n - 1):
        if c in zero_cols:
            continue
        for r in rng.choice(np.arange(c + 1, n), size=min(per_col, n - c - 1), replace=False):
            L0[r, c] = float(rng.integers(-2, 3))
    return L0


def planted_ldlt(n, zeros, seed, pivots=(-1.0, 1.0, 2.0)):
    """(A, L0, d0) with d0 = 0 at the positions zeros, else from pivots."""
    rng = np.random.default_rng(seed)
    L0 = unit_lower(rng, n, zeros)
    d0 = rng.choice(list(pivots), size=n)
    d0[list(zeros)] = 0.0
    return L0 @ np.diag(d0) @ L0.T, L0, d0


def planted_lu(n, zeros, seed, pivots=(-3.0, 1.0, 2.0)):
    """(A, L0, U0) with u_jj = 0 at the positions zeros, else from pivots."""
    rng = np.random.default_rng(seed)
    L0 = unit_lower(rng, n, zeros)
    U0t = unit_lower(rng, n, zeros)
    u = rng.choice(list(pivots), size=n)
    u[list(zeros)] = 0.0
    U0 = np.diag(u) @ U0t.T
    return L0 @ U0, L0, U0


def unpack(sym, P, n):
    """Dense lower panel contents (diagonal blocks square) in the final order."""
    a = sym.arrays
    F = np.zeros((n, n))
    for k in range(len(a["fcol"])):
        f, l, ld, off = int(a["fcol"][k]), int(a["lcol"][k]), int(a["stride"][k]), int(a["panel_off"][k])
        wd = l - f + 1
        blk = P[off:off + ld * wd].reshape(wd, ld).T
        F[f:f + wd, f:f + wd] = blk[:wd]
        rows = []
        for b in range(int(a["bptr"][k]) + 1, int(a["bptr"][k + 1])):
            rows.extend(range(int(a["frow"][b]), int(a["lrow"][b]) + 1))
        if rows:
            F[np.array(rows), f:f + wd] = blk[wd:]
    return F
