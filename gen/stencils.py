"""Synthetic sparse matrices shaped like the paper's workloads.

The paper measures on matrices of the University of Florida collection
(Table 1: 0.5-1.6 million unknowns, SPD / symmetric-indefinite /
unsymmetric).  Those matrices are not available, so structured stencil
matrices of the same order of size stand in for them.

Storage convention: compressed sparse column (CSC), 0-based, row indices
sorted ascending inside every column, no duplicates, the FULL symmetric
pattern (both triangles).  ``colptr`` is int64, ``rowind`` int32, values
float64.  Grid nodes are numbered lexicographically with x fastest:
idx = x + nx * (y + ny * z).  Out-of-grid neighbours are dropped
(Dirichlet boundary).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

CONFIG_NAMES = {
    1: "laplace2d_5pt_64x64",
    2: "laplace3d_7pt_100^3_shift1e-3",
    3: "convdiff3d_7pt_80^3",
    4: "batch512_wgrid2d_16-96",
    5: "elasticity3d_q1_40^3_3dof",
}


@dataclass
class Problem:
    n: int
    colptr: np.ndarray  # int64 [n+1]
    rowind: np.ndarray  # int32 [nnz]
    values: np.ndarray  # float64 [nnz]
    b: np.ndarray | None = None  # float64 [n, nrhs], column-major per RHS
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.colptr[-1])


def _coo_to_csc(n: int, rows: np.ndarray, cols: np.ndarray, vals: np.ndarray):
    """Sort COO triplets into CSC (rows ascending within a column).

    Duplicate (row, col) pairs are summed.
    """
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    vals = np.asarray(vals, dtype=np.float64)
    key = cols * n + rows
    order = np.argsort(key, kind="stable")
    key = key[order]
    vals = vals[order]
    uniq, start = np.unique(key, return_index=True)
    summed = np.add.reduceat(vals, start) if len(vals) else vals
    ucols = uniq // n
    urows = uniq - ucols * n
    colptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(colptr, ucols + 1, 1)
    colptr = np.cumsum(colptr)
    return colptr.astype(np.int64), urows.astype(np.int32), summed.astype(np.float64)


def grid_laplacian(dims, diag: float | None = None, shift: float = 0.0, offdiag: float = -1.0) -> Problem:
    """Constant-coefficient 5-point (2-D) or 7-point (3-D) Laplacian.

    a_ii = 2*d + shift (d = number of dimensions) unless ``diag`` is given,
    a_ij = ``offdiag`` for grid neighbours.  A 1-D tuple gives tridiag(-1,2,-1).
    """
    dims = tuple(int(d) for d in dims)
    nd = len(dims)
    n = int(np.prod(dims))
    if diag is None:
        diag = 2.0 * nd
    diag = diag + shift
    coords = np.indices(dims[::-1]).reshape(nd, -1)[::-1]  # coords[0] = x (fastest)
    idx = np.arange(n, dtype=np.int64)
    rows = [idx]
    cols = [idx]
    vals = [np.full(n, diag)]
    stride = 1
    for d in range(nd):
        ok = coords[d] < dims[d] - 1
        a = idx[ok]
        bnb = a + stride
        rows += [a, bnb]
        cols += [bnb, a]
        vals += [np.full(len(a), offdiag), np.full(len(a), offdiag)]
        stride *= dims[d]
    colptr, rowind, values = _coo_to_csc(n, np.concatenate(rows), np.concatenate(cols), np.concatenate(vals))
    return Problem(n, colptr, rowind, values, name="laplace%dd_%s" % (nd, "x".join(map(str, dims))),
                   meta={"dims": dims, "diag": diag, "offdiag": offdiag, "shift": shift})


def convection_diffusion(dims, seed: int, cmax: float = 0.5) -> Problem:
    """Unsymmetric 7-point (3-D) or 5-point (2-D) convection-diffusion
    stencil: for every cell i and axis d a convection coefficient
    b ~ uniform[-cmax, cmax] (drawn per cell, axis by axis), a_{i,i+e_d} =
    -1 + b/2, a_{i,i-e_d} = -1 - b/2 (central differences), a_ii = 2 * ndim;
    out-of-grid neighbours are dropped.  With cmax <= 2 every interior row
    is weakly diagonally dominant (sum of the off-diagonal magnitudes equal
    to a_ii) and every boundary row strictly, so the matrix is irreducibly
    diagonally dominant; the pattern is symmetric, the values are not."""
    dims = tuple(int(d) for d in dims)
    nd = len(dims)
    n = int(np.prod(dims))
    rng = np.random.default_rng(seed)
    coords = np.indices(dims[::-1]).reshape(nd, -1)[::-1]
    idx = np.arange(n, dtype=np.int64)
    rows, cols, vals = [idx], [idx], [np.full(n, 2.0 * nd)]
    stride = 1
    for d in range(nd):
        bconv = rng.uniform(-cmax, cmax, n)
        up = coords[d] < dims[d] - 1
        dn = coords[d] > 0
        a = idx[up]
        rows.append(a); cols.append(a + stride); vals.append(-1.0 + 0.5 * bconv[up])
        a = idx[dn]
        rows.append(a); cols.append(a - stride); vals.append(-1.0 - 0.5 * bconv[dn])
        stride *= dims[d]
    colptr, rowind, values = _coo_to_csc(n, np.concatenate(rows), np.concatenate(cols), np.concatenate(vals))
    return Problem(n, colptr, rowind, values, name="convdiff%dd_%s" % (nd, "x".join(map(str, dims))),
                   meta={"dims": dims, "cmax": cmax, "seed": seed})


def random_pattern(n: int, density: float, seed: int):
    """Random symmetric pattern (with the full diagonal) as CSC index arrays."""
    rng = np.random.default_rng(seed)
    m = max(0, int(round(density * n * (n - 1) / 2)))
    i = rng.integers(0, n, size=m)
    j = rng.integers(0, n, size=m)
    keep = i != j
    i, j = i[keep], j[keep]
    rows = np.concatenate([i, j, np.arange(n)])
    cols = np.concatenate([j, i, np.arange(n)])
    colptr, rowind, _ = _coo_to_csc(n, rows, cols, np.ones(len(rows)))
    return colptr, rowind


def random_spd(n: int, density: float, seed: int) -> Problem:
    """Random sparse symmetric, strictly diagonally dominant matrix (SPD).

    Off-diagonal values uniform in [-1, 1]; a_ii = 1 + sum_j |a_ij|.
    """
    rng = np.random.default_rng(seed)
    colptr, rowind = random_pattern(n, density, seed)
    cols = np.repeat(np.arange(n), np.diff(colptr))
    rows = rowind.astype(np.int64)
    upper = rows < cols
    vals = np.zeros(len(rows))
    # draw one value per unordered pair (stored at the upper entry), mirror it
    vu = rng.uniform(-1.0, 1.0, size=int(upper.sum()))
    vals[upper] = vu
    # mirror: entry (r, c) lower gets value of (c, r) upper
    key_up = cols[upper] * n + rows[upper]          # key of (row=c', col=...) ordering
    lower = rows > cols
    key_lo = rows[lower] * n + cols[lower]          # transpose key matches upper's (col, row)
    order = np.argsort(key_up)
    pos = np.searchsorted(key_up[order], key_lo)
    vals[lower] = vu[order][pos]
    offsum = np.zeros(n)
    np.add.at(offsum, cols[rows != cols], np.abs(vals[rows != cols]))
    diag = rows == cols
    vals[diag] = 1.0 + offsum[cols[diag]]
    return Problem(n, colptr, rowind, vals, name="random_spd_n%d_s%d" % (n, seed),
                   meta={"density": density, "seed": seed})


def rhs(n: int, nrhs: int, seed: int) -> np.ndarray:
    """Right-hand sides uniform in [-1, 1], drawn as (nrhs, n) then transposed.

    Returned as a Fortran-ordered (n, nrhs) array: column r is RHS r.
    """
    rng = np.random.default_rng(seed)
    return np.asfortranarray(rng.uniform(-1.0, 1.0, size=(nrhs, n)).T)


def weighted_grid(nx: int, ny: int, rng) -> Problem:
    """Weighted graph Laplacian of an nx x ny grid with ghost edges: every grid
    edge and every boundary-to-ghost edge (one per missing neighbour of a
    boundary node) gets a weight ~ lognormal(0, 1); a_ij = -w_ij for grid
    edges, a_ii = sum of the weights of all edges at i (ghost edges included),
    so A is symmetric positive definite.  Draw order: x-edges, y-edges, ghost
    edges (x-low, x-high, y-low, y-high)."""
    n = nx * ny
    x = np.arange(n) % nx
    y = np.arange(n) // nx
    idx = np.arange(n, dtype=np.int64)
    ex = idx[x < nx - 1]
    ey = idx[y < ny - 1]
    wx = rng.lognormal(0.0, 1.0, len(ex))
    wy = rng.lognormal(0.0, 1.0, len(ey))
    diag = np.zeros(n)
    np.add.at(diag, ex, wx)
    np.add.at(diag, ex + 1, wx)
    np.add.at(diag, ey, wy)
    np.add.at(diag, ey + nx, wy)
    for ghost in (x == 0, x == nx - 1, y == 0, y == ny - 1):
        g = idx[ghost]
        diag[g] += rng.lognormal(0.0, 1.0, len(g))
    rows = np.concatenate([idx, ex, ex + 1, ey, ey + nx])
    cols = np.concatenate([idx, ex + 1, ex, ey + nx, ey])
    vals = np.concatenate([diag, -wx, -wx, -wy, -wy])
    colptr, rowind, values = _coo_to_csc(n, rows, cols, vals)
    return Problem(n, colptr, rowind, values, name="wgrid_%dx%d" % (nx, ny), meta={"dims": (nx, ny)})


def grid_batch(nsys: int = 512, seed: int = 1004, lo: int = 16, hi: int = 96, nrhs: int = 1):
    """Independent weighted grid Laplacians of uneven size: sides nx, ny drawn
    uniformly from {lo..hi}, then each system's weights (``weighted_grid``)
    and right-hand side uniform in [-1, 1], system by system."""
    rng = np.random.default_rng(seed)
    sides = rng.integers(lo, hi + 1, size=(nsys, 2))
    out = []
    for q in range(nsys):
        p = weighted_grid(int(sides[q, 0]), int(sides[q, 1]), rng)
        p.b = np.asfortranarray(rng.uniform(-1.0, 1.0, (nrhs, p.n)).T)
        out.append(p)
    return out


def make_config(i: int, seed: int | None = None) -> Problem:
    """The benchmark workloads.

    1: 2-D 5-point Laplacian on a 64x64 grid, a_ii = 4, a_ij = -1, one RHS.
    2: 3-D 7-point Laplacian on a 100^3 grid plus a diagonal shift 1e-3, one RHS.
    3: 3-D convection-diffusion 7-point stencil on an 80^3 grid (N = 512,000,
       unsymmetric values on a symmetric pattern; the L U workload),
       convection coefficients drawn with the config's seed, four RHS.
    5: clamped Q1 elasticity on a 42^3-node mesh (40^3 free nodes, 3 dof
       each, N = 192,000, 27-point 3-dof stencil), element moduli
       lognormal(0, 0.5) drawn with the config's seed, eight RHS.
    The right-hand side seed is 1000 + i unless ``seed`` is given.
    """
    if seed is None:
        seed = 1000 + i
    if i == 1:
        p = grid_laplacian((64, 64))
        nrhs = 1
    elif i == 2:
        p = grid_laplacian((100, 100, 100), shift=1e-3)
        nrhs = 1
    elif i == 3:
        p = convection_diffusion((80, 80, 80), seed)
        nrhs = 4
    elif i == 5:
        from .elasticity import elasticity3d
        p = elasticity3d(42, seed)
        nrhs = 8
    else:
        raise ValueError("unknown config %r" % (i,))
    p.b = rhs(p.n, nrhs, seed)
    p.name = CONFIG_NAMES[i]
    p.meta["config"] = i
    p.meta["seed"] = seed
    return p
