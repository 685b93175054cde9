"""Pins of the oracle's symbolic analysis against brute force and hand-worked cases.

The symbolic factorization (Section III: elimination tree, predicted nonzero
pattern of the factor, grouping into blocks, amalgamation) is checked
against boolean Gaussian elimination on small patterns, which is the
definition of fill-in.
"""
import os

import numpy as np
import pytest

from gen import grid_laplacian, random_pattern

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    with open(os.path.join(GOLD, name)) as f:
        rows = [ln for ln in f if not ln.startswith("#") and ln.strip()]
    return np.array(rows[0].split(), dtype=np.int64)


def _dense_pattern(n, colptr, rowind):
    M = np.zeros((n, n), dtype=bool)
    for j in range(n):
        for p in range(colptr[j], colptr[j + 1]):
            M[rowind[p], j] = True
            M[j, rowind[p]] = True
    return M


def _brute_fill(M, perm):
    """Boolean Gaussian elimination of the permuted pattern; returns lower struct(L)."""
    n = M.shape[0]
    F = M[np.ix_(perm, perm)].copy()
    np.fill_diagonal(F, True)
    for k in range(n):
        nz = np.nonzero(F[k + 1:, k])[0] + k + 1
        if len(nz):
            F[np.ix_(nz, nz)] = True
    return np.tril(F)


def _cases():
    out = []
    for n, dens, seed in [(12, 0.2, 1), (25, 0.12, 2), (40, 0.08, 3), (40, 0.3, 4), (33, 0.05, 5)]:
        cp, ri = random_pattern(n, dens, seed)
        out.append(("rand%d_%d" % (n, seed), n, cp, ri))
    for dims in [(6, 5), (4, 3, 3), (7,)]:
        p = grid_laplacian(dims)
        out.append(("grid" + "x".join(map(str, dims)), p.n, p.colptr, p.rowind))
    return out


CASES = _cases()


def test_nd_golden_path(orc):
    p = grid_laplacian((7,))
    xadj, adj = orc.graph(p.n, p.colptr, p.rowind)
    assert list(orc.nd_order(p.n, xadj, adj, leaf=1)) == list(_golden("nd_path7.txt"))


def test_nd_golden_grid(orc):
    p = grid_laplacian((3, 3))
    xadj, adj = orc.graph(p.n, p.colptr, p.rowind)
    assert list(orc.nd_order(p.n, xadj, adj, leaf=1)) == list(_golden("nd_grid3x3.txt"))


def test_graph_is_symmetrized(orc):
    # pattern given as the lower triangle only must give the same graph as the full one
    p = grid_laplacian((5, 4))
    cols = np.repeat(np.arange(p.n), np.diff(p.colptr))
    keep = p.rowind >= cols
    cp = np.zeros(p.n + 1, np.int64)
    np.add.at(cp, cols[keep] + 1, 1)
    cp = np.cumsum(cp)
    x1, a1 = orc.graph(p.n, p.colptr, p.rowind)
    x2, a2 = orc.graph(p.n, cp, p.rowind[keep])
    assert np.array_equal(x1, x2) and np.array_equal(a1, a2)
    assert len(a1) == p.nnz - p.n


@pytest.mark.parametrize("name,n,cp,ri", CASES, ids=[c[0] for c in CASES])
def test_etree_counts_bruteforce(orc, name, n, cp, ri):
    M = _dense_pattern(n, cp, ri)
    xadj, adj = orc.graph(n, cp, ri)
    rng = np.random.default_rng(7)
    for perm in [np.arange(n), rng.permutation(n), orc.nd_order(n, xadj, adj, leaf=4)]:
        parent, eta = orc.etree_counts(n, xadj, adj, perm)
        Lp = _brute_fill(M, perm)
        assert np.array_equal(eta, Lp.sum(axis=0))
        for j in range(n):
            below = np.nonzero(Lp[j + 1:, j])[0]
            assert parent[j] == (below[0] + j + 1 if len(below) else -1)


def test_postorder_rules(orc):
    # forest: 5 -> 2, 0 -> 2, 3 -> 4, 1 root, 2 root, 4 root (parent array)
    parent = np.array([2, -1, -1, 4, -1, 2], np.int32)
    post = orc.postorder(parent)
    # roots ascending (1, 2, 4); children ascending (0 before 5); node after children
    assert list(post) == [1, 0, 5, 2, 3, 4]


@pytest.mark.parametrize("name,n,cp,ri", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("amalg", [0, 12, 50])
@pytest.mark.parametrize("split", [256, 3])
def test_block_structure_covers_fill(orc, name, n, cp, ri, amalg, split):
    s = orc.analyze(n, cp, ri, leaf=4, amalg_pct=amalg, split_width=split)
    perm = s.perm
    assert sorted(perm) == list(range(n))
    assert np.array_equal(s.iperm[perm], np.arange(n))
    M = _dense_pattern(n, cp, ri)
    Lp = _brute_fill(M, perm)
    # exact count of the factor's nonzeros does not depend on the equivalent reordering
    assert s.stats["nnz_exact"] == int(Lp.sum())
    # column elimination tree in the final numbering, by definition
    for j in range(n):
        below = np.nonzero(Lp[j + 1:, j])[0]
        assert s.etree[j] == (below[0] + j + 1 if len(below) else -1)
    # block structure: every cblk holds its dense lower diagonal block and whole row blocks
    B = np.zeros((n, n), dtype=bool)
    cnt = 0
    for k in range(s.stats["ncblk"]):
        f, l = s.fcol[k], s.lcol[k]
        w = l - f + 1
        assert 1 <= w <= split
        b0, b1 = s.bptr[k], s.bptr[k + 1]
        assert s.frow[b0] == f and s.lrow[b0] == l and s.fcblk[b0] == k and s.coefind[b0] == 0
        h = w
        prev_row = l
        for b in range(b0 + 1, b1):
            fr, lr, j = s.frow[b], s.lrow[b], s.fcblk[b]
            assert fr > prev_row and lr >= fr
            # the block lies inside the columns of its facing cblk
            assert s.fcol[j] <= fr and lr <= s.lcol[j] and j > k
            assert s.coefind[b] == h
            h += lr - fr + 1
            prev_row = lr
        assert s.stride[k] == h
        assert s.panel_off[k + 1] - s.panel_off[k] == h * w
        for c in range(f, l + 1):
            B[c:l + 1, c] = True
            for b in range(b0 + 1, b1):
                B[s.frow[b]:s.lrow[b] + 1, c] = True
        cnt += w * (w + 1) // 2 + w * (h - w)
    assert not np.any(Lp & ~B), "factor nonzero outside the block structure"
    assert cnt == s.stats["nnz_amalg"] == s.stats["nnz_exact"] + s.stats["zeros_used"]
    assert s.stats["zeros_used"] <= s.stats["budget"] == amalg * s.stats["nnz_exact"] // 100
    if amalg == 0:
        assert s.stats["zeros_used"] == 0 and not np.any(B & ~Lp)
    # maximal runs: two consecutive blocks of a cblk either have a row gap or face different cblks
    for k in range(s.stats["ncblk"]):
        for b in range(s.bptr[k] + 1, s.bptr[k + 1] - 1):
            assert s.lrow[b] + 1 < s.frow[b + 1] or s.fcblk[b] != s.fcblk[b + 1]
    # update pairs: distinct facing cblks in ascending order; dependency counts
    dep = np.zeros(s.stats["ncblk"], np.int64)
    for k in range(s.stats["ncblk"]):
        t = sorted(set(s.fcblk[s.bptr[k] + 1:s.bptr[k + 1]].tolist()))
        assert list(s.utgt[s.uptr[k]:s.uptr[k + 1]]) == t
        for j in t:
            dep[j] += 1
        assert s.cparent[k] == (t[0] if t else -1)
    assert np.array_equal(dep, s.dep)


def test_split_rule(orc):
    # a dense 10x10 pattern is a single supernode of width 10; split width 4 ->
    # ceil(10/4) = 3 parts, the first 10 % 3 = 1 one column wider: 4, 3, 3
    n = 10
    cp = np.arange(0, n * n + 1, n, dtype=np.int64)
    ri = np.tile(np.arange(n, dtype=np.int32), n)
    s = orc.analyze(n, cp, ri, split_width=4)
    assert list(s.lcol - s.fcol + 1) == [4, 3, 3]
    assert s.stats["nsn"] == 1


def test_flop_convention_dense(orc):
    # Sum of squared column counts = n^3/3 + n^2/2 + n/6 for a dense matrix
    for n in [1, 2, 7, 30]:
        cp = np.arange(0, n * n + 1, n, dtype=np.int64)
        ri = np.tile(np.arange(n, dtype=np.int32), n)
        s = orc.analyze(n, cp, ri)
        assert s.stats["flops_alg"] == n * (n + 1) * (2 * n + 1) // 6
        assert s.stats["flops_exec"] == s.stats["flops_alg"]
        # L U: sum over e = 1..n of 2 (e - 1)^2 + (e - 1) = (n - 1) n (2n - 1) / 3 + n (n - 1) / 2,
        # about 2 n^3 / 3
        assert s.stats["flops_alg_lu"] == (n - 1) * n * (2 * n - 1) // 3 + n * (n - 1) // 2
        assert s.stats["flops_exec_lu"] == s.stats["flops_alg_lu"]


def test_nd_reduces_fill_on_grid(orc):
    p = grid_laplacian((64, 64))
    s_nd = orc.analyze(p.n, p.colptr, p.rowind, amalg_pct=0)
    s_nat = orc.analyze(p.n, p.colptr, p.rowind, amalg_pct=0, user_perm=np.arange(p.n))
    # natural order fill is about n * 64; nested dissection is O(n log n) with a small constant
    assert s_nat.stats["nnz_exact"] > 2 * s_nd.stats["nnz_exact"]


def test_user_perm_identity_chain(orc):
    p = grid_laplacian((50,))
    s = orc.analyze(p.n, p.colptr, p.rowind, user_perm=np.arange(p.n))
    assert np.array_equal(s.perm, np.arange(p.n))


def test_invalid_patterns(orc):
    with pytest.raises(ValueError):
        orc.analyze(3, np.array([0, 2, 3, 4]), np.array([1, 0, 1, 2]))  # unsorted rows
    with pytest.raises(ValueError):
        orc.analyze(3, np.array([0, 1, 2, 3]), np.array([0, 1, 5]))  # out of range
