"""The library's symbolic analysis against the oracle's, bit for bit.

Both implement the same reading of Section III (nested dissection,
elimination tree, supernodes, amalgamation, splitting, blocking) with
different algorithms and no shared code; every exported array must agree.
Host-only: no GPU needed.
"""
import numpy as np
import pytest

from gen import grid_laplacian, make_config, random_pattern

ARRAYS = ["perm", "iperm", "etree", "snptr", "fcol", "lcol", "stride", "panel_off", "bptr", "cparent",
          "frow", "lrow", "fcblk", "coefind", "uptr", "utgt", "dep"]


def _compare(orc, n, cp, ri, **kw):
    from paper_1405_2636_amd import Solver
    s = Solver(n, cp, ri, **kw)
    sy = s.symbolic()
    o = orc.analyze(n, cp, ri, leaf=kw.get("leaf_size", 64), amalg_pct=kw.get("amalg_pct", 12),
                    split_width=kw.get("split_width", 256), user_perm=kw.get("user_perm"))
    for name in ARRAYS:
        assert np.array_equal(sy[name], o.arrays[name]), name
    info = s.info()
    assert info["nnz_l"] == o.stats["nnz_exact"]
    assert info["nnz_l_stored"] == o.stats["nnz_amalg"]
    assert info["flops_alg"] == o.stats["flops_alg"]
    assert info["flops_exec"] == o.stats["flops_exec"]
    assert info["panel_entries"] == o.stats["panel_size"]
    lu = Solver(n, cp, ri, method="lu", **kw).info()
    assert lu["flops_alg"] == o.stats["flops_alg_lu"] and lu["flops_exec"] == o.stats["flops_exec_lu"]
    return sy


@pytest.mark.parametrize("n,dens,seed", [(1, 0.0, 1), (2, 1.0, 2), (40, 0.1, 3), (500, 0.01, 4), (2000, 0.002, 5),
                                         (300, 0.05, 6), (1000, 0.0005, 7)])
@pytest.mark.parametrize("opts", [{}, {"leaf_size": 8, "amalg_pct": 30, "split_width": 5},
                                  {"leaf_size": 1, "amalg_pct": 0, "split_width": 1}])
def test_random_patterns(orc, n, dens, seed, opts):
    cp, ri = random_pattern(n, dens, seed)
    _compare(orc, n, cp, ri, **opts)


@pytest.mark.parametrize("dims", [(64, 64), (20, 20, 20), (7, 1, 9), (300,)])
def test_grids(orc, dims):
    p = grid_laplacian(dims)
    _compare(orc, p.n, p.colptr, p.rowind)


def test_user_permutation(orc):
    p = grid_laplacian((12, 11))
    perm = np.random.default_rng(3).permutation(p.n).astype(np.int32)
    _compare(orc, p.n, p.colptr, p.rowind, user_perm=perm)


def test_lower_triangle_pattern(orc):
    p = grid_laplacian((9, 8, 7))
    cols = np.repeat(np.arange(p.n), np.diff(p.colptr))
    keep = p.rowind >= cols
    cp = np.concatenate([[0], np.cumsum(np.bincount(cols[keep], minlength=p.n))]).astype(np.int64)
    a = _compare(orc, p.n, cp, p.rowind[keep])
    from paper_1405_2636_amd import Solver
    b = Solver(p.n, p.colptr, p.rowind).symbolic()
    assert all(np.array_equal(a[k], b[k]) for k in ARRAYS)


@pytest.mark.slow
def test_config2_full_size(orc):
    """The 100^3 7-point Laplacian of the benchmark: identical plans."""
    p = make_config(2)
    sy = _compare(orc, p.n, p.colptr, p.rowind)
    assert sy["ncblk"] > 1000


@pytest.mark.parametrize("config", [3, 5])
def test_other_workloads_full_size(orc, config):
    """The 80^3 convection-diffusion pattern (L U workload) and the 40^3
    Q1 elasticity pattern (L D L^T workload, 192,000 unknowns): identical
    plans."""
    p = make_config(config)
    sy = _compare(orc, p.n, p.colptr, p.rowind)
    assert sy["ncblk"] > 500


def _block_diagonal(problems):
    import scipy.sparse as sp
    mats = [sp.csc_matrix((p.values, p.rowind, p.colptr), shape=(p.n, p.n)) for p in problems]
    A = sp.block_diag(mats, format="csc")
    A.sort_indices()
    return A.shape[0], A.indptr.astype(np.int64), A.indices.astype(np.int32), A.data


def test_batch_analysis_is_block_diagonal_analysis(orc):
    # spx_analyze_batch: the systems' patterns placed on the diagonal, analysed
    # as one system; bit-exact against the oracle's analysis of that pattern
    from gen import grid_batch
    from paper_1405_2636_amd import Solver
    ps = grid_batch(12, seed=7, lo=5, hi=30)
    n, cp, ri, _ = _block_diagonal(ps)
    s = Solver.batch([(p.n, p.colptr, p.rowind) for p in ps], graph=False, tune=False)
    assert s.n == n and s.nnz == cp[-1] and s.info()["nsys"] == 12
    sy = s.symbolic()
    o = orc.analyze(n, cp, ri)
    for name in ARRAYS:
        assert np.array_equal(sy[name], o.arrays[name]), name
    # each system is a separate tree of the elimination forest
    roots = np.sum(sy["etree"] < 0)
    assert roots >= 12


@pytest.mark.parametrize("n", [5, 12])
def test_elasticity_patterns(orc, n):
    # 27-point, 3-dof coupling (dense 3x3 node blocks): supernodes follow
    # the node blocks
    from gen import elasticity3d
    p = elasticity3d(n, seed=1)
    _compare(orc, p.n, p.colptr, p.rowind)
    _compare(orc, p.n, p.colptr, p.rowind, leaf_size=8, amalg_pct=30, split_width=33)


def test_convection_diffusion_pattern(orc):
    # unsymmetric values on a symmetric pattern: the analysis reads the pattern only
    from gen import convection_diffusion
    p = convection_diffusion((14, 13, 12), seed=5)
    _compare(orc, p.n, p.colptr, p.rowind)
