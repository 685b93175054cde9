"""GPU parity of the L D L^T factorization (static pivoting, FP64) against
the oracle's L D L^T, on the same seeded inputs and the same panel layout
(unit L below the diagonal, d_j on it).  Tolerances as for L L^T:
  * elementwise max|F_gpu - F_oracle| <= 1e-10 * max|F_oracle| (different
    summation orders of the updates);
  * reconstruction ||P A P^T - L D L^T||_F / ||A||_F <= 1e-12;
  * log |det A| within 1e-12 relative and the negative-pivot count equal
    (the inertia, fixed by Sylvester's law);
  * the refined solve reaches omega <= 1e-14.
Inputs: SPD matrices (random, grid) and quasi-definite saddle-point
matrices [[H, B^T], [B, -C]] (H, C SPD), for which every symmetric ordering
has an L D L^T; sparse and dense, several split widths."""
import numpy as np
import pytest
import scipy.sparse as sp

from gen import grid_laplacian, random_spd
from gen.stencils import Problem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


def _quasi_definite(n1, n2, seed, dens1=0.05, dens2=0.08, densb=0.05):
    rng = np.random.default_rng(seed)
    p1 = random_spd(n1, dens1, seed)
    H = sp.csc_matrix((p1.values, p1.rowind, p1.colptr), shape=(n1, n1))
    p2 = random_spd(n2, dens2, seed + 1)
    Cm = sp.csc_matrix((p2.values, p2.rowind, p2.colptr), shape=(n2, n2))
    B = sp.random(n2, n1, density=densb, random_state=rng, format="csc") * 2.0
    K = sp.bmat([[H, B.T], [B, -Cm]], format="csc")
    K.sort_indices()
    return Problem(n1 + n2, K.indptr.astype(np.int64), K.indices.astype(np.int32), K.data.copy())


def _dense_quasi_definite(n1, n2, seed):
    rng = np.random.default_rng(seed)
    M1 = rng.uniform(-1, 1, (n1, n1))
    M2 = rng.uniform(-1, 1, (n2, n2))
    Bm = rng.uniform(-1, 1, (n2, n1))
    K = np.block([[M1 @ M1.T / n1 + np.eye(n1), Bm.T], [Bm, -(M2 @ M2.T / n2 + np.eye(n2))]])
    Kc = sp.csc_matrix(K)
    return Problem(n1 + n2, Kc.indptr.astype(np.int64), Kc.indices.astype(np.int32), Kc.data.copy())


def _check(orc, torch, p, nrhs=1, **kw):
    from paper_1405_2636_amd import Solver
    print("ldlt case n=%d nnz=%d opts=%s" % (p.n, p.nnz, kw), flush=True)
    s = Solver(p.n, p.colptr, p.rowind, method="ldlt", **kw)
    s.factorize(torch.tensor(p.values, dtype=torch.float64, device="cuda"))
    F = s.factor_values().cpu().numpy()
    sym = orc.analyze(p.n, p.colptr, p.rowind, leaf=kw.get("leaf_size", 64), amalg_pct=kw.get("amalg_pct", 12),
                      split_width=kw.get("split_width", 256))
    P = orc.factor_ldlt(sym, p.colptr, p.rowind, p.values)
    assert F.shape == P.shape
    assert np.max(np.abs(F - P)) <= 1e-10 * np.max(np.abs(P))
    # reconstruction from the GPU factor
    ri, ci, v = orc.unpack(sym, F)
    dg = ri == ci
    D = np.zeros(p.n)
    D[ri[dg]] = v[dg]
    Lu = sp.csc_matrix((v[~dg], (ri[~dg], ci[~dg])), shape=(p.n, p.n)) + sp.identity(p.n, format="csc")
    A = sp.csc_matrix((p.values, p.rowind, p.colptr), shape=(p.n, p.n))
    PA = A[sym.perm][:, sym.perm]
    assert sp.linalg.norm(PA - Lu @ sp.diags(D) @ Lu.T) / sp.linalg.norm(PA) <= 1e-12
    info = s.info()
    lad, nneg = orc.logabsdet_ldlt(sym, P)
    assert abs(info["logdet"] - lad) <= 1e-12 * max(1.0, abs(lad))
    assert info["nneg"] == nneg
    rng = np.random.default_rng(p.n)
    B = rng.uniform(-1, 1, (p.n, nrhs))
    b = torch.tensor(np.ascontiguousarray(B.T if nrhs > 1 else B[:, 0]), device="cuda")
    x, sinfo = s.solve(b.clone())
    assert sinfo["omega"] <= 1e-14 and sinfo["converged"]
    xo = orc.solve_ldlt(sym, P, B)
    xg = x.cpu().numpy()
    xg = xg.T if nrhs > 1 else xg[:, None]
    assert np.max(np.abs(xg - xo)) <= 1e-9 * np.max(np.abs(xo))
    return s, nneg


@pytest.mark.parametrize("case", ["spd_rand", "grid3", "grid3_split", "grid3_split_nomerge", "qd", "qd_split",
                                  "qd_split_merge2", "qd_wide"])
def test_ldlt_parity(orc, torch, case):
    if case == "spd_rand":
        _check(orc, torch, random_spd(400, 0.01, 4))
    elif case == "grid3":
        _check(orc, torch, grid_laplacian((12, 11, 10), shift=1e-3), nrhs=2)
    elif case == "grid3_split":   # many pieces; their updates merged in groups of 4 (the default)
        _check(orc, torch, grid_laplacian((12, 11, 10), shift=1e-3), split_width=7, leaf_size=16)
    elif case == "grid3_split_nomerge":
        _check(orc, torch, grid_laplacian((12, 11, 10), shift=1e-3), split_width=7, leaf_size=16, merge_split=1)
    elif case == "qd":
        _, nneg = _check(orc, torch, _quasi_definite(300, 150, 5))
        assert nneg == 150
    elif case == "qd_split":
        _, nneg = _check(orc, torch, _quasi_definite(500, 200, 6), split_width=33, amalg_pct=40)
        assert nneg == 200
    elif case == "qd_split_merge2":
        _, nneg = _check(orc, torch, _quasi_definite(500, 200, 6), split_width=16, merge_split=2)
        assert nneg == 200
    else:
        _, nneg = _check(orc, torch, _quasi_definite(800, 400, 7, 0.02, 0.02, 0.01))
        assert nneg == 400


@pytest.mark.parametrize("n1,n2,split", [(20, 11, 256), (150, 107, 256), (200, 150, 100)])
def test_ldlt_dense_parity(orc, torch, n1, n2, split):
    # one dense supernode (several 32-column steps, tiles factored ahead)
    # with n2 negative pivots
    _, nneg = _check(orc, torch, _dense_quasi_definite(n1, n2, n1 + n2), split_width=split)
    assert nneg == n2


def test_ldlt_zero_pivot(orc, torch):
    from paper_1405_2636_amd import NotPositiveDefinite, Solver
    colptr = np.array([0, 2, 4], np.int64)
    rowind = np.array([0, 1, 0, 1], np.int32)
    for vals in [np.array([0.0, 1.0, 1.0, 0.0]), np.array([1.0, 1.0, 1.0, 1.0])]:
        sym = orc.analyze(2, colptr, rowind)
        with pytest.raises(orc.ZeroPivot) as eo:
            orc.factor_ldlt(sym, colptr, rowind, vals)
        s = Solver(2, colptr, rowind, method="ldlt", static_pivot_eps=0)
        with pytest.raises(NotPositiveDefinite) as eg:
            s.factorize(torch.tensor(vals, device="cuda"))
        assert eg.value.col == eo.value.col_orig
    # the handle stays usable
    s.factorize(torch.tensor(np.array([2.0, 1.0, 1.0, -3.0]), device="cuda"))
    assert s.info()["nneg"] == 1


def test_ldlt_equals_scaled_llt(orc, torch):
    # on an SPD matrix the two GPU factors satisfy d_j = l_jj^2 and
    # L_ldl = L_llt diag(1/l_jj)
    from paper_1405_2636_amd import Solver
    p = grid_laplacian((10, 9, 8), shift=1e-3)
    v = torch.tensor(p.values, device="cuda")
    s1 = Solver(p.n, p.colptr, p.rowind)
    s1.factorize(v)
    s2 = Solver(p.n, p.colptr, p.rowind, method="ldlt")
    s2.factorize(v)
    sym = orc.analyze(p.n, p.colptr, p.rowind)
    ri, ci, vc = orc.unpack(sym, s1.factor_values().cpu().numpy())
    _, _, vl = orc.unpack(sym, s2.factor_values().cpu().numpy())
    dc = np.zeros(p.n)
    dc[ri[ri == ci]] = vc[ri == ci]
    expect = np.where(ri == ci, vc ** 2, vc / dc[ci])
    assert np.max(np.abs(vl - expect) / np.maximum(np.abs(expect), 1e-300)) <= 1e-11
    assert abs(s1.info()["logdet"] - s2.info()["logdet"]) <= 1e-12 * abs(s1.info()["logdet"])


def test_ldlt_batch(orc, torch):
    # independent quasi-definite systems in one graph-replayed, tuned launch:
    # each member's solution against the oracle's, inertia summed
    from paper_1405_2636_amd import Solver
    ps = [_quasi_definite(120 + 40 * q, 50 + 10 * q, 20 + q) for q in range(4)] + [_dense_quasi_definite(40, 25, 9)]
    s = Solver.batch([(p.n, p.colptr, p.rowind) for p in ps], method="ldlt", graph=True, tune=True)
    vals = torch.tensor(np.concatenate([p.values for p in ps]), device="cuda")
    rng = np.random.default_rng(3)
    B = [rng.uniform(-1, 1, p.n) for p in ps]
    for rep in range(2):   # tuning run, then a graph replay
        s.factorize(vals)
        x, si = s.solve(torch.tensor(np.concatenate(B), device="cuda"))
        assert si["omega"] <= 1e-14 and si["converged"]
        nneg = 0
        for p, xq, bq in zip(ps, s.split(x.cpu().numpy()), B):
            sym = orc.analyze(p.n, p.colptr, p.rowind)
            P = orc.factor_ldlt(sym, p.colptr, p.rowind, p.values)
            xo = orc.solve_ldlt(sym, P, bq[:, None])[:, 0]
            assert np.max(np.abs(xq - xo)) <= 1e-9 * np.max(np.abs(xo))
            nneg += orc.logabsdet_ldlt(sym, P)[1]
        assert s.info()["nneg"] == nneg


@pytest.mark.parametrize("case", ["grid3", "qd_split"])
def test_ldlt_parity_without_fused_small(orc, torch, case):
    # the FACT / TRSM / UPDATE path for the small blocks too (fused small
    # items are the default)
    if case == "grid3":
        _check(orc, torch, grid_laplacian((12, 11, 10), shift=1e-3), nrhs=2, fuse_small=False)
    else:
        _, nneg = _check(orc, torch, _quasi_definite(500, 200, 6), split_width=33, amalg_pct=40, fuse_small=False)
        assert nneg == 200


def _check_refined(orc, torch, p, precision, nrhs=1, **kw):
    """FP32-storage factors: the backward-error bound of L D L^T in precision
    u (2^-24; 2^-16 for the split-BF16 products hi*hi + hi*lo + lo*hi),
    ||P A P^T - L D L^T||_F <= gamma_{m+1} || |L| |D| |L|^T ||_F with m the
    largest column count (element growth of an indefinite factorization is
    inside |L| |D| |L|^T), the oracle's inertia, and the refined solve to
    omega <= 1e-14 and the oracle's x within 1e-9."""
    from paper_1405_2636_amd import Solver
    print("ldlt refined case n=%d nnz=%d prec=%s opts=%s" % (p.n, p.nnz, precision, kw), flush=True)
    s = Solver(p.n, p.colptr, p.rowind, method="ldlt", precision=precision, **kw)
    s.factorize(torch.tensor(p.values, dtype=torch.float64, device="cuda"))
    F = s.factor_values().cpu().numpy().astype(np.float64)
    sym = orc.analyze(p.n, p.colptr, p.rowind, leaf=kw.get("leaf_size", 64), amalg_pct=kw.get("amalg_pct", 12),
                      split_width=kw.get("split_width", 256))
    P = orc.factor_ldlt(sym, p.colptr, p.rowind, p.values)
    ri, ci, v = orc.unpack(sym, F)
    dg = ri == ci
    D = np.zeros(p.n)
    D[ri[dg]] = v[dg]
    Lu = sp.csc_matrix((v[~dg], (ri[~dg], ci[~dg])), shape=(p.n, p.n)) + sp.identity(p.n, format="csc")
    A = sp.csc_matrix((p.values, p.rowind, p.colptr), shape=(p.n, p.n))
    PA = A[sym.perm][:, sym.perm]
    u = 2.0 ** -24 if precision == "fp32_ir" else 2.0 ** -16
    m = int(np.max(np.diff(Lu.tocsc().indptr)))
    g = (m + 1) * u / (1 - (m + 1) * u)
    absL = abs(Lu)
    bound = g * sp.linalg.norm(absL @ sp.diags(np.abs(D)) @ absL.T)
    res = sp.linalg.norm(PA - Lu @ sp.diags(D) @ Lu.T)
    assert res <= bound, (res, bound)
    lad, nneg = orc.logabsdet_ldlt(sym, P)
    info = s.info()
    assert info["nneg"] == nneg
    assert abs(info["logdet"] - lad) <= 1e-4 * max(1.0, abs(lad))
    rng = np.random.default_rng(p.n + 1)
    B = rng.uniform(-1, 1, (p.n, nrhs))
    b = torch.tensor(np.ascontiguousarray(B.T if nrhs > 1 else B[:, 0]), device="cuda")
    x, sinfo = s.solve(b)
    assert sinfo["omega"] <= 1e-14 and sinfo["converged"], sinfo
    xo = orc.solve_ldlt(sym, P, B)
    xo = xo + orc.solve_ldlt(sym, P, B - (A @ xo))    # one FP64 refinement step of the oracle's solve
    xg = x.cpu().numpy()
    xg = xg.T if nrhs > 1 else xg[:, None]
    assert np.max(np.abs(xg - xo)) <= 1e-9 * np.max(np.abs(xo))
    return nneg


@pytest.mark.parametrize("precision", ["fp32_ir", "bf16x3_ir"])
@pytest.mark.parametrize("case", ["qd", "qd_split_merge", "grid3", "dense", "qd_nofuse"])
def test_ldlt_refinement_modes(orc, torch, precision, case):
    if case == "qd":
        assert _check_refined(orc, torch, _quasi_definite(300, 150, 5), precision, nrhs=3) == 150
    elif case == "qd_split_merge":
        assert _check_refined(orc, torch, _quasi_definite(500, 200, 6), precision, split_width=16,
                              merge_split=4) == 200
    elif case == "grid3":
        _check_refined(orc, torch, grid_laplacian((12, 11, 10), shift=1e-3), precision, nrhs=4)
    elif case == "dense":
        assert _check_refined(orc, torch, _dense_quasi_definite(150, 107, 11), precision, split_width=100) == 107
    else:
        assert _check_refined(orc, torch, _quasi_definite(400, 160, 8), precision, fuse_small=False) == 160
