"""GPU parity of the L U factorization with static pivoting (method "lu")
against the oracle's L U, on the same seeded inputs and the same panel
layout (the L panels with the square diagonal blocks, then the U^T panels).
Tolerances (FP64):
  * elementwise max|F_gpu - F_oracle| <= 1e-10 * max|F_oracle| on both panel
    arrays (the two sum the updates of a target in different orders);
  * reconstruction ||P A P^T - L U||_F / ||A||_F <= 1e-12;
  * log |det A| within 1e-12 relative and the number of negative pivots
    equal;
  * the refined solve reaches omega <= 1e-14 and x matches the oracle's
    refined x within 1e-10 relative.
The FP32 and split-BF16 factors are checked through the refined solve
(omega <= 1e-14, x within 1e-9 of the oracle's) and their reconstruction
(1e-6 and 1e-5: units of FP32 rounding and of the split products' 2^-16).
Inputs: convection-diffusion stencils (2-D and 3-D), random unsymmetric
matrices with symmetric and with unsymmetric patterns, dense unsymmetric
matrices (wide diagonal blocks: several 32-column steps of the diagonal
factorization, split widths 256 and 64); update tile shapes and merged
updates of split pieces on and off."""
import numpy as np
import pytest
import scipy.sparse as sp

from gen import convection_diffusion, rhs
from gen.stencils import Problem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


def _from_dense(A):
    M = sp.csc_matrix(A)
    M.sort_indices()
    return Problem(M.shape[0], M.indptr.astype(np.int64), M.indices.astype(np.int32), M.data.copy())


def _unsym_random(n, seed, symmetric_pattern=True, density=0.02):
    rng = np.random.default_rng(seed)
    M = sp.random(n, n, density=density, random_state=rng, format="csc")
    if symmetric_pattern:
        M = M + M.T.multiply(rng.uniform(-1, 1))
    M = M.tocsc()
    A = M + sp.diags(np.abs(M).sum(axis=1).A1 + 1.0)
    A = A.tocsc()
    A.sort_indices()
    return Problem(n, A.indptr.astype(np.int64), A.indices.astype(np.int32), A.data.copy())


def _dense_unsym(n, seed):
    rng = np.random.default_rng(seed)
    A = rng.uniform(-1, 1, (n, n))
    A += np.diag(np.abs(A).sum(axis=1))
    return _from_dense(A)


def _dense_lu(sv, F, n):
    """Dense unit-lower L and upper U of P A P^T from the panels [L | U^T]."""
    pe = int(sv["panel_off"][-1])
    PL, PU = F[:pe], F[pe:2 * pe]
    L = np.eye(n)
    U = np.zeros((n, n))
    for k in range(sv["ncblk"]):
        f, l, ld, off = int(sv["fcol"][k]), int(sv["lcol"][k]), int(sv["stride"][k]), int(sv["panel_off"][k])
        wd = l - f + 1
        blk = PL[off:off + ld * wd].reshape(wd, ld).T
        ublk = PU[off:off + ld * wd].reshape(wd, ld).T
        sq = blk[:wd, :wd]
        L[f:f + wd, f:f + wd] += np.tril(sq, -1)
        U[f:f + wd, f:f + wd] = np.triu(sq)
        rows = []
        for b in range(int(sv["bptr"][k]) + 1, int(sv["bptr"][k + 1])):
            rows.extend(range(int(sv["frow"][b]), int(sv["lrow"][b]) + 1))
        if rows:
            rows = np.array(rows)
            L[rows, f:f + wd] = blk[wd:, :]
            U[f:f + wd, rows] = ublk[wd:, :].T
    return L, U


def _check(orc, torch, p, nrhs=2, precision="fp64", **kw):
    from paper_1405_2636_amd import Solver
    print("lu case n=%d nnz=%d prec=%s opts=%s" % (p.n, p.nnz, precision, kw), flush=True)
    s = Solver(p.n, p.colptr, p.rowind, method="lu", precision=precision, **kw)
    s.factorize(torch.tensor(p.values, dtype=torch.float64, device="cuda"))
    F = s.factor_values().cpu().numpy()
    sym = orc.analyze(p.n, p.colptr, p.rowind, leaf=kw.get("leaf_size", 64), amalg_pct=kw.get("amalg_pct", 12),
                      split_width=kw.get("split_width", 256))
    PL, PU = orc.factor_lu(sym, p.colptr, p.rowind, p.values)
    pe = len(PL)
    assert F.shape == (2 * pe,)
    sv = s.symbolic()
    L, U = _dense_lu(sv, F, p.n)
    A = sp.csc_matrix((p.values, p.rowind, p.colptr), shape=(p.n, p.n)).toarray()
    PA = A[np.ix_(sv["perm"], sv["perm"])]
    res = np.linalg.norm(PA - L @ U) / np.linalg.norm(PA)
    B = rhs(p.n, nrhs, 77)
    x, info = s.solve(torch.tensor(np.ascontiguousarray(B.T), device="cuda"))
    assert info["omega"] <= 1e-14 and info["converged"], info
    xo = orc.solve_lu(sym, PL, PU, B)
    Asp = sp.csc_matrix((p.values, p.rowind, p.colptr), shape=(p.n, p.n))
    xo = xo + orc.solve_lu(sym, PL, PU, B - Asp @ xo)     # one FP64 refinement step of the oracle's solve
    xg = x.cpu().numpy().T
    inf = s.info()
    lad, nneg = orc.logabsdet_lu(sym, PL)
    if precision == "fp64":
        assert np.max(np.abs(F[:pe] - PL)) <= 1e-10 * np.max(np.abs(PL))
        assert np.max(np.abs(F[pe:] - PU)) <= 1e-10 * max(np.max(np.abs(PU)), 1e-300)
        assert res <= 1e-12, res
        assert abs(inf["logdet"] - lad) <= 1e-12 * max(1.0, abs(lad))
        assert inf["nneg"] == nneg
        assert np.max(np.abs(xg - xo)) <= 1e-10 * np.max(np.abs(xo))
    else:
        assert res <= (1e-6 if precision == "fp32_ir" else 1e-5), res
        assert np.max(np.abs(xg - xo)) <= 1e-9 * np.max(np.abs(xo))
    return s


@pytest.mark.parametrize("case", ["cd3", "cd2", "rand_sym", "rand_unsym", "dense200", "dense600"])
def test_lu_parity_fp64(orc, torch, case):
    p = {"cd3": lambda: convection_diffusion((11, 10, 9), seed=3),
         "cd2": lambda: convection_diffusion((40, 33), seed=4),
         "rand_sym": lambda: _unsym_random(700, 5),
         "rand_unsym": lambda: _unsym_random(700, 6, symmetric_pattern=False),
         "dense200": lambda: _dense_unsym(200, 7),
         "dense600": lambda: _dense_unsym(600, 8)}[case]()
    _check(orc, torch, p)


@pytest.mark.parametrize("opts", [dict(split_width=64), dict(split_width=64, merge_split=1), dict(tile=1),
                                  dict(split_width=100, leaf_size=16)])
def test_lu_parity_options(orc, torch, opts):
    _check(orc, torch, convection_diffusion((13, 12, 11), seed=9), **opts)
    _check(orc, torch, _dense_unsym(520, 10), **opts)


@pytest.mark.parametrize("precision", ["fp32_ir", "bf16x3_ir"])
def test_lu_refinement_modes(orc, torch, precision):
    _check(orc, torch, convection_diffusion((12, 11, 10), seed=11), nrhs=4, precision=precision)
    _check(orc, torch, _dense_unsym(300, 12), nrhs=1, precision=precision)


def test_lu_zero_pivot(orc, torch):
    from paper_1405_2636_amd import Solver, NotPositiveDefinite
    colptr = np.array([0, 2, 4], np.int64)
    rowind = np.array([0, 1, 0, 1], np.int32)
    # [[1, 2], [3, 6]]: the second pivot is 6 - 3 * 2 = 0
    vals = np.array([1.0, 3.0, 2.0, 6.0])
    s = Solver(2, colptr, rowind, method="lu", static_pivot_eps=0)
    with pytest.raises(NotPositiveDefinite) as e:
        s.factorize(torch.tensor(vals, device="cuda"))
    sym = orc.analyze(2, colptr, rowind)
    with pytest.raises(orc.ZeroPivot) as eo:
        orc.factor_lu(sym, colptr, rowind, vals)
    assert e.value.col == eo.value.col_orig


def test_lu_values_grad_refused(torch):
    from paper_1405_2636_amd import Solver, SpxError
    p = convection_diffusion((5, 4, 3), seed=1)
    s = Solver(p.n, p.colptr, p.rowind, method="lu")
    s.factorize(torch.tensor(p.values, device="cuda"))
    x = torch.zeros(p.n, dtype=torch.float64, device="cuda")
    with pytest.raises(SpxError):
        s.values_grad(x, x)
