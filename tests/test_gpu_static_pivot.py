"""GPU static pivot replacement (Section III: static pivoting, no row or
column exchange) against the oracle's, for L D L^T and L U: a pivot p with
|p| < tau = eps * max |a_ij| becomes +-tau (+tau for p = 0) and is counted.

Inputs are planted-zero-pivot matrices (exact integers on a dense pattern
with the identity ordering), large enough that the planted pivots fall in
different 32-column steps of the diagonal-block factorization, in tiles
factored ahead of their step and in different pieces of a split supernode.
The kept pivots are powers of two and eps is chosen so that tau is one
too: the kept inverses of the diagonal blocks (which hold 1/tau) are then
exact dyadic numbers, every step is exact in FP64, and the GPU factor must
equal the oracle's bit for bit, with the same replaced count.  In the FP32
modes tau = 1/16 keeps the inverses' entries within FP32's significand; the
factor is compared within 1e-6 (FP32) and 1e-5 (split BF16, whose dropped
low-by-low products give 2^-16-relative terms) of the oracle's, and the
replaced pivots by magnitude (their sign follows a residue that is exactly
zero only in exact arithmetic)."""
import math

import numpy as np
import pytest

from planted import dense_problem, planted_ldlt, planted_lu, unpack

pytestmark = pytest.mark.gpu

ZEROS = (3, 31, 32, 70, 131, 200, 257)
N = 300


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


def _eps_for(amax, tau):
    """eps with eps * amax == tau exactly in FP64 (both sides form tau that way)."""
    eps = tau / amax
    for _ in range(4):
        if eps * amax == tau:
            return eps
        eps = np.nextafter(eps, np.inf if eps * amax < tau else -np.inf)
    raise AssertionError("no eps gives tau exactly")


def _solver(torch, p, method, precision="fp64", **kw):
    from paper_1405_2636_amd import Solver
    print("static pivot case n=%d method=%s prec=%s opts=%s" % (p.n, method, precision, kw), flush=True)
    s = Solver(p.n, p.colptr, p.rowind, method=method, precision=precision, user_perm=np.arange(p.n), **kw)
    s.factorize(torch.tensor(p.values, dtype=torch.float64, device="cuda"))
    return s


@pytest.mark.parametrize("split", [256, 64, 40])
def test_ldlt_planted_zero_pivots(orc, torch, split):
    A, _, _ = planted_ldlt(N, ZEROS, 21, pivots=(-1.0, 1.0, 2.0, -2.0))
    eps = _eps_for(np.max(np.abs(A)), 2.0 ** -20)
    p = dense_problem(A)
    s = _solver(torch, p, "ldlt", static_pivot_eps=eps, split_width=split)
    sym = orc.analyze(p.n, p.colptr, p.rowind, split_width=split, user_perm=np.arange(p.n))
    P, nrep = orc.factor_ldlt(sym, p.colptr, p.rowind, p.values, pivot_eps=eps, return_nrep=True)
    assert nrep == len(ZEROS)
    F = s.factor_values().cpu().numpy()
    assert np.array_equal(F, P)
    inf = s.info()
    assert inf["pivots_replaced"] == nrep
    lad, nneg = orc.logabsdet_ldlt(sym, P)
    assert inf["nneg"] == nneg
    assert abs(inf["logdet"] - lad) <= 1e-12 * max(1.0, abs(lad))
    # refactorizing the same handle counts afresh
    s.factorize(torch.tensor(p.values, dtype=torch.float64, device="cuda"))
    assert s.info()["pivots_replaced"] == nrep


@pytest.mark.parametrize("precision,split", [("fp64", 256), ("fp64", 64), ("fp32_ir", 256), ("fp32_ir", 64),
                                             ("bf16x3_ir", 100)])
def test_lu_planted_zero_pivots(orc, torch, precision, split):
    A, _, _ = planted_lu(N, ZEROS, 22, pivots=(-2.0, -1.0, 1.0, 2.0))
    tau = 2.0 ** -20 if precision == "fp64" else 2.0 ** -4
    eps = _eps_for(np.max(np.abs(A)), tau)
    p = dense_problem(A)
    s = _solver(torch, p, "lu", precision, static_pivot_eps=eps, split_width=split)
    sym = orc.analyze(p.n, p.colptr, p.rowind, split_width=split, user_perm=np.arange(p.n))
    PL, PU, nrep = orc.factor_lu(sym, p.colptr, p.rowind, p.values, pivot_eps=eps, return_nrep=True)
    assert nrep == len(ZEROS)
    F = s.factor_values().cpu().numpy().astype(np.float64)
    pe = len(PL)
    assert s.info()["pivots_replaced"] == nrep
    if precision == "fp64":
        assert np.array_equal(F[:pe], PL) and np.array_equal(F[pe:], PU)
        return
    tol = 1e-6 if precision == "fp32_ir" else 1e-5
    GL, RL = unpack(sym, F[:pe], N), unpack(sym, PL, N)
    GU, RU = unpack(sym, F[pe:], N), unpack(sym, PU, N)
    z = np.array(ZEROS)
    assert np.array_equal(np.abs(GL[z, z]), np.full(len(z), tau))
    GL[z, z] = RL[z, z]
    scale = max(np.max(np.abs(RL)), np.max(np.abs(RU)))
    assert np.max(np.abs(GL - RL)) <= tol * scale
    assert np.max(np.abs(GU - RU)) <= tol * scale


def test_default_eps_and_off(orc, torch):
    """Default eps: sqrt of the factor precision's unit roundoff; 0: off."""
    from paper_1405_2636_amd import NotPositiveDefinite, Solver
    cp = np.array([0, 2, 4], np.int64)
    ri = np.array([0, 1, 0, 1], np.int32)
    sym = orc.analyze(2, cp, ri)
    # [[1, 1], [1, 1]]: d_2 = 0 -> sqrt(2^-53) in FP64
    vals = np.array([1.0, 1.0, 1.0, 1.0])
    s = Solver(2, cp, ri, method="ldlt")
    s.factorize(torch.tensor(vals, device="cuda"))
    P, nrep = orc.factor_ldlt(sym, cp, ri, vals, pivot_eps=math.sqrt(2.0 ** -53), return_nrep=True)
    assert np.array_equal(s.factor_values().cpu().numpy(), P) and s.info()["pivots_replaced"] == nrep == 1
    s0 = Solver(2, cp, ri, method="ldlt", static_pivot_eps=0)
    with pytest.raises(NotPositiveDefinite):
        s0.factorize(torch.tensor(vals, device="cuda"))
    # [[1, 2], [3, 6]]: u_22 = 0 -> 6 * 2^-12 in the FP32 modes
    vals = np.array([1.0, 3.0, 2.0, 6.0])
    for prec, eps in [("fp64", math.sqrt(2.0 ** -53)), ("fp32_ir", 2.0 ** -12), ("bf16x3_ir", 2.0 ** -12)]:
        s = Solver(2, cp, ri, method="lu", precision=prec)
        s.factorize(torch.tensor(vals, device="cuda"))
        PL, PU, nrep = orc.factor_lu(sym, cp, ri, vals, pivot_eps=eps, return_nrep=True)
        F = s.factor_values().cpu().numpy()
        assert np.array_equal(F, np.concatenate([PL, PU]).astype(F.dtype)), (prec, F)
        assert s.info()["pivots_replaced"] == nrep == 1
        s0 = Solver(2, cp, ri, method="lu", precision=prec, static_pivot_eps=0)
        with pytest.raises(NotPositiveDefinite):
            s0.factorize(torch.tensor(vals, device="cuda"))
