"""Paired pieces in the triangular sweeps (the solve of Section III's
factorization): on levels of at most 16 blocks, consecutive pieces p, q of a
split supernode are one block of the sweeps, through the pair's inverse
[[D_p, 0], [-D_q L_qp D_p, D_q]] formed on the matrix cores after the
factorization; p's rows facing q are left out of its off-diagonal step.
Checked through an unrefined solve (no refinement step: every error of the
pair's inverse shows in x) against the oracle's solve, x within 1e-10 of its
largest entry in FP64 and 1e-4 in the FP32 modes (the FP32 factor's own
error), for one, three, eight and thirteen right-hand sides (the sweeps'
blocks of 1, 4 and 8, and two grid rows of 8 with a partial second one),
and through the level count: fewer levels than the unpaired
dependency levels, computed here from the oracle's update lists (for a
single chain of pieces; elsewhere pairs off the longest path leave the
count unchanged).
Inputs: dense SPD matrices (one supernode in 3 to 5 balanced pieces; with
split_width 160 the pieces are about 140 wide, so the pairs' widths are
not multiples of 16), a 3-D grid Laplacian (the separators' chains),
convection-diffusion L U (pairs of the L and of the U^T side) and
L D L^T of dense quasi-definite matrices (the pair's inverse
-Y_q L_qp D_p Y_p of the kept Y = D^{-1} L^{-1}, and the backward step's
scaling by the pivots of both pieces)."""
import numpy as np
import pytest
import scipy.sparse as sp

from gen import convection_diffusion, grid_laplacian
from gen.stencils import Problem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


def _dense_spd(n, seed):
    rng = np.random.default_rng(seed)
    M = rng.uniform(-1, 1, (n, n))
    A = M @ M.T / n + np.eye(n)
    Ac = sp.csc_matrix(A)
    return Problem(n, Ac.indptr.astype(np.int64), Ac.indices.astype(np.int32), Ac.data.copy())


def _quasi_definite(n1, n2, seed):
    """[[H, B^T], [B, -C]], H and C dense SPD: L D L^T without pivoting exists."""
    rng = np.random.default_rng(seed)
    M = rng.uniform(-1, 1, (n1, n1))
    N = rng.uniform(-1, 1, (n2, n2))
    H = M @ M.T / n1 + np.eye(n1)
    C = N @ N.T / n2 + np.eye(n2)
    B = rng.uniform(-0.5, 0.5, (n2, n1))
    A = sp.csc_matrix(np.block([[H, B.T], [B, -C]]))
    return Problem(A.shape[0], A.indptr.astype(np.int64), A.indices.astype(np.int32), A.data.copy())


def _unpaired_levels(sym):
    """Dependency levels of the column blocks: 1 + the deepest updating block."""
    nc = sym.stats["ncblk"]
    lvl = np.zeros(nc, np.int64)
    for k in range(nc):
        t = sym.utgt[sym.uptr[k]:sym.uptr[k + 1]]
        if len(t):
            lvl[t] = np.maximum(lvl[t], lvl[k] + 1)
    return int(lvl.max()) + 1


CASES = {
    "dense700": (lambda: _dense_spd(700, 1), dict()),
    "dense1100": (lambda: _dense_spd(1100, 2), dict()),
    "dense900_160": (lambda: _dense_spd(900, 3), dict(split_width=160)),
    "dense1100_fp32": (lambda: _dense_spd(1100, 4), dict(precision="fp32_ir")),
    "dense900_bf16": (lambda: _dense_spd(900, 5), dict(precision="bf16x3_ir", split_width=160)),
    "grid": (lambda: grid_laplacian((18, 17, 16), shift=1e-3), dict(split_width=64, leaf_size=32)),
    "lu_cd": (lambda: convection_diffusion((16, 15, 14), seed=5), dict(method="lu", split_width=64, leaf_size=32)),
    "lu_cd_fp32": (lambda: convection_diffusion((16, 15, 14), seed=6),
                   dict(method="lu", precision="fp32_ir", split_width=96)),
    "dense_ldlt": (lambda: _quasi_definite(600, 500, 7), dict(method="ldlt")),
    "dense_ldlt_160": (lambda: _quasi_definite(500, 400, 8), dict(method="ldlt", split_width=160)),
    "dense_ldlt_fp32": (lambda: _quasi_definite(600, 500, 9), dict(method="ldlt", precision="fp32_ir")),
}


@pytest.mark.parametrize("nrhs", [1, 3, 8, 13])
@pytest.mark.parametrize("case", list(CASES))
def test_paired_sweeps(orc, torch, case, nrhs):
    from paper_1405_2636_amd import Solver
    gen, kw = CASES[case]
    p = gen()
    method = kw.get("method", "llt")
    print("solve pairs case %s nrhs %d n=%d opts=%s" % (case, nrhs, p.n, kw), flush=True)
    s = Solver(p.n, p.colptr, p.rowind, ir_max_iter=0, **kw)
    s.factorize(torch.tensor(p.values, device="cuda"))
    inf = s.info()
    sym = orc.analyze(p.n, p.colptr, p.rowind, leaf=kw.get("leaf_size", 64), split_width=kw.get("split_width", 256))
    assert inf["solve_pairs"] > 0
    if case.startswith("dense"):   # one chain of pieces: every pair shortens it
        assert inf["solve_levels"] < _unpaired_levels(sym)
    else:                          # pairs off the longest path leave the count
        assert inf["solve_levels"] <= _unpaired_levels(sym)
    rng = np.random.default_rng(7 + nrhs)
    B = rng.uniform(-1, 1, (p.n, nrhs))
    x, _ = s.solve(torch.tensor(np.ascontiguousarray(B.T if nrhs > 1 else B[:, 0]), device="cuda"),
                   raise_on_noconv=False)
    xg = x.cpu().numpy()
    xg = xg.T if nrhs > 1 else xg[:, None]
    if method == "lu":
        PL, PU = orc.factor_lu(sym, p.colptr, p.rowind, p.values)
        xo = orc.solve_lu(sym, PL, PU, B)
    elif method == "ldlt":
        P = orc.factor_ldlt(sym, p.colptr, p.rowind, p.values)
        xo = orc.solve_ldlt(sym, P, B)
    else:
        P = orc.factor(sym, p.colptr, p.rowind, p.values)
        xo = orc.solve(sym, P, B)
    xo = xo.reshape(p.n, nrhs)
    tol = 1e-10 if kw.get("precision", "fp64") == "fp64" else 1e-4
    assert np.max(np.abs(xg - xo)) <= tol * np.max(np.abs(xo))
