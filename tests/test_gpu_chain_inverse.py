"""Blocks of elimination chains (L L^T, width >= 128, alone in their
dependency level): FACT stores L_kk and the diagonal tiles of its inverse,
the panel solves are block substitutions with those tiles, and a separate
INV item forms the off-diagonal tiles of D = L_kk^{-1} (block forward
substitution) beside them.  Checked through what uses them: the panel
solves (the factor against the oracle's elementwise, 1e-10 of its largest
entry in FP64, 1e-5 in FP32) and the triangular sweeps, which use D (a
solve with no refinement step, x against the oracle's x within 1e-10 in
FP64; 1e-4 in FP32, whose unrefined solve carries the FP32 factor's
error).  The trace shows that INV items and substitution panel solves ran,
after their FACT.  Inputs: dense SPD matrices (one supernode in balanced pieces of at
most 256 or 160 columns, widths not multiples of 32) and a 3-D grid
Laplacian."""
import numpy as np
import pytest
import scipy.sparse as sp

from gen import grid_laplacian
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


@pytest.mark.parametrize("case,prec", [("dense700", "fp64"), ("dense700_160", "fp64"), ("dense600_fp32", "fp32_ir"),
                                       ("grid", "fp64")])
def test_chain_inverse(orc, torch, case, prec):
    from paper_1405_2636_amd import Solver
    kw = {}
    if case == "dense700":
        p = _dense_spd(700, 1)
    elif case == "dense700_160":
        p = _dense_spd(700, 2)
        kw = dict(split_width=160)   # balanced pieces of about 140 columns
    elif case == "dense600_fp32":
        p = _dense_spd(600, 3)
    else:
        p = grid_laplacian((16, 15, 14), shift=1e-3)
    print("chain inverse case %s prec %s n=%d" % (case, prec, p.n), flush=True)
    s = Solver(p.n, p.colptr, p.rowind, precision=prec, ir_max_iter=0, trace=True, **kw)
    s.factorize(torch.tensor(p.values, device="cuda"))
    t, k = s.trace()
    inv = np.where(k[:, 0] == 4)[0]
    assert len(inv) > 0
    for i in inv:   # the INV item and the block's panel solves after its FACT
        blk = k[i, 1]
        f = np.where((k[:, 0] == 0) & (k[:, 1] == blk))[0][0]
        assert t[i, 1] >= t[f, 2]
        tr = np.where((k[:, 0] == 1) & (k[:, 1] == blk))[0]
        if len(tr):
            assert t[tr, 1].min() >= t[f, 2]
    F = s.factor_values().cpu().numpy()
    sym = orc.analyze(p.n, p.colptr, p.rowind, split_width=kw.get("split_width", 256))
    P = orc.factor(sym, p.colptr, p.rowind, p.values)
    rng = np.random.default_rng(5)
    B = rng.uniform(-1, 1, (p.n, 2))
    x, info = s.solve(torch.tensor(np.ascontiguousarray(B.T), device="cuda"), raise_on_noconv=False)
    xo = orc.solve(sym, P, B)
    xg = x.cpu().numpy().T
    if prec == "fp64":
        assert np.max(np.abs(F - P)) <= 1e-10 * np.max(np.abs(P))
        assert np.max(np.abs(xg - xo)) <= 1e-10 * np.max(np.abs(xo))
    else:
        assert np.max(np.abs(F - P)) <= 1e-5 * np.max(np.abs(P))
        assert np.max(np.abs(xg - xo)) <= 1e-4 * np.max(np.abs(xo))
