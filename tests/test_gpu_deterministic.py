"""Deterministic accumulation mode (Section III: the runtimes serialize the
tasks that write one panel; here updates into a column block are applied in
ascending order of their source block).  Two factorizations of the same
values, on the same handle, on a second handle of the same pattern and with
the per-item trace on (which changes the timing of every item) must agree
bit for bit: factor, log |det| and the negative-pivot count.  The factor is
also checked against the oracle's within the any-order mode's tolerance
(1e-10 of the largest entry in FP64; 1e-4 and 1e-3 in the FP32 storage
and split-BF16 product modes, on well-conditioned inputs), and against the
any-order mode's factor.
Inputs: 3-D grid Laplacians (many sources per target, split supernodes
whose merged updates are single pairs), a quasi-definite L D L^T matrix and
convection-diffusion L U in the three precision modes."""
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


def _quasi_definite(n1, n2, seed):
    rng = np.random.default_rng(seed)
    H = sp.random(n1, n1, density=0.03, random_state=rng)
    H = H + H.T + sp.diags(np.full(n1, 8.0))
    C = sp.random(n2, n2, density=0.05, random_state=rng)
    C = C + C.T + sp.diags(np.full(n2, 8.0))
    B = sp.random(n2, n1, density=0.04, random_state=rng)
    A = sp.bmat([[H, B.T], [B, -C]]).tocsc()
    A.sort_indices()
    return Problem(A.shape[0], A.indptr.astype(np.int64), A.indices.astype(np.int32), A.data.copy())


def _factor(torch, p, **kw):
    from paper_1405_2636_amd import Solver
    s = Solver(p.n, p.colptr, p.rowind, **kw)
    s.factorize(torch.tensor(p.values, dtype=torch.float64, device="cuda"))
    inf = s.info()
    return s, s.factor_values().cpu().numpy().copy(), (inf["logdet"], inf["nneg"])


def _oracle(orc, p, method, **kw):
    sym = orc.analyze(p.n, p.colptr, p.rowind, leaf=kw.get("leaf_size", 64), amalg_pct=kw.get("amalg_pct", 12),
                      split_width=kw.get("split_width", 256))
    if method == "llt":
        return orc.factor(sym, p.colptr, p.rowind, p.values)
    if method == "ldlt":
        return orc.factor_ldlt(sym, p.colptr, p.rowind, p.values)
    return np.concatenate(orc.factor_lu(sym, p.colptr, p.rowind, p.values))


CASES = {
    "llt_grid": (lambda: grid_laplacian((24, 22, 20), shift=1e-3), dict(method="llt")),
    "llt_split": (lambda: grid_laplacian((16, 15, 14), shift=1e-3),
                  dict(method="llt", split_width=24, leaf_size=16)),
    "llt_fp32": (lambda: grid_laplacian((20, 20, 18), shift=0.5), dict(method="llt", precision="fp32_ir")),
    "ldlt_qd": (lambda: _quasi_definite(900, 400, 3), dict(method="ldlt", split_width=64)),
    "lu_cd": (lambda: convection_diffusion((18, 17, 16), seed=5), dict(method="lu")),
    "lu_fp32": (lambda: convection_diffusion((16, 15, 14), seed=6), dict(method="lu", precision="fp32_ir")),
    "lu_bf16": (lambda: convection_diffusion((16, 15, 14), seed=7), dict(method="lu", precision="bf16x3_ir")),
}


@pytest.mark.parametrize("case", list(CASES))
def test_deterministic_bitwise(orc, torch, case):
    gen, kw = CASES[case]
    p = gen()
    print("deterministic case %s n=%d opts=%s" % (case, p.n, kw), flush=True)
    s, F1, d1 = _factor(torch, p, deterministic=True, **kw)
    # the same handle again
    s.factorize(torch.tensor(p.values, dtype=torch.float64, device="cuda"))
    assert np.array_equal(s.factor_values().cpu().numpy(), F1)
    inf = s.info()
    assert (inf["logdet"], inf["nneg"]) == d1
    # a second handle, and one with the item trace on
    _, F2, d2 = _factor(torch, p, deterministic=True, **kw)
    assert np.array_equal(F2, F1) and d2 == d1
    _, F3, d3 = _factor(torch, p, deterministic=True, trace=True, **kw)
    assert np.array_equal(F3, F1) and d3 == d1
    # parity with the oracle and with the any-order mode
    ref = _oracle(orc, p, **kw)
    prec = kw.get("precision", "fp64")
    tol = {"fp64": 1e-10, "fp32_ir": 1e-4, "bf16x3_ir": 1e-3}[prec]
    scale = np.max(np.abs(ref))
    assert np.max(np.abs(F1.astype(np.float64) - ref)) <= tol * scale
    _, F4, _ = _factor(torch, p, **kw)
    assert np.max(np.abs(F1.astype(np.float64) - F4.astype(np.float64))) <= tol * scale
