"""The allocation-free solve (spx_solve_noalloc) against spx_solve.

Both entry points are called through the C ABI on the same factorization
and the same right-hand sides; the allocation-free one works in the
library's fixed per-device array.  Two calls in a row, the second on a
smaller problem (the array keeps the first call's contents), then a call
larger than the array's limit, which must be refused on the host before any
device work.  Bar (FP64): omega <= 1e-14 for both, x within 1e-12 relative
of spx_solve's (the off-diagonal sweep steps add with atomics, so the two
may round differently) and within 1e-10 of the oracle's refined solution.
"""
import ctypes as C

import numpy as np
import pytest

from gen import grid_laplacian, make_config, rhs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


def _factor(torch, p):
    from paper_1405_2636_amd import Solver
    s = Solver(p.n, p.colptr, p.rowind)
    s.factorize(torch.tensor(p.values, device="cuda"))
    return s


def _abi_solve(torch, s, B, noalloc):
    """B: (nrhs, n) float64 CUDA tensor; returns (rc, x, solve info)."""
    from paper_1405_2636_amd import spx
    x = B.clone().contiguous()
    nrhs = x.shape[0]
    si = spx.SolveInfo()
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if noalloc:
        rc = s._lib.spx_solve_noalloc(s._h, nrhs, C.c_void_p(x.data_ptr()), s.n, C.byref(si), stream)
    else:
        rc = s._lib.spx_solve(s._h, nrhs, C.c_void_p(x.data_ptr()), s.n, 1, C.byref(si), stream)
    torch.cuda.synchronize()
    return rc, x, si


def _check(orc, torch, p, nrhs, seed):
    print("no-alloc case n=%d nrhs=%d seed=%d" % (p.n, nrhs, seed), flush=True)
    s = _factor(torch, p)
    b = rhs(p.n, nrhs, seed)                       # (n, nrhs)
    B = torch.tensor(np.ascontiguousarray(b.T), device="cuda")
    rc0, x0, si0 = _abi_solve(torch, s, B, noalloc=False)
    rc1, x1, si1 = _abi_solve(torch, s, B, noalloc=True)
    assert rc0 == 0 and rc1 == 0
    assert si0.omega <= 1e-14 and si1.omega <= 1e-14 and si1.converged == 1
    xa, xb = x0.cpu().numpy(), x1.cpu().numpy()
    assert np.max(np.abs(xb - xa)) <= 1e-12 * np.max(np.abs(xa))
    sym = orc.analyze(p.n, p.colptr, p.rowind)
    P = orc.factor(sym, p.colptr, p.rowind, p.values)
    xo, _ = orc.solve_refined(sym, P, p.colptr, p.rowind, p.values, b)
    assert np.max(np.abs(xb.T - xo)) <= 1e-10 * np.max(np.abs(xo))
    return s


def test_noalloc_matches_solve_two_calls(orc, torch):
    # first call: 24^3 Laplacian, 3 right-hand sides; second: the 64 x 64
    # 2-D Laplacian, 1 right-hand side (smaller), on the same fixed array
    _check(orc, torch, grid_laplacian((24, 24, 24), shift=1e-3), 3, 7)
    _check(orc, torch, make_config(1), 1, 8)


def test_noalloc_rejects_oversize(torch):
    from paper_1405_2636_amd import spx
    p = make_config(1)                               # n = 4096
    s = _factor(torch, p)
    nrhs = 300                                       # 7 * 4096 * 300 doubles > 64 MiB
    B = torch.zeros((nrhs, p.n), dtype=torch.float64, device="cuda")
    rc, x, si = _abi_solve(torch, s, B, noalloc=True)
    assert rc == spx.SPX_EINVAL
    assert b"work memory" in s._lib.spx_last_error(s._h)
    assert torch.count_nonzero(x).item() == 0        # nothing was written
    # the handle still solves afterwards
    _, info = s.solve_noalloc(torch.tensor(np.ascontiguousarray(p.b[:, 0]), device="cuda"))
    assert info["omega"] <= 1e-14
