"""The C ABI library: it loads, exports every function declared in
include/spx.h, and rejects bad input with the documented codes (host-only
calls; no compute call needs a GPU here)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    with open(os.path.join(ROOT, "include", "spx.h")) as f:
        src = f.read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(spx_[a-z_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    from paper_1405_2636_amd import spx
    lib = C.CDLL(spx.LIB_PATH)
    names = _declared()
    assert len(names) >= 10
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(spx.EXPORTED)


def test_strerror_and_codes():
    from paper_1405_2636_amd import spx
    L = spx.load_library()
    for code in [0, -1, -2, -3, -4, -5, -6]:
        assert L.spx_strerror(code)
    assert L.spx_strerror(-99) == b"unknown status"


@pytest.mark.parametrize("colptr,rowind,what", [
    ([0, 2, 3, 4], [1, 0, 1, 2], "unsorted"),
    ([0, 1, 2, 3], [0, 1, 5], "range"),
    ([0, 2, 3, 4], [0, 0, 1, 2], "duplicate"),
    ([1, 1, 2, 3], [0, 1, 2], "colptr"),
])
def test_analyze_rejects_bad_patterns(colptr, rowind, what):
    from paper_1405_2636_amd import Solver, SpxError
    with pytest.raises(SpxError) as ei:
        Solver(3, np.array(colptr), np.array(rowind))
    assert ei.value.code == -1


def test_bad_options():
    from paper_1405_2636_amd import Solver, SpxError
    from gen import grid_laplacian
    p = grid_laplacian((4, 4))
    with pytest.raises(SpxError):
        Solver(p.n, p.colptr, p.rowind, split_width=300)
    with pytest.raises(SpxError):
        Solver(p.n, p.colptr, p.rowind, user_perm=np.zeros(p.n, np.int32))
    for kw in [dict(merge_split=0), dict(merge_split=17), dict(tile=2), dict(static_pivot_eps=1.0),
               dict(static_pivot_eps=-0.5), dict(static_pivot_eps=float("nan"))]:
        with pytest.raises(SpxError):
            Solver(p.n, p.colptr, p.rowind, **kw)
    with pytest.raises(ValueError):
        Solver(p.n, p.colptr, p.rowind, precision="bf16")
    # every precision mode and option set in range is accepted at analysis
    for prec in ["fp64", "fp32_ir", "bf16x3_ir"]:
        Solver(p.n, p.colptr, p.rowind, precision=prec, merge_split=16, fuse_small=False, tile=1)
    # L D L^T and L U: every precision mode; an unknown method code is
    # rejected by the library
    for prec in ["fp64", "fp32_ir", "bf16x3_ir"]:
        Solver(p.n, p.colptr, p.rowind, method="ldlt", precision=prec, merge_split=16)
    for prec in ["fp64", "fp32_ir", "bf16x3_ir"]:
        Solver(p.n, p.colptr, p.rowind, method="lu", precision=prec)
    with pytest.raises(ValueError):
        Solver(p.n, p.colptr, p.rowind, method="qr")
    from paper_1405_2636_amd import spx
    L = spx.load_library()
    opt = spx.Options()
    L.spx_default_options(C.byref(opt))
    assert opt.method == 0 and opt.static_pivot_eps == -1.0
    Solver(p.n, p.colptr, p.rowind, method="lu", static_pivot_eps=0.0)
    Solver(p.n, p.colptr, p.rowind, method="ldlt", static_pivot_eps=1e-3)
    opt.method = 3
    h = C.c_void_p()
    assert L.spx_analyze(p.n, p.colptr.ctypes.data, p.rowind.ctypes.data, C.byref(opt), C.byref(h)) == -1


def test_null_safety():
    from paper_1405_2636_amd import spx
    L = spx.load_library()
    L.spx_destroy(None)
    assert L.spx_factorize(None, None, 0, None) == -1
    assert L.spx_get_info(None, None) == -1
    h = C.c_void_p()
    assert L.spx_analyze(-1, None, None, None, C.byref(h)) == -1


def test_empty_matrix():
    from paper_1405_2636_amd import Solver
    s = Solver(0, np.zeros(1, np.int64), np.zeros(0, np.int32))
    assert s.info()["ncblk"] == 0
