"""Python driver of the oracle (plain serial FP64 CPU supernodal LL^T).

TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the
benchmark's CPU-baseline leg.  The product path never imports it.

The C source ``orc.c`` next to this file is compiled with gcc into
``liborc.so`` (``build()``), then loaded with ctypes.  Arrays cross the
boundary as numpy buffers.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "orc.c")
LIB = os.path.join(HERE, "liborc.so")

ENOTPD = -5

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, no BLAS, serial)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        build(force=True)
    L = C.CDLL(LIB)
    vp = C.c_void_p
    i32, i64, dbl = C.c_int32, C.c_int64, C.c_double
    L.orc_graph.restype = i64
    L.orc_graph.argtypes = [i32, vp, vp, vp, vp]
    L.orc_nd.restype = C.c_int
    L.orc_nd.argtypes = [i32, vp, vp, i32, vp]
    L.orc_etree_counts.restype = C.c_int
    L.orc_etree_counts.argtypes = [i32, vp, vp, vp, vp, vp]
    L.orc_postorder.restype = C.c_int
    L.orc_postorder.argtypes = [i32, vp, vp]
    L.orc_analyze.restype = C.c_int
    L.orc_analyze.argtypes = [i32, vp, vp, i32, i32, i32, vp, C.POINTER(vp)]
    L.orc_free.restype = None
    L.orc_free.argtypes = [vp]
    L.orc_sym_int.restype = i32
    L.orc_sym_int.argtypes = [vp, C.c_int]
    L.orc_sym_i64.restype = i64
    L.orc_sym_i64.argtypes = [vp, C.c_int]
    L.orc_sym_dbl.restype = dbl
    L.orc_sym_dbl.argtypes = [vp, C.c_int]
    L.orc_sym_copy.restype = C.c_int
    L.orc_sym_copy.argtypes = [vp, C.c_int, vp]
    L.orc_assemble.restype = C.c_int
    L.orc_assemble.argtypes = [vp, vp, vp, vp, vp]
    L.orc_factor.restype = C.c_int
    L.orc_factor.argtypes = [vp, vp, C.POINTER(i32)]
    L.orc_factor_upto.restype = C.c_int
    L.orc_factor_upto.argtypes = [vp, vp, i32, C.POINTER(i32)]
    L.orc_factor_range.restype = C.c_int
    L.orc_factor_range.argtypes = [vp, vp, i32, i32, C.POINTER(i32)]
    L.orc_values_grad.restype = None
    L.orc_values_grad.argtypes = [i32, vp, vp, i32, vp, vp, i64, vp]
    L.orc_assemble_range.restype = C.c_int
    L.orc_assemble_range.argtypes = [vp, vp, vp, vp, vp, i32, i32]
    L.orc_solve.restype = C.c_int
    L.orc_solve.argtypes = [vp, vp, i32, vp, i64, vp, i64]
    L.orc_residual.restype = None
    L.orc_residual.argtypes = [i32, vp, vp, vp, vp, vp, vp, vp]
    L.orc_omega.restype = dbl
    L.orc_omega.argtypes = [i32, vp, vp]
    L.orc_logdet.restype = dbl
    L.orc_logdet.argtypes = [vp, vp]
    L.orc_unpack.restype = i64
    L.orc_unpack.argtypes = [vp, vp, vp, vp, vp]
    L.orc_factor_ldlt.restype = C.c_int
    L.orc_factor_ldlt.argtypes = [vp, vp, C.POINTER(i32)]
    L.orc_factor_ldlt_sp.restype = C.c_int
    L.orc_factor_ldlt_sp.argtypes = [vp, vp, dbl, C.POINTER(i32), C.POINTER(i32)]
    L.orc_factor_lu_sp.restype = C.c_int
    L.orc_factor_lu_sp.argtypes = [vp, vp, vp, dbl, C.POINTER(i32), C.POINTER(i32)]
    L.orc_solve_ldlt.restype = C.c_int
    L.orc_solve_ldlt.argtypes = [vp, vp, i32, vp, i64, vp, i64]
    L.orc_logabsdet_ldlt.restype = dbl
    L.orc_logabsdet_ldlt.argtypes = [vp, vp, C.POINTER(i32)]
    L.orc_assemble_lu.restype = C.c_int
    L.orc_assemble_lu.argtypes = [vp, vp, vp, vp, vp, vp]
    L.orc_factor_lu.restype = C.c_int
    L.orc_factor_lu.argtypes = [vp, vp, vp, C.POINTER(i32)]
    L.orc_solve_lu.restype = C.c_int
    L.orc_solve_lu.argtypes = [vp, vp, vp, i32, vp, i64, vp, i64]
    L.orc_logabsdet_lu.restype = dbl
    L.orc_logabsdet_lu.argtypes = [vp, vp, C.POINTER(i32)]
    _lib = L
    return L


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


# ---------------------------------------------------------------- steps
def graph(n, colptr, rowind):
    """O1: adjacency of A + A^T without the diagonal (sorted, unique)."""
    L = _load()
    colptr = _c(colptr, np.int64)
    rowind = _c(rowind, np.int32)
    xadj = np.zeros(n + 1, np.int64)
    adj = np.zeros(2 * int(colptr[-1]) + 1, np.int32)
    m = L.orc_graph(n, _p(colptr), _p(rowind), _p(xadj), _p(adj))
    if m < 0:
        raise ValueError("bad pattern")
    return xadj, adj[:m].copy()


def nd_order(n, xadj, adj, leaf=64):
    """O2: nested-dissection order (new -> old)."""
    L = _load()
    xadj = _c(xadj, np.int64)
    adj = _c(adj, np.int32)
    order = np.zeros(n, np.int32)
    rc = L.orc_nd(n, _p(xadj), _p(adj), leaf, _p(order))
    if rc != 0:
        raise RuntimeError("orc_nd failed %d" % rc)
    return order


def etree_counts(n, xadj, adj, perm):
    """O3/O4: elimination tree and column counts (diagonal included) of P A P^T."""
    L = _load()
    xadj = _c(xadj, np.int64)
    adj = _c(adj, np.int32)
    perm = _c(perm, np.int32)
    parent = np.zeros(n, np.int32)
    eta = np.zeros(n, np.int64)
    rc = L.orc_etree_counts(n, _p(xadj), _p(adj), _p(perm), _p(parent), _p(eta))
    if rc != 0:
        raise RuntimeError("orc_etree_counts failed")
    return parent, eta


def postorder(parent):
    L = _load()
    parent = _c(parent, np.int32)
    post = np.zeros(len(parent), np.int32)
    rc = L.orc_postorder(len(parent), _p(parent), _p(post))
    if rc != 0:
        raise RuntimeError("orc_postorder failed")
    return post


# ---------------------------------------------------------------- analysis
_ARRAYS = [
    ("perm", np.int32, "n"), ("iperm", np.int32, "n"), ("etree", np.int32, "n"),
    ("snptr", np.int32, "nsn+1"), ("fcol", np.int32, "ncblk"), ("lcol", np.int32, "ncblk"),
    ("stride", np.int32, "ncblk"), ("panel_off", np.int64, "ncblk+1"), ("bptr", np.int32, "ncblk+1"),
    ("cparent", np.int32, "ncblk"), ("frow", np.int32, "nblok"), ("lrow", np.int32, "nblok"),
    ("fcblk", np.int32, "nblok"), ("coefind", np.int32, "nblok"), ("uptr", np.int32, "ncblk+1"),
    ("utgt", np.int32, "nupd"), ("dep", np.int32, "ncblk"), ("colcount", np.int64, "n"),
]


@dataclass
class Symbolic:
    handle: int
    n: int
    arrays: dict
    stats: dict

    def __getattr__(self, name):
        arrays = self.__dict__.get("arrays", {})
        if name in arrays:
            return arrays[name]
        raise AttributeError(name)

    def __del__(self):
        try:
            if self.handle and _lib is not None:
                _lib.orc_free(C.c_void_p(self.handle))
                self.handle = 0
        except Exception:
            pass


def analyze(n, colptr, rowind, leaf=64, amalg_pct=12, split_width=256, user_perm=None) -> Symbolic:
    L = _load()
    colptr = _c(colptr, np.int64)
    rowind = _c(rowind, np.int32)
    up = None if user_perm is None else _c(user_perm, np.int32)
    h = C.c_void_p()
    rc = L.orc_analyze(n, _p(colptr), _p(rowind), leaf, amalg_pct, split_width,
                       None if up is None else _p(up), C.byref(h))
    if rc != 0:
        raise ValueError("orc_analyze failed: %d" % rc)
    sizes = {"n": L.orc_sym_int(h, 0), "ncblk": L.orc_sym_int(h, 1), "nblok": L.orc_sym_int(h, 2),
             "nsn": L.orc_sym_int(h, 3), "nupd": L.orc_sym_int(h, 5)}
    arrays = {}
    for idx, (name, dt, sz) in enumerate(_ARRAYS):
        cnt = sizes[sz.split("+")[0]] + (1 if sz.endswith("+1") else 0)
        a = np.zeros(max(cnt, 1), dt)
        L.orc_sym_copy(h, idx, _p(a))
        arrays[name] = a[:cnt]
    stats = dict(sizes)
    stats.update({
        "nsn_fund": L.orc_sym_int(h, 4),
        "nnz_exact": L.orc_sym_i64(h, 0), "nnz_amalg": L.orc_sym_i64(h, 1),
        "zeros_used": L.orc_sym_i64(h, 2), "budget": L.orc_sym_i64(h, 3),
        "panel_size": L.orc_sym_i64(h, 4),
        "flops_alg": L.orc_sym_dbl(h, 0), "flops_exec": L.orc_sym_dbl(h, 1),
        "flops_alg_lu": L.orc_sym_dbl(h, 2), "flops_exec_lu": L.orc_sym_dbl(h, 3),
    })
    return Symbolic(h.value, n, arrays, stats)


# ---------------------------------------------------------------- numeric
class NotPositiveDefinite(RuntimeError):
    def __init__(self, col_new, col_orig):
        super().__init__("pivot not positive at column %d (original %d)" % (col_new, col_orig))
        self.col_new = col_new
        self.col_orig = col_orig


def assemble(sym: Symbolic, colptr, rowind, values):
    L = _load()
    P = np.zeros(max(int(sym.stats["panel_size"]), 1), np.float64)
    rc = L.orc_assemble(C.c_void_p(sym.handle), _p(_c(colptr, np.int64)), _p(_c(rowind, np.int32)),
                        _p(_c(values, np.float64)), _p(P))
    if rc != 0:
        raise ValueError("assemble failed")
    return P


def factor(sym: Symbolic, colptr, rowind, values):
    """Assemble and factor; returns the panel array (same layout as the library's)."""
    L = _load()
    P = assemble(sym, colptr, rowind, values)
    fc = C.c_int32(-1)
    rc = L.orc_factor(C.c_void_p(sym.handle), _p(P), C.byref(fc))
    if rc == ENOTPD:
        raise NotPositiveDefinite(fc.value, int(sym.perm[fc.value]))
    if rc != 0:
        raise RuntimeError("orc_factor failed %d" % rc)
    return P


def factor_upto(sym: Symbolic, colptr, rowind, values, kend):
    """Assemble, then process column blocks 0..kend-1 only; those panels hold
    their final values afterwards (each block is updated by smaller ones)."""
    L = _load()
    P = assemble(sym, colptr, rowind, values)
    fc = C.c_int32(-1)
    rc = L.orc_factor_upto(C.c_void_p(sym.handle), _p(P), int(kend), C.byref(fc))
    if rc == ENOTPD:
        raise NotPositiveDefinite(fc.value, int(sym.perm[fc.value]))
    if rc != 0:
        raise RuntimeError("orc_factor_upto failed %d" % rc)
    return P


def subtree_first(sym: Symbolic):
    """First column block of the subtree rooted at every block of the block
    elimination tree (blocks are numbered in postorder, so the subtree of r is
    the range first[r] .. r)."""
    nc = int(sym.stats["ncblk"])
    first = np.arange(nc, dtype=np.int64)
    par = sym.cparent
    for k in range(nc):
        p = int(par[k])
        if p >= 0 and first[k] < first[p]:
            first[p] = first[k]
    return first


def factor_subtree(sym: Symbolic, colptr, rowind, values, root):
    """Assemble and factor the subtree of block ``root`` only (its updates into
    the blocks above it included).  Returns (P, assembly seconds,
    factorization seconds); the subtree's panels hold their final values."""
    import time
    L = _load()
    k0 = int(subtree_first(sym)[root])
    k1 = int(root) + 1
    P = np.zeros(max(int(sym.stats["panel_size"]), 1), np.float64)
    t0 = time.perf_counter()
    rc = L.orc_assemble_range(C.c_void_p(sym.handle), _p(_c(colptr, np.int64)), _p(_c(rowind, np.int32)),
                              _p(_c(values, np.float64)), _p(P), k0, k1)
    t1 = time.perf_counter()
    if rc != 0:
        raise ValueError("assemble_range failed")
    fc = C.c_int32(-1)
    rc = L.orc_factor_range(C.c_void_p(sym.handle), _p(P), k0, k1, C.byref(fc))
    t2 = time.perf_counter()
    if rc == ENOTPD:
        raise NotPositiveDefinite(fc.value, int(sym.perm[fc.value]))
    if rc != 0:
        raise RuntimeError("orc_factor_range failed %d" % rc)
    return P, t1 - t0, t2 - t1


class ZeroPivot(RuntimeError):
    def __init__(self, col_new, col_orig):
        super().__init__("zero or non-finite pivot at column %d (original %d)" % (col_new, col_orig))
        self.col_new = col_new
        self.col_orig = col_orig


def static_pivot_tau(colptr, rowind, values, eps, lower_only):
    """tau = eps * max |a_ij| over the entries the factorization reads (the
    lower triangle for L D L^T, all entries for L U)."""
    colptr = np.asarray(colptr, np.int64)
    rowind = np.asarray(rowind, np.int64)
    v = np.abs(np.asarray(values, np.float64))
    if lower_only:
        col = np.repeat(np.arange(len(colptr) - 1), np.diff(colptr))
        v = v[rowind >= col]
    return float(eps) * (float(v.max()) if v.size else 0.0)


def factor_ldlt(sym: Symbolic, colptr, rowind, values, pivot_eps=0.0, return_nrep=False):
    """Assemble and factor as L D L^T (static pivoting: the analysis' order);
    returns the panel array: D on the diagonal of each diagonal block, the
    strictly lower entries of the unit lower L elsewhere.  pivot_eps > 0:
    pivots below pivot_eps * max |a_ij| in magnitude are replaced (with
    return_nrep, (P, number replaced) is returned)."""
    L = _load()
    P = assemble(sym, colptr, rowind, values)
    fc = C.c_int32(-1)
    nrep = C.c_int32(0)
    tau = static_pivot_tau(colptr, rowind, values, pivot_eps, True) if pivot_eps > 0 else 0.0
    rc = L.orc_factor_ldlt_sp(C.c_void_p(sym.handle), _p(P), tau, C.byref(nrep), C.byref(fc))
    if rc == ENOTPD:
        raise ZeroPivot(fc.value, int(sym.perm[fc.value]))
    if rc != 0:
        raise RuntimeError("orc_factor_ldlt failed %d" % rc)
    return (P, nrep.value) if return_nrep else P


def solve_ldlt(sym: Symbolic, P, b):
    L = _load()
    b = np.asfortranarray(np.asarray(b, np.float64).reshape(sym.n, -1))
    x = np.zeros_like(b, order="F")
    L.orc_solve_ldlt(C.c_void_p(sym.handle), _p(P), b.shape[1], _p(b), sym.n, _p(x), sym.n)
    return x


def logabsdet_ldlt(sym: Symbolic, P):
    """(log |det A|, number of negative pivots) of an L D L^T factor."""
    L = _load()
    nneg = C.c_int32(0)
    v = L.orc_logabsdet_ldlt(C.c_void_p(sym.handle), _p(P), C.byref(nneg))
    return v, nneg.value


def factor_lu(sym: Symbolic, colptr, rowind, values, pivot_eps=0.0, return_nrep=False):
    """Assemble both triangles and factor as L U (static pivoting: the
    analysis' order on the pattern of A + A^T); returns (PL, PU): PL holds
    the diagonal blocks' L (strictly lower) and U (upper) and L below them,
    PU holds U^T below the diagonal blocks.  pivot_eps > 0: pivots below
    pivot_eps * max |a_ij| in magnitude are replaced (with return_nrep,
    (PL, PU, number replaced) is returned)."""
    L = _load()
    PL = np.zeros(max(int(sym.stats["panel_size"]), 1), np.float64)
    PU = np.zeros_like(PL)
    rc = L.orc_assemble_lu(C.c_void_p(sym.handle), _p(_c(colptr, np.int64)), _p(_c(rowind, np.int32)),
                           _p(_c(values, np.float64)), _p(PL), _p(PU))
    if rc != 0:
        raise ValueError("assemble_lu failed")
    fc = C.c_int32(-1)
    nrep = C.c_int32(0)
    tau = static_pivot_tau(colptr, rowind, values, pivot_eps, False) if pivot_eps > 0 else 0.0
    rc = L.orc_factor_lu_sp(C.c_void_p(sym.handle), _p(PL), _p(PU), tau, C.byref(nrep), C.byref(fc))
    if rc == ENOTPD:
        raise ZeroPivot(fc.value, int(sym.perm[fc.value]))
    if rc != 0:
        raise RuntimeError("orc_factor_lu failed %d" % rc)
    return (PL, PU, nrep.value) if return_nrep else (PL, PU)


def solve_lu(sym: Symbolic, PL, PU, b):
    L = _load()
    b = np.asfortranarray(np.asarray(b, np.float64).reshape(sym.n, -1))
    x = np.zeros_like(b, order="F")
    L.orc_solve_lu(C.c_void_p(sym.handle), _p(PL), _p(PU), b.shape[1], _p(b), sym.n, _p(x), sym.n)
    return x


def logabsdet_lu(sym: Symbolic, PL):
    """(log |det A|, number of negative pivots u_jj) of an L U factor."""
    L = _load()
    nneg = C.c_int32(0)
    v = L.orc_logabsdet_lu(C.c_void_p(sym.handle), _p(PL), C.byref(nneg))
    return v, nneg.value


def solve(sym: Symbolic, P, b):
    L = _load()
    b = np.asfortranarray(np.asarray(b, np.float64).reshape(sym.n, -1))
    x = np.zeros_like(b, order="F")
    L.orc_solve(C.c_void_p(sym.handle), _p(P), b.shape[1], _p(b), sym.n, _p(x), sym.n)
    return x


def residual(n, colptr, rowind, values, x, b):
    """r = b - A x, s = |A||x| + |b| (lower triangle mirrored), per RHS column."""
    L = _load()
    colptr = _c(colptr, np.int64)
    rowind = _c(rowind, np.int32)
    values = _c(values, np.float64)
    x = np.asfortranarray(np.asarray(x, np.float64).reshape(n, -1))
    b = np.asfortranarray(np.asarray(b, np.float64).reshape(n, -1))
    r = np.zeros_like(x, order="F")
    s = np.zeros_like(x, order="F")
    for c in range(x.shape[1]):
        xc, bc = np.ascontiguousarray(x[:, c]), np.ascontiguousarray(b[:, c])
        rc, sc = np.zeros(n), np.zeros(n)
        L.orc_residual(n, _p(colptr), _p(rowind), _p(values), _p(xc), _p(bc), _p(rc), _p(sc))
        r[:, c], s[:, c] = rc, sc
    return r, s


def omega(r, s):
    L = _load()
    r = np.asarray(r, np.float64).reshape(r.shape[0], -1)
    s = np.asarray(s, np.float64).reshape(r.shape[0], -1)
    out = 0.0
    for c in range(r.shape[1]):
        rc, sc = np.ascontiguousarray(r[:, c]), np.ascontiguousarray(s[:, c])
        out = max(out, L.orc_omega(r.shape[0], _p(rc), _p(sc)))
    return out


def solve_refined(sym: Symbolic, P, colptr, rowind, values, b, max_steps=2, tol=1e-14):
    """FP64 solve followed by at most ``max_steps`` FP64 refinement steps.

    Returns x, the list of componentwise backward errors (one per iterate).
    """
    x = solve(sym, P, b)
    r, s = residual(sym.n, colptr, rowind, values, x, b)
    om = [omega(r, s)]
    for _ in range(max_steps):
        if om[-1] <= tol:
            break
        x = x + solve(sym, P, r)
        r, s = residual(sym.n, colptr, rowind, values, x, b)
        om.append(omega(r, s))
    return x, om


def logdet(sym: Symbolic, P):
    return _load().orc_logdet(C.c_void_p(sym.handle), _p(_c(P, np.float64)))


def unpack(sym: Symbolic, P):
    """Factor L as (rows, cols, vals) triplets in the final numbering."""
    L = _load()
    cnt = 0
    w = sym.lcol - sym.fcol + 1
    cnt = int(np.sum(w * (w + 1) // 2 + w * (sym.stride - w)))
    ri = np.zeros(cnt, np.int32)
    ci = np.zeros(cnt, np.int32)
    v = np.zeros(cnt, np.float64)
    q = L.orc_unpack(C.c_void_p(sym.handle), _p(_c(P, np.float64)), _p(ri), _p(ci), _p(v))
    assert q == cnt
    return ri, ci, v


def values_grad(n, colptr, rowind, x, db):
    """Gradient of a loss through x = A^{-1} b with respect to the stored values
    of A, given x and db = A^{-T} xbar (the derivative of x = A^{-1} b with
    respect to A is dA = -db x^T, summed over right-hand sides).  A stored
    lower entry a_ij (i > j) sets both A_ij and A_ji, so its gradient is
    -(db_i x_j + db_j x_i); a diagonal entry gets -db_i x_i; an entry above
    the diagonal is not read by the factorization and gets 0."""
    L = _load()
    colptr = _c(colptr, np.int64)
    rowind = _c(rowind, np.int32)
    x = np.asarray(x, np.float64).reshape(n, -1)
    db = np.asarray(db, np.float64).reshape(n, -1)
    xf, dbf = np.asfortranarray(x), np.asfortranarray(db)
    g = np.zeros(max(len(rowind), 1))
    L.orc_values_grad(n, _p(colptr), _p(rowind), x.shape[1], _p(xf), _p(dbf), n, _p(g))
    return g[:len(rowind)]


def adjoint(sym: Symbolic, P, colptr, rowind, values, x, xbar):
    """Backward pass of x = A^{-1} b for symmetric A: db = A^{-T} xbar = A^{-1} xbar
    (the same factor, refined), and the value gradient of ``values_grad``."""
    db, _ = solve_refined(sym, P, colptr, rowind, values, xbar)
    return db, values_grad(sym.n, colptr, rowind, x, db)
