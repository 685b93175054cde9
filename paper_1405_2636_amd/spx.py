"""ctypes binding of the C ABI declared in include/spx.h.

Argument marshalling only: device memory and streams come from torch
tensors, every step of analysis, factorization and solve runs in the native
library.  The library must be built (``python -m paper_1405_2636_amd._build``);
loading fails loudly otherwise, there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libspx.so")

SPX_OK, SPX_EINVAL, SPX_ENOMEM, SPX_EDEVICE, SPX_ESTATE, SPX_ENOTPD, SPX_ENOCONV = 0, -1, -2, -3, -4, -5, -6
PRECISIONS = {"fp64": 0, "fp32_ir": 1, "bf16x3_ir": 2}   # enum spx_precision
METHODS = {"llt": 0, "ldlt": 1, "lu": 2}                 # enum spx_method


class SpxError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("spx error %d: %s" % (code, msg))
        self.code = code


class NotPositiveDefinite(SpxError):
    def __init__(self, code, msg, col):
        super().__init__(code, msg)
        self.col = col


class NotConverged(SpxError):
    def __init__(self, code, msg, x, info):
        super().__init__(code, msg)
        self.x = x
        self.info = info


class Options(C.Structure):
    _fields_ = [("method", C.c_int32), ("leaf_size", C.c_int32), ("amalg_pct", C.c_int32),
                ("split_width", C.c_int32), ("user_perm", C.c_void_p), ("precision", C.c_int32),
                ("ir_max_iter", C.c_int32), ("ir_tol", C.c_double), ("trace", C.c_int32),
                ("graph", C.c_int32), ("tune", C.c_int32), ("tile", C.c_int32), ("fuse_small", C.c_int32),
                ("merge_split", C.c_int32), ("static_pivot_eps", C.c_double),
                ("deterministic", C.c_int32)]


class Info(C.Structure):
    _fields_ = [("n", C.c_int32), ("ncblk", C.c_int32), ("nblok", C.c_int32), ("nsnode", C.c_int32),
                ("nnz_a", C.c_int64), ("nnz_l", C.c_int64), ("nnz_l_stored", C.c_int64),
                ("panel_entries", C.c_int64), ("flops_alg", C.c_double), ("flops_exec", C.c_double),
                ("ntasks", C.c_int64), ("fail_col", C.c_int32), ("factorized", C.c_int32),
                ("logdet", C.c_double), ("factor_kernel_ms", C.c_double), ("assemble_ms", C.c_double),
                ("tile_rows", C.c_int32), ("tile_cols", C.c_int32), ("hp_policy", C.c_int32), ("nsys", C.c_int32),
                ("nfused_tiles", C.c_int64), ("nsmall", C.c_int32), ("nneg", C.c_int32),
                ("pivots_replaced", C.c_int32), ("solve_levels", C.c_int32), ("solve_pairs", C.c_int32)]


class SolveInfo(C.Structure):
    _fields_ = [("ir_iters", C.c_int32), ("converged", C.c_int32), ("omega", C.c_double), ("eta", C.c_double)]


SYMBOLIC_FIELDS = [
    ("perm", "n"), ("iperm", "n"), ("etree", "n"), ("snptr", "nsnode+1"), ("fcol", "ncblk"),
    ("lcol", "ncblk"), ("stride", "ncblk"), ("panel_off", "ncblk+1"), ("bptr", "ncblk+1"),
    ("cparent", "ncblk"), ("frow", "nblok"), ("lrow", "nblok"), ("fcblk", "nblok"),
    ("coefind", "nblok"), ("uptr", "ncblk+1"), ("utgt", "nupd"), ("dep", "ncblk"),
]


class SymView(C.Structure):
    _fields_ = ([("n", C.c_int32), ("ncblk", C.c_int32), ("nblok", C.c_int32), ("nsnode", C.c_int32),
                 ("nupd", C.c_int32)] + [(name, C.c_void_p) for name, _ in SYMBOLIC_FIELDS])


EXPORTED = ["spx_default_options", "spx_analyze", "spx_factorize", "spx_solve", "spx_get_info",
            "spx_export_symbolic", "spx_copy_factor", "spx_get_trace", "spx_destroy", "spx_strerror",
            "spx_last_error", "spx_values_grad", "spx_analyze_batch", "spx_solve_noalloc", "spx_update_bench"]

_lib = None


def load_library():
    """Load libspx.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("%s is missing: build it with `python -m paper_1405_2636_amd._build`" % LIB_PATH)
    L = C.CDLL(LIB_PATH)
    vp = C.c_void_p
    L.spx_default_options.restype = None
    L.spx_default_options.argtypes = [C.POINTER(Options)]
    L.spx_analyze.restype = C.c_int
    L.spx_analyze.argtypes = [C.c_int32, vp, vp, C.POINTER(Options), C.POINTER(vp)]
    L.spx_factorize.restype = C.c_int
    L.spx_factorize.argtypes = [vp, vp, C.c_int32, vp]
    L.spx_solve.restype = C.c_int
    L.spx_solve.argtypes = [vp, C.c_int32, vp, C.c_int64, C.c_int32, C.POINTER(SolveInfo), vp]
    L.spx_solve_noalloc.restype = C.c_int
    L.spx_solve_noalloc.argtypes = [vp, C.c_int32, vp, C.c_int64, C.POINTER(SolveInfo), vp]
    L.spx_get_info.restype = C.c_int
    L.spx_get_info.argtypes = [vp, C.POINTER(Info)]
    L.spx_export_symbolic.restype = C.c_int
    L.spx_export_symbolic.argtypes = [vp, C.POINTER(SymView)]
    L.spx_copy_factor.restype = C.c_int
    L.spx_copy_factor.argtypes = [vp, vp, C.c_int32, vp]
    L.spx_get_trace.restype = C.c_int64
    L.spx_get_trace.argtypes = [vp, vp, C.c_int64, vp]
    L.spx_analyze_batch.restype = C.c_int
    L.spx_analyze_batch.argtypes = [C.c_int32, vp, vp, vp, vp, vp]
    L.spx_values_grad.restype = C.c_int
    L.spx_values_grad.argtypes = [vp, C.c_int32, vp, vp, C.c_int64, vp, vp]
    L.spx_update_bench.restype = C.c_int
    L.spx_update_bench.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32, vp, vp, C.c_int32,
                                   C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_double)]
    L.spx_destroy.restype = None
    L.spx_destroy.argtypes = [vp]
    L.spx_strerror.restype = C.c_char_p
    L.spx_strerror.argtypes = [C.c_int]
    L.spx_last_error.restype = C.c_char_p
    L.spx_last_error.argtypes = [vp]
    _lib = L
    return L


def _stream_ptr(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


class Solver:
    """Sparse SPD solver: analyze at construction, then factorize(values), solve(b).

    colptr/rowind: CSC pattern (host arrays, full symmetric pattern or its lower
    triangle).  values passed to factorize are aligned with the pattern.
    precision: "fp64" (FP64 factor), "fp32_ir" (FP32 factor, FP64 residual
    and refinement) or "bf16x3_ir" (FP32 factor whose update products are
    split-BF16 products, FP64 refinement).  ir_max_iter None: the library's
    default for the precision (2 for fp64, 10 otherwise).  method: "llt"
    (P A P^T = L L^T, A positive definite) or "ldlt" (L D L^T with static
    pivoting, A symmetric with non-zero pivots, e.g. quasi-definite; fp64
    only; info()["logdet"] is then log |det A| and info()["nneg"] the number
    of negative pivots), or "lu" (P A P^T = L U with static pivoting, A
    unsymmetric, values of both triangles read; all precisions; the factor
    is the L panels followed by the U^T panels; no value gradient).
    static_pivot_eps (L D L^T and L U): None = the library's default (sqrt of
    the factor precision's unit roundoff), 0 = no replacement (a zero pivot
    is an error), else pivots below eps * max|a_ij| in magnitude are replaced
    (count in info()["pivots_replaced"]).
    deterministic: updates into each column block in ascending source order
    (the factor is reproducible bit for bit; fused small items off).
    """

    def __init__(self, n, colptr, rowind, leaf_size=64, amalg_pct=12, split_width=256, user_perm=None,
                 precision="fp64", ir_max_iter=None, ir_tol=1e-14, trace=False, graph=False, tune=False, tile=0,
                 fuse_small=True, merge_split=4, method="llt", static_pivot_eps=None, deterministic=False):
        L = load_library()
        self._lib = L
        self.n = int(n)
        self._colptr = np.ascontiguousarray(colptr, dtype=np.int64)
        self._rowind = np.ascontiguousarray(rowind, dtype=np.int32)
        self.nnz = int(self._colptr[-1]) if len(self._colptr) else 0
        self.sizes = [self.n]
        opt, up = self._options(L, leaf_size, amalg_pct, split_width, user_perm, precision, ir_max_iter, ir_tol,
                                trace, graph, tune, tile, fuse_small, merge_split, method, static_pivot_eps,
                                deterministic)
        h = C.c_void_p()
        rc = L.spx_analyze(self.n, self._colptr.ctypes.data, self._rowind.ctypes.data, C.byref(opt), C.byref(h))
        if rc != SPX_OK:
            raise SpxError(rc, "analyze failed: %s" % L.spx_last_error(None).decode())
        self._h = h

    def _options(self, L, leaf_size, amalg_pct, split_width, user_perm, precision, ir_max_iter, ir_tol, trace,
                 graph, tune, tile=0, fuse_small=True, merge_split=4, method="llt", static_pivot_eps=None,
                 deterministic=False):
        opt = Options()
        L.spx_default_options(C.byref(opt))
        opt.deterministic = 1 if deterministic else 0
        if static_pivot_eps is not None:
            opt.static_pivot_eps = float(static_pivot_eps)
        if method not in METHODS:
            raise ValueError("method must be one of %s" % sorted(METHODS))
        self.method = method
        opt.method = METHODS[method]
        opt.leaf_size, opt.amalg_pct, opt.split_width = leaf_size, amalg_pct, split_width
        if precision not in PRECISIONS:
            raise ValueError("precision must be one of %s" % sorted(PRECISIONS))
        self.precision = precision
        opt.precision = PRECISIONS[precision]
        opt.ir_max_iter = -1 if ir_max_iter is None else int(ir_max_iter)
        opt.ir_tol = ir_tol
        opt.trace = 1 if trace else 0
        opt.graph = 1 if graph else 0
        opt.tune = 1 if tune else 0
        opt.tile = int(tile)
        opt.fuse_small = 1 if fuse_small else 0
        opt.merge_split = int(merge_split)
        up = None
        if user_perm is not None:
            up = np.ascontiguousarray(user_perm, dtype=np.int32)
            opt.user_perm = up.ctypes.data
        return opt, up

    @classmethod
    def batch(cls, systems, precision="fp64", ir_max_iter=None, ir_tol=1e-14, graph=True, tune=True, **kw):
        """Independent systems [(n, colptr, rowind), ...] analysed, factored and
        solved together (one factorization launch for all, spx_analyze_batch).
        Values and right-hand sides are the systems' arrays concatenated in
        order; ``split`` cuts a concatenated vector back into systems."""
        self = cls.__new__(cls)
        L = load_library()
        self._lib = L
        ns = np.array([int(s[0]) for s in systems], np.int32)
        cps = [np.ascontiguousarray(s[1], dtype=np.int64) for s in systems]
        ris = [np.ascontiguousarray(s[2], dtype=np.int32) for s in systems]
        self.sizes = [int(v) for v in ns]
        self.n = int(ns.sum())
        self.nnz = int(sum(int(c[-1]) for c in cps))
        self._keep = (cps, ris)
        opt, _ = self._options(L, kw.get("leaf_size", 64), kw.get("amalg_pct", 12), kw.get("split_width", 256),
                               None, precision, ir_max_iter, ir_tol, kw.get("trace", False), graph, tune,
                               kw.get("tile", 0), kw.get("fuse_small", True), kw.get("merge_split", 4),
                               kw.get("method", "llt"), kw.get("static_pivot_eps"),
                               kw.get("deterministic", False))
        cpp = (C.c_void_p * len(cps))(*[c.ctypes.data for c in cps])
        rip = (C.c_void_p * len(ris))(*[r.ctypes.data for r in ris])
        h = C.c_void_p()
        rc = L.spx_analyze_batch(len(systems), ns.ctypes.data, C.cast(cpp, C.c_void_p), C.cast(rip, C.c_void_p),
                                 C.byref(opt), C.byref(h))
        if rc != SPX_OK:
            raise SpxError(rc, "analyze_batch failed: %s" % L.spx_last_error(None).decode())
        self._h = h
        return self

    def split(self, v):
        """A concatenated vector (last axis of length n) cut into the systems."""
        out, o = [], 0
        for m in self.sizes:
            out.append(v[..., o:o + m])
            o += m
        return out

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._lib.spx_destroy(h)
            self._h = None

    def _check(self, rc, what):
        if rc == SPX_OK:
            return
        msg = self._lib.spx_last_error(self._h).decode()
        if rc == SPX_ENOTPD:
            raise NotPositiveDefinite(rc, "%s: %s" % (what, msg), self.info()["fail_col"])
        raise SpxError(rc, "%s: %s" % (what, msg))

    # ---------------------------------------------------------------- calls
    def factorize(self, values, stream=None):
        """values: torch tensor on the GPU (float64) or a host numpy array."""
        import torch
        if isinstance(values, torch.Tensor):
            if values.dtype != torch.float64 or values.numel() != self.nnz:
                raise ValueError("values must be float64 with nnz entries")
            values = values.contiguous()
            on_dev = 1 if values.is_cuda else 0
            ptr = values.data_ptr()
            keep = values
        else:
            keep = np.ascontiguousarray(values, dtype=np.float64)
            if keep.size != self.nnz:
                raise ValueError("values must have nnz entries")
            on_dev, ptr = 0, keep.ctypes.data
        rc = self._lib.spx_factorize(self._h, C.c_void_p(ptr), on_dev, _stream_ptr(stream))
        del keep
        self._gen = getattr(self, "_gen", 0) + 1   # factorizations started on this handle
        self._check(rc, "factorize")

    def solve(self, b, stream=None, raise_on_noconv=True):
        """Solve A x = b.  b: torch CUDA tensor of shape (n,) or (nrhs, n)
        (each row one right-hand side), overwritten with x and returned with
        the refinement statistics."""
        import torch
        if not (isinstance(b, torch.Tensor) and b.is_cuda and b.dtype == torch.float64 and b.is_contiguous()):
            raise ValueError("b must be a contiguous float64 CUDA tensor")
        nrhs = 1 if b.dim() == 1 else b.shape[0]
        if b.shape[-1] != self.n:
            raise ValueError("b has the wrong length")
        si = SolveInfo()
        rc = self._lib.spx_solve(self._h, nrhs, C.c_void_p(b.data_ptr()), self.n, 1, C.byref(si), _stream_ptr(stream))
        info = {"ir_iters": si.ir_iters, "converged": bool(si.converged), "omega": si.omega, "eta": si.eta}
        if rc == SPX_ENOCONV and not raise_on_noconv:
            return b, info
        if rc == SPX_ENOCONV:
            raise NotConverged(rc, self._lib.spx_last_error(self._h).decode(), b, info)
        self._check(rc, "solve")
        return b, info

    def solve_noalloc(self, b, stream=None, raise_on_noconv=True):
        """solve() through spx_solve_noalloc: no device allocation (fixed work
        array of the library, n * nrhs up to about 1.19e6; calls on one device
        must not overlap).  b: contiguous float64 CUDA tensor (n,) or (nrhs, n)."""
        import torch
        if not (isinstance(b, torch.Tensor) and b.is_cuda and b.dtype == torch.float64 and b.is_contiguous()):
            raise ValueError("b must be a contiguous float64 CUDA tensor")
        nrhs = 1 if b.dim() == 1 else b.shape[0]
        if b.shape[-1] != self.n:
            raise ValueError("b has the wrong length")
        si = SolveInfo()
        rc = self._lib.spx_solve_noalloc(self._h, nrhs, C.c_void_p(b.data_ptr()), self.n, C.byref(si),
                                         _stream_ptr(stream))
        info = {"ir_iters": si.ir_iters, "converged": bool(si.converged), "omega": si.omega, "eta": si.eta}
        if rc == SPX_ENOCONV and not raise_on_noconv:
            return b, info
        if rc == SPX_ENOCONV:
            raise NotConverged(rc, self._lib.spx_last_error(self._h).decode(), b, info)
        self._check(rc, "solve_noalloc")
        return b, info

    def info(self) -> dict:
        inf = Info()
        rc = self._lib.spx_get_info(self._h, C.byref(inf))
        if rc != SPX_OK:
            raise SpxError(rc, "get_info failed")
        return {name: getattr(inf, name) for name, _ in Info._fields_}

    def symbolic(self) -> dict:
        """Copies of the exported symbolic arrays (numpy)."""
        v = SymView()
        rc = self._lib.spx_export_symbolic(self._h, C.byref(v))
        if rc != SPX_OK:
            raise SpxError(rc, "export_symbolic failed")
        sizes = {"n": v.n, "ncblk": v.ncblk, "nblok": v.nblok, "nsnode": v.nsnode, "nupd": v.nupd}
        out = {}
        for name, sz in SYMBOLIC_FIELDS:
            cnt = sizes[sz.split("+")[0]] + (1 if sz.endswith("+1") else 0)
            dt = np.int64 if name == "panel_off" else np.int32
            ptr = getattr(v, name)
            if cnt == 0 or not ptr:
                out[name] = np.zeros(0, dt)
                continue
            ct = C.c_int64 if dt == np.int64 else C.c_int32
            buf = (ct * cnt).from_address(ptr)
            out[name] = np.ctypeslib.as_array(buf).copy()
        out.update(sizes)
        return out

    def trace(self):
        """Per-item trace of the last factorization: (times int64 [items, 4], kinds int32 [items, 4])."""
        cnt = self.info()["ntasks"]
        t = np.zeros((max(cnt, 1), 4), np.int64)
        k = np.zeros((max(cnt, 1), 4), np.int32)
        rc = self._lib.spx_get_trace(self._h, t.ctypes.data, cnt, k.ctypes.data)
        if rc < 0:
            self._check(int(rc), "get_trace")
        return t[:cnt], k[:cnt]

    def factor_values(self, out=None, stream=None):
        """The factor panels (panel_entries doubles) as a torch CUDA tensor."""
        import torch
        cnt = self.info()["panel_entries"] * (2 if self.method == "lu" else 1)
        if out is None:
            out = torch.empty(max(cnt, 1), dtype=torch.float64, device="cuda")
        rc = self._lib.spx_copy_factor(self._h, C.c_void_p(out.data_ptr()), 1, _stream_ptr(stream))
        self._check(rc, "copy_factor")
        return out[:cnt]

    def values_grad(self, x, db, stream=None):
        """Adjoint of the solve: gradient with respect to the values given x and
        db = A^{-1} xbar (torch CUDA float64 tensors of shape (n,) or (nrhs, n),
        one right-hand side per row).  Returns a float64 CUDA tensor of nnz
        entries (zero for entries above the diagonal, which are not read)."""
        import torch
        for t in (x, db):
            if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
                raise ValueError("x and db must be contiguous float64 CUDA tensors")
        if x.shape != db.shape or x.shape[-1] != self.n:
            raise ValueError("x and db must have the same shape (n,) or (nrhs, n)")
        nrhs = 1 if x.dim() == 1 else x.shape[0]
        grad = torch.empty(max(self.nnz, 1), dtype=torch.float64, device=x.device)
        rc = self._lib.spx_values_grad(self._h, nrhs, C.c_void_p(x.data_ptr()), C.c_void_p(db.data_ptr()), self.n,
                                       C.c_void_p(grad.data_ptr()), _stream_ptr(stream))
        self._check(rc, "values_grad")
        return grad[:self.nnz]


def update_bench(panels, rmap, n_inner, m, k, ldc, precision="fp64", method="llt", tile=0, calls=1, nstreams=1):
    """The library's update-kernel microbenchmark (spx_update_bench): calls
    updates C -= A B^T (L D L^T: A D B^T) of the synthetic source panel into
    the target panel, both in the device tensor `panels` (float64 for
    "fp64", float32 otherwise; layout in include/spx.h), through the int32
    device row map `rmap`.  Returns the elapsed milliseconds."""
    import torch
    L = load_library()
    if precision not in PRECISIONS or method not in ("llt", "ldlt"):
        raise ValueError("precision or method")
    want = torch.float64 if precision == "fp64" else torch.float32
    if panels.dtype != want or not panels.is_cuda or not panels.is_contiguous():
        raise ValueError("panels must be a contiguous %s device tensor" % want)
    if rmap.dtype != torch.int32 or not rmap.is_cuda or rmap.numel() != m:
        raise ValueError("rmap must be an int32 device tensor of m entries")
    if panels.numel() < (n_inner + m) * n_inner + ldc * k:
        raise ValueError("panels too small")
    ms = C.c_double()
    rc = L.spx_update_bench(PRECISIONS[precision], METHODS[method], n_inner, m, k, C.c_void_p(panels.data_ptr()),
                            C.c_void_p(rmap.data_ptr()), ldc, tile, calls, nstreams, C.byref(ms))
    if rc != 0:
        raise SpxError(rc, L.spx_last_error(None).decode())
    return ms.value


def _solve_function():
    import torch

    class SolveFunction(torch.autograd.Function):
        """x = A(values)^{-1} b with a hand-written adjoint: the backward pass
        solves with the same factor (db = A^{-1} xbar, A symmetric) and forms the
        value gradient -db x^T restricted to the pattern (spx_values_grad).
        If the solver was factorized again between this forward pass and its
        backward pass (another solve_autograd call on the same solver), the
        backward pass first refactorizes the values saved by the forward pass,
        so that db and the gradient belong to this pass's matrix."""

        @staticmethod
        def forward(ctx, values, b, solver):
            v = values.detach().contiguous()
            solver.factorize(v)
            x, _ = solver.solve(b.detach().clone().contiguous())
            ctx.solver = solver
            ctx.gen = solver._gen
            ctx.save_for_backward(x, v)
            return x

        @staticmethod
        def backward(ctx, xbar):
            x, v = ctx.saved_tensors
            solver = ctx.solver
            if solver._gen != ctx.gen:
                solver.factorize(v)
                ctx.gen = solver._gen
            db, _ = solver.solve(xbar.detach().clone().contiguous())
            gv = solver.values_grad(x, db) if ctx.needs_input_grad[0] else None
            return gv, (db if ctx.needs_input_grad[1] else None), None

    return SolveFunction


_SOLVE_FN = None


def solve_autograd(solver, values, b):
    """Differentiable x = A^{-1} b for the pattern analysed by ``solver``:
    values (nnz,) and b ((n,) or (nrhs, n)) are float64 CUDA tensors; gradients
    flow to both.  Each call factorizes ``values``."""
    global _SOLVE_FN
    if _SOLVE_FN is None:
        _SOLVE_FN = _solve_function()
    return _SOLVE_FN.apply(values, b, solver)
