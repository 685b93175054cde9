"""GPU checks at the benchmark workloads' full sizes, where the oracle's own
factorization would take many minutes: properties that hold at any size.

* 100^3 7-point Laplacian + 1e-3 (N = 1e6), the three precision modes:
  - log det against the closed form sum log(lambda) over the eigenvalues
    lambda = sum_d (2 - 2 cos(i_d pi / 101)) + 1e-3 (relative 1e-10; one wrong
    update moves it by O(1));
  - the factor residual ||P A P^T - L L^T||_F / ||A||_F estimated with 8
    Rademacher probes v: sqrt(sum ||A v - L (L^T v)||^2 / sum ||A v||^2)
    (each sum is an unbiased estimate of 8 ||.||_F^2): <= 1e-12 in FP64; the
    FP32 factor at 1e-6 (16 units of FP32 rounding 2^-24; measured 6.6e-8)
    and the split-BF16 one at 1e-5 (the 2^-16 = 1.5e-5 of its products;
    measured 7.4e-7);
  - the refined solve reaches omega <= 1e-14 in every mode, and the three
    modes' solutions agree to kappa * omega (kappa ~ 3.1e3).
* the 512-system batch (2-D weighted grids, sides 16..96), FP64 and
  FP32 + refinement, graph-replayed and tuned: every system's x against the
  oracle's refined solution.
* 80^3 convection-diffusion (N = 512,000), L U with static pivoting and 4
  right-hand sides, the three precision modes: omega <= 1e-14, the probe
  residual of L U (1e-12 in FP64; FP32 gates as above), no negative pivot
  (an M-matrix), solutions agreeing across modes.
* 40^3 clamped elasticity (N = 192,000, 27-point 3-dof), L D L^T with 8
  right-hand sides: omega <= 1e-14, probe residual of L D L^T <= 1e-12,
  log |det| and inertia equal to those of the L L^T factorization of the same
  matrix, and the adjoint against central finite differences of the solve.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from gen import grid_batch, make_config, rhs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


def _panel_rows(sv):
    """Global row (new numbering) of every panel row, cblk by cblk, and the
    offset of each cblk's rows."""
    nb = len(sv["frow"])
    lens = sv["lrow"] - sv["frow"] + 1
    starts = np.repeat(sv["frow"] - np.concatenate([[0], np.cumsum(lens)[:-1]]), lens)
    rows = (np.arange(int(lens.sum())) + starts).astype(np.int64)
    assert len(rows) == int(sv["stride"].astype(np.int64).sum()) and nb == sv["nblok"]
    off = np.concatenate([[0], np.cumsum(sv["stride"].astype(np.int64))])
    return rows, off


def _probe_residual(torch, s, p, ldlt=False, nprobe=8, seed=5, lu=False):
    """Rademacher estimate of ||P A P^T - L L^T||_F / ||A||_F (L D L^T with
    ldlt, L U with lu); the factor products on the GPU (torch), A v on the
    host."""
    sv = s.symbolic()
    F = s.factor_values()
    if lu:
        return _probe_residual_lu(torch, sv, F, p, nprobe, seed)
    rows, roff = _panel_rows(sv)
    rows_d = torch.tensor(rows, device="cuda")
    n = p.n
    rng = np.random.default_rng(seed)
    V = rng.integers(0, 2, (n, nprobe)).astype(np.float64) * 2.0 - 1.0   # new numbering
    Vd = torch.tensor(V, device="cuda")
    T = torch.zeros_like(Vd)
    Y = torch.zeros_like(Vd)
    blocks = []
    for k in range(sv["ncblk"]):
        f, w, ld, off = int(sv["fcol"][k]), int(sv["lcol"][k] - sv["fcol"][k] + 1), int(sv["stride"][k]), \
            int(sv["panel_off"][k])
        Pk = F[off:off + ld * w].view(w, ld).t()          # (ld, w), column-major panel
        if ldlt:
            d = torch.diagonal(Pk[:w, :w]).clone()
            Pk = Pk.clone()
            Pk[:w, :w].fill_diagonal_(1.0)
        else:
            d = None
        blocks.append((f, w, Pk, d, rows_d[roff[k]:roff[k + 1]]))
    for f, w, Pk, d, r in blocks:                      # T = L^T V  (D L^T V)
        t = Pk.t() @ Vd[r]
        T[f:f + w] = t * d[:, None] if ldlt else t
    for f, w, Pk, d, r in blocks:                      # Y = L T
        Y.index_add_(0, r, Pk @ T[f:f + w])
    A = sp.csr_matrix((p.values, p.rowind, p.colptr), shape=(n, n)).T.tocsr()   # CSC arrays -> A
    perm = sv["perm"]
    U = np.empty_like(V)
    U[perm] = V
    R = (A @ U)[perm]
    num = float(((torch.tensor(R, device="cuda") - Y) ** 2).sum())
    return np.sqrt(num / float((R ** 2).sum()))


def _probe_residual_lu(torch, sv, F, p, nprobe, seed):
    rows, roff = _panel_rows(sv)
    rows_d = torch.tensor(rows, device="cuda")
    n = p.n
    pe = int(sv["panel_off"][-1])
    rng = np.random.default_rng(seed)
    V = rng.integers(0, 2, (n, nprobe)).astype(np.float64) * 2.0 - 1.0
    Vd = torch.tensor(V, device="cuda")
    T = torch.zeros_like(Vd)
    Y = torch.zeros_like(Vd)
    blocks = []
    for k in range(sv["ncblk"]):
        f, w, ld, off = int(sv["fcol"][k]), int(sv["lcol"][k] - sv["fcol"][k] + 1), int(sv["stride"][k]), \
            int(sv["panel_off"][k])
        Pk = F[off:off + ld * w].view(w, ld).t()              # L panel (ld, w)
        Uk = F[pe + off:pe + off + ld * w].view(w, ld).t()    # U^T panel (ld, w)
        sq = Pk[:w, :w]
        blocks.append((f, w, torch.tril(sq, -1) + torch.eye(w, dtype=sq.dtype, device="cuda"), torch.triu(sq),
                       Pk[w:], Uk[w:], rows_d[roff[k] + w:roff[k + 1]]))
    for f, w, Lsq, Usq, Lo, Uo, r in blocks:             # T = U V
        T[f:f + w] = Usq @ Vd[f:f + w] + Uo.t() @ Vd[r]
    for f, w, Lsq, Usq, Lo, Uo, r in blocks:             # Y = L T
        Y[f:f + w] += Lsq @ T[f:f + w]
        Y.index_add_(0, r, Lo @ T[f:f + w])
    A = sp.csr_matrix((p.values, p.rowind, p.colptr), shape=(n, n)).T.tocsr()
    perm = sv["perm"]
    U = np.empty_like(V)
    U[perm] = V
    R = (A @ U)[perm]
    num = float(((torch.tensor(R, device="cuda") - Y) ** 2).sum())
    return np.sqrt(num / float((R ** 2).sum()))


def _laplace_logdet_100():
    ev = 2.0 - 2.0 * np.cos(np.arange(1, 101) * np.pi / 101)
    lam = ev[:, None, None] + ev[None, :, None] + ev[None, None, :] + 1e-3
    return float(np.sum(np.log(lam)))


@pytest.fixture(scope="module")
def c2():
    return make_config(2)


@pytest.fixture(scope="module")
def c2_x64(torch, c2):
    from paper_1405_2636_amd import Solver
    s = Solver(c2.n, c2.colptr, c2.rowind)
    s.factorize(torch.tensor(c2.values, device="cuda"))
    x, info = s.solve(torch.tensor(np.ascontiguousarray(c2.b[:, 0]), device="cuda"))
    return s, x.cpu().numpy(), info


def test_laplace100_fp64_closed_form_and_residual(torch, c2, c2_x64):
    s, x, info = c2_x64
    print("100^3 fp64: omega %.2e ir %d" % (info["omega"], info["ir_iters"]), flush=True)
    ref = _laplace_logdet_100()
    ld = s.info()["logdet"]
    assert abs(ld - ref) <= 1e-10 * abs(ref), (ld, ref)
    res = _probe_residual(torch, s, c2)
    print("100^3 fp64 probe residual %.3e" % res, flush=True)
    assert res <= 1e-12
    assert info["omega"] <= 1e-14 and info["converged"]


@pytest.mark.parametrize("prec,gate", [("fp32_ir", 1e-6), ("bf16x3_ir", 1e-5)])
def test_laplace100_refinement_modes(torch, c2, c2_x64, prec, gate):
    from paper_1405_2636_amd import Solver
    _, x64, _ = c2_x64
    s = Solver(c2.n, c2.colptr, c2.rowind, precision=prec)
    s.factorize(torch.tensor(c2.values, device="cuda"))
    x, info = s.solve(torch.tensor(np.ascontiguousarray(c2.b[:, 0]), device="cuda"))
    res = _probe_residual(torch, s, c2)
    ld = s.info()["logdet"]
    ref = _laplace_logdet_100()
    print("100^3 %s: omega %.2e ir %d probe residual %.3e logdet rel %.2e"
          % (prec, info["omega"], info["ir_iters"], res, abs(ld - ref) / abs(ref)), flush=True)
    assert info["omega"] <= 1e-14 and info["converged"]
    assert res <= gate
    xg = x.cpu().numpy()
    assert np.max(np.abs(xg - x64)) <= 3.1e3 * 1e-14 * 10 * np.max(np.abs(x64))


def test_batch512_against_oracle(orc, torch):
    from paper_1405_2636_amd import Solver
    ps = grid_batch(512)
    assert len(ps) == 512 and min(min(q.meta["dims"]) for q in ps) >= 16
    assert max(max(q.meta["dims"]) for q in ps) <= 96
    xs = []
    for q in ps:
        sym = orc.analyze(q.n, q.colptr, q.rowind)
        P = orc.factor(sym, q.colptr, q.rowind, q.values)
        xo, _ = orc.solve_refined(sym, P, q.colptr, q.rowind, q.values, q.b)
        xs.append(xo[:, 0])
    systems = [(q.n, q.colptr, q.rowind) for q in ps]
    vals = torch.tensor(np.concatenate([q.values for q in ps]), device="cuda")
    b0 = torch.tensor(np.concatenate([q.b[:, 0] for q in ps]), device="cuda")
    for prec in ("fp64", "fp32_ir"):
        print("batch512 %s" % prec, flush=True)
        s = Solver.batch(systems, precision=prec, graph=True, tune=True)
        for rep in range(2):   # tuning run, then a graph replay
            s.factorize(vals)
            x, info = s.solve(b0.clone())
            assert info["omega"] <= 1e-14 and info["converged"]
            for xg, xo in zip(s.split(x.cpu().numpy()), xs):
                assert np.max(np.abs(xg - xo)) <= 1e-8 * np.max(np.abs(xo))


@pytest.fixture(scope="module")
def c5():
    return make_config(5)


def test_elasticity40_ldlt_8rhs(torch, c5):
    from paper_1405_2636_amd import Solver
    p = c5
    assert p.n == 192000 and p.nnz == 14787288 and p.b.shape == (p.n, 8)
    s = Solver(p.n, p.colptr, p.rowind, method="ldlt")
    vals = torch.tensor(p.values, device="cuda")
    s.factorize(vals)
    B = torch.tensor(np.ascontiguousarray(p.b.T), device="cuda")
    x, info = s.solve(B.clone())
    print("elasticity ldlt: omega %.2e ir %d" % (info["omega"], info["ir_iters"]), flush=True)
    assert info["omega"] <= 1e-14 and info["converged"]
    res = _probe_residual(torch, s, p, ldlt=True)
    print("elasticity ldlt probe residual %.3e" % res, flush=True)
    assert res <= 1e-12
    inf = s.info()
    sl = Solver(p.n, p.colptr, p.rowind)
    sl.factorize(vals)
    ll = sl.info()["logdet"]
    assert inf["nneg"] == 0
    assert abs(inf["logdet"] - ll) <= 1e-12 * abs(ll)
    xl, _ = sl.solve(B.clone())
    assert torch.max(torch.abs(xl - x)).item() <= 1e-9 * torch.max(torch.abs(xl)).item()


def test_elasticity40_ldlt_adjoint_finite_differences(torch, c5):
    # loss = sum(c * x) over the 8 right-hand sides; directional derivative
    # along a random perturbation of the stored lower values (scaled to the
    # entries, so the matrix stays definite), central differences of the GPU
    # solve itself
    from paper_1405_2636_amd import Solver, solve_autograd
    p = c5
    s = Solver(p.n, p.colptr, p.rowind, method="ldlt")
    rng = np.random.default_rng(17)
    C = torch.tensor(rng.uniform(-1, 1, (8, p.n)), device="cuda")
    B = torch.tensor(np.ascontiguousarray(p.b.T), device="cuda")
    v0 = torch.tensor(p.values, device="cuda")
    dv = torch.tensor(rng.uniform(-1, 1, p.nnz) * 1e-3 * np.abs(p.values), device="cuda")
    # (step: 1e-4 of each entry; truncation ~1e-8, rounding of the two losses
    # ~ kappa * 1e-14 / 1e-4 relative)
    v = v0.clone().requires_grad_(True)
    loss = (C * solve_autograd(s, v, B)).sum()
    (g,) = torch.autograd.grad(loss, v)
    analytic = float((g * dv).sum())
    h = 0.1

    def L(vals):
        with torch.no_grad():
            return float((C * solve_autograd(s, vals, B)).sum())

    fd = (L(v0 + h * dv) - L(v0 - h * dv)) / (2 * h)
    print("elasticity adjoint: analytic %.10e fd %.10e" % (analytic, fd), flush=True)
    assert abs(fd - analytic) <= 1e-5 * max(1.0, abs(fd))


@pytest.fixture(scope="module")
def c3():
    return make_config(3)


@pytest.fixture(scope="module")
def c3_x64(torch, c3):
    from paper_1405_2636_amd import Solver
    s = Solver(c3.n, c3.colptr, c3.rowind, method="lu")
    s.factorize(torch.tensor(c3.values, device="cuda"))
    x, info = s.solve(torch.tensor(np.ascontiguousarray(c3.b.T), device="cuda"))
    return s, x.cpu().numpy(), info


def test_convdiff80_lu_fp64(torch, c3, c3_x64):
    s, x, info = c3_x64
    assert c3.n == 512000 and c3.nnz == 3545600 and c3.b.shape == (c3.n, 4)
    print("80^3 lu fp64: omega %.2e ir %d" % (info["omega"], info["ir_iters"]), flush=True)
    assert info["omega"] <= 1e-14 and info["converged"]
    res = _probe_residual(torch, s, c3, lu=True)
    print("80^3 lu fp64 probe residual %.3e" % res, flush=True)
    assert res <= 1e-12
    # the matrix is an irreducibly diagonally dominant M-matrix: every pivot
    # of L U without pivoting is positive
    assert s.info()["nneg"] == 0


@pytest.mark.parametrize("prec,gate", [("fp32_ir", 1e-6), ("bf16x3_ir", 1e-5)])
def test_convdiff80_lu_refinement_modes(torch, c3, c3_x64, prec, gate):
    from paper_1405_2636_amd import Solver
    s64, x64, _ = c3_x64
    s = Solver(c3.n, c3.colptr, c3.rowind, method="lu", precision=prec)
    s.factorize(torch.tensor(c3.values, device="cuda"))
    x, info = s.solve(torch.tensor(np.ascontiguousarray(c3.b.T), device="cuda"))
    res = _probe_residual(torch, s, c3, lu=True)
    ld, ld64 = s.info()["logdet"], s64.info()["logdet"]
    print("80^3 lu %s: omega %.2e ir %d probe residual %.3e logdet rel diff to fp64 %.2e"
          % (prec, info["omega"], info["ir_iters"], res, abs(ld - ld64) / abs(ld64)), flush=True)
    assert info["omega"] <= 1e-14 and info["converged"]
    assert res <= gate
    # both refined to omega <= 1e-14; kappa of the stencil ~ 3e3
    assert np.max(np.abs(x.cpu().numpy() - x64)) <= 3e3 * 1e-14 * 10 * np.max(np.abs(x64))
