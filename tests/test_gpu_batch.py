"""Batched independent systems (spx_analyze_batch): one factorization launch
for all systems, the factorization replayed from a captured HIP graph, the
work decomposition chosen by the autotuner.  Every system's solution is
compared with the oracle solving that system alone; every graph replay is
checked (the same tolerances as the single-system tests)."""
import numpy as np
import pytest

from gen import grid_batch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


def _oracle_x(orc, p, values, b):
    sym = orc.analyze(p.n, p.colptr, p.rowind)
    P = orc.factor(sym, p.colptr, p.rowind, values)
    x, _ = orc.solve_refined(sym, P, p.colptr, p.rowind, values, b)
    return x[:, 0]


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir", "bf16x3_ir"])
def test_batch_parity_with_graph_replays(orc, torch, precision):
    ps = grid_batch(40, seed=11, lo=6, hi=48)
    print("batch of %d systems, n=%d, %s" % (len(ps), sum(p.n for p in ps), precision), flush=True)
    from paper_1405_2636_amd import Solver
    s = Solver.batch([(p.n, p.colptr, p.rowind) for p in ps], precision=precision, graph=True, tune=True)
    b = np.concatenate([p.b[:, 0] for p in ps])
    for rep, scale in enumerate([1.0, 2.5, 0.5]):
        vals = np.concatenate([p.values for p in ps]) * scale
        s.factorize(torch.tensor(vals, device="cuda"))
        x, info = s.solve(torch.tensor(b, device="cuda"))
        assert info["converged"] and info["omega"] <= 1e-14, (rep, info)
        xs = s.split(x.cpu().numpy())
        for q, p in enumerate(ps):
            xo = _oracle_x(orc, p, p.values * scale, p.b)
            assert np.max(np.abs(xs[q] - xo)) <= 1e-10 * np.max(np.abs(xo)), (rep, q)
    inf = s.info()
    assert (inf["tile_rows"], inf["tile_cols"]) in [(256, 64), (128, 128)] and inf["hp_policy"] in (0, 1)
    assert inf["nsys"] == 40


@pytest.mark.parametrize("tile,graph", [(0, False), (1, False), (1, True)])
def test_tile_shapes_agree(orc, torch, tile, graph):
    # 256x64 and 128x128 update tiles (forced), eager and graph-replayed:
    # the factor equals the oracle's, factorized twice in a row
    from gen.stencils import grid_laplacian
    from paper_1405_2636_amd import Solver
    p = grid_laplacian((24, 22, 20), shift=1e-3)
    sym = orc.analyze(p.n, p.colptr, p.rowind)
    P = orc.factor(sym, p.colptr, p.rowind, p.values)
    s = Solver(p.n, p.colptr, p.rowind, tile=tile, graph=graph)
    inf = s.info()
    assert (inf["tile_rows"], inf["tile_cols"]) == ((128, 128) if tile else (256, 64))
    for _ in range(2):
        s.factorize(torch.tensor(p.values, device="cuda"))
        F = s.factor_values().cpu().numpy()
        assert np.max(np.abs(F - P)) <= 1e-10 * np.max(np.abs(P))
