"""The update-kernel microbenchmark entry point (spx_update_bench) computes
what the update tiles must: after `calls` calls the target panel holds
C0 - calls * A_rows B^T (L D L^T: A_rows D B^T) on the target rows given by
the row map, lower triangle of the target's diagonal block only, and is
unchanged elsewhere.  Reference: the same product in numpy FP64 on the same
panels.  Tolerances: 1e-12 relative to the largest |update| in FP64, 1e-5
for FP32 products, 1e-4 for the split-BF16 products (2^-16 per product).
Dense and gapped targets (the Fig. 2 recipe), both tile shapes, one grid
and several streams, ragged M and K.  Bad arguments are refused."""
import numpy as np
import pytest

from gen import update_panels

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


def _run(torch, n, m, k, gapped, precision="fp64", method="llt", tile=0, calls=2, nstreams=2, seed=0):
    from paper_1405_2636_amd.spx import update_bench
    print("update bench case n=%d m=%d k=%d gapped=%s prec=%s method=%s tile=%d calls=%d streams=%d"
          % (n, m, k, gapped, precision, method, tile, calls, nstreams), flush=True)
    P, rmap, ldc = update_panels(n, m, k, gapped, seed)
    rng = np.random.default_rng(seed + 1)
    C0 = rng.uniform(-1, 1, ldc * k)
    dt = torch.float64 if precision == "fp64" else torch.float32
    buf = torch.tensor(np.concatenate([P, C0]), dtype=dt, device="cuda")
    Pr = buf[:P.size].cpu().numpy().astype(np.float64).reshape(n, n + m).T   # the values as stored
    C0r = buf[P.size:].cpu().numpy().astype(np.float64)
    update_bench(buf, torch.tensor(rmap, device="cuda"), n, m, k, ldc, precision, method, tile, calls, nstreams)
    C = buf[P.size:].cpu().numpy().astype(np.float64).reshape(k, ldc).T
    A = Pr[n:, :]
    Dd = np.diag(Pr[:n, :n]) if method == "ldlt" else np.ones(n)
    W = (A * Dd) @ A[:k, :].T      # m x k
    ref = C0r.reshape(k, ldc).T.copy()
    mask = np.zeros((ldc, k), bool)
    for i in range(m):
        cols = np.arange(k) if i >= k else np.arange(i + 1)
        ref[rmap[i], cols] -= calls * W[i, cols]
        mask[rmap[i], cols] = True
    tol = {"fp64": 1e-12, "fp32_ir": 1e-5, "bf16x3_ir": 1e-4}[precision]
    scale = calls * np.max(np.abs(W))
    assert np.max(np.abs(C - ref)) <= tol * scale
    assert np.array_equal(C[~mask], ref[~mask])   # rows outside the map and the strict upper triangle untouched


@pytest.mark.parametrize("gapped", [False, True])
@pytest.mark.parametrize("n,m,k", [(64, 600, 64), (128, 1000, 128), (256, 1500, 256), (40, 333, 37)])
def test_update_bench_fp64(torch, gapped, n, m, k):
    _run(torch, n, m, k, gapped)


@pytest.mark.parametrize("precision", ["fp32_ir", "bf16x3_ir"])
@pytest.mark.parametrize("method", ["llt", "ldlt"])
def test_update_bench_modes(torch, precision, method):
    _run(torch, 128, 900, 128, True, precision, method)


@pytest.mark.parametrize("tile,nstreams,calls", [(1, 1, 1), (1, 3, 5), (0, 0, 4), (1, 0, 3)])
def test_update_bench_launch_shapes(torch, tile, nstreams, calls):
    _run(torch, 96, 700, 96, True, tile=tile, nstreams=nstreams, calls=calls)
    _run(torch, 64, 300, 64, False, method="ldlt", tile=tile, nstreams=nstreams, calls=calls)


def test_update_bench_rejects(torch):
    from paper_1405_2636_amd import SpxError
    from paper_1405_2636_amd.spx import update_bench
    P, rmap, ldc = update_panels(32, 100, 32, True, 3)
    buf = torch.zeros(P.size + ldc * 32, dtype=torch.float64, device="cuda")
    bad = rmap.copy()
    bad[50], bad[51] = bad[51], bad[50]           # not increasing
    with pytest.raises(SpxError):
        update_bench(buf, torch.tensor(bad, device="cuda"), 32, 100, 32, ldc)
    bad = rmap.copy()
    bad[-1] = ldc                                 # outside the target
    with pytest.raises(SpxError):
        update_bench(buf, torch.tensor(bad, device="cuda"), 32, 100, 32, ldc)
    with pytest.raises(SpxError):
        update_bench(buf, torch.tensor(rmap, device="cuda"), 32, 100, 32, ldc, nstreams=4)
    with pytest.raises(ValueError):
        update_bench(buf.float(), torch.tensor(rmap, device="cuda"), 32, 100, 32, ldc)
