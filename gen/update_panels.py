"""Synthetic panels of the update-kernel study (Section V-B, Fig. 2): one
source panel (an n x n diagonal block over the m rows of A) and the row map
of A's rows into a target panel.  B is the first k rows of A (the target's
own columns).  Dense target: m rows, A's rows in order.  Gapped target: 2m
rows; below its k x k diagonal block the target is cut into blocks of random
height (mean 200 rows), and every block holds one block of A's remaining
rows at a random offset inside it (no two A blocks overlap), the A blocks'
heights in proportion to their target blocks."""
from __future__ import annotations

import numpy as np


def update_panels(n: int, m: int, k: int, gapped: bool, seed: int = 0, mean_block: int = 200):
    """Returns (panel, rmap, ldc): panel = float64 array of (n + m) * n
    entries (column-major source panel; the diagonal block holds pivots of
    magnitude 0.5 .. 1.5 with random signs on its diagonal, the rows of A
    values uniform in [-1, 1]), rmap = int32 array of the target row of each
    row of A, ldc = the target panel's height."""
    if not (1 <= k <= m):
        raise ValueError("need 1 <= k <= m")
    rng = np.random.default_rng(seed)
    ld = n + m
    P = np.zeros((ld, n))
    P[:n, :n] = np.diag(rng.uniform(0.5, 1.5, n) * rng.choice([-1.0, 1.0], n))
    P[n:, :] = rng.uniform(-1.0, 1.0, (m, n))
    if not gapped:
        return P.ravel(order="F"), np.arange(m, dtype=np.int32), m
    ldc = 2 * m
    below = ldc - k          # target rows below its diagonal block
    rest = m - k             # rows of A below B
    heights = []
    while sum(heights) < below:
        heights.append(int(rng.integers(mean_block // 2, 3 * mean_block // 2 + 1)))
    heights[-1] -= sum(heights) - below
    if heights[-1] <= 0:
        heights.pop()
        heights[-1] += below - sum(heights)
    h = np.array(heights)
    # A-block heights in proportion to the target blocks, summing to `rest`
    a = np.floor(h * rest / below).astype(int)
    short = rest - int(a.sum())
    order = np.argsort(-(h * rest / below - a))
    for q in order[:short]:
        a[q] += 1
    assert np.all(a <= h) and int(a.sum()) == rest
    rmap = list(range(k))
    start = k
    for hq, aq in zip(h, a):
        off = int(rng.integers(0, hq - aq + 1))
        rmap.extend(range(start + off, start + off + aq))
        start += hq
    return P.ravel(order="F"), np.array(rmap, dtype=np.int32), ldc
