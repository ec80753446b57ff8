"""Helpers for the GPU tests: device copies of seeded inputs, comparisons."""
import numpy as np

import oracle


def torch_dev():
    import torch
    return torch


def to_dev(a):
    """uint32 numpy -> int32 torch tensor on cuda:0 (same bits)."""
    torch = torch_dev()
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int32)).to("cuda:0")


def from_dev(t):
    torch = torch_dev()
    torch.cuda.synchronize()
    return t.cpu().numpy().view(np.uint32)


def sample_positions(m, n, count, seed):
    """Sampled output positions: the four corners, a full first and last row
    and column where small, and seeded random positions."""
    rng = np.random.default_rng(seed)
    rows = [0, 0, m - 1, m - 1]
    cols = [0, n - 1, 0, n - 1]
    rows += list(rng.integers(0, m, count))
    cols += list(rng.integers(0, n, count))
    # every tile edge of the 128 x 128 / 128 x 64 / 32 x 32 tilings
    for e in (31, 32, 63, 64, 127, 128):
        if e < m and e < n:
            rows.append(e); cols.append(e)
    return np.array(rows, dtype=np.int64), np.array(cols, dtype=np.int64)


def check_sampled(p, A, B, C0, Cout, alpha, beta, transA=False, transB=False,
                  count=1024, seed=0, trials=3):
    """Compare Cout with the oracle on sampled entries and run Freivalds on
    the whole matrix.  Returns a description of the first failure or None."""
    m, n = Cout.shape
    rows, cols = sample_positions(m, n, count, seed)
    want = oracle.fgemm_entries(p, A, B, rows, cols, C0[rows, cols], alpha, beta,
                                transA, transB)
    got = Cout[rows, cols]
    bad = np.nonzero(got != want)[0]
    if bad.size:
        i = bad[0]
        return (f"{bad.size} sampled mismatches, first at ({rows[i]}, {cols[i]}): "
                f"got {got[i]} want {want[i]}")
    X = np.random.default_rng(seed + 1).integers(0, p, (trials, n), dtype=np.uint32)
    nbad = oracle.freivalds(p, A, B, C0, Cout, X, alpha, beta, transA, transB)
    if nbad:
        return f"Freivalds: {nbad} of {trials} trials disagree"
    return None
