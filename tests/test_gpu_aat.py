"""Parity of the HIP symmetric product alpha A diag(D) A^T + beta C
(Section 6) with the CPU oracle, bit-exact.  The result is unique, so the
whole output is compared element by element; at 4096 (the benchmark's
configuration) sampled entries of the lower triangle are computed by the
oracle one by one and the whole output must be symmetric."""
import numpy as np
import pytest

import oracle
from gpu_util import from_dev, to_dev
from paper_cs_0601133_amd import ffgemm as ff
from paper_cs_0601133_amd import synth

pytestmark = pytest.mark.gpu


def gpu_aat(p, A, d, alpha, beta, C, **opts):
    dA, dC = to_dev(A), to_dev(C)
    dD = to_dev(d) if d is not None else None
    ff.aat(p, dA, dC, dD, alpha, beta, opts=ff.make_opts(**opts))
    return from_dev(dC)


@pytest.mark.parametrize("p", [2, 251, 65521, 8388593, 2147483647])
def test_matches_the_oracle(p):
    for si, (m, k) in enumerate([(1, 1), (5, 3), (64, 64), (129, 70), (300, 500), (513, 100)]):
        A = synth.residues(synth.seed_for(200 + si, 1), (m, k), p)
        d = synth.residues(synth.seed_for(200 + si, 2), (k,), p)
        C = synth.residues(synth.seed_for(200 + si, 3), (m, m), p)
        for dd, alpha, beta in ((None, 1, 0), (d, 3 % p, (p - 1) % p)):
            got = gpu_aat(p, A, dd, alpha, beta, C)
            want = oracle.aat(p, A, dd, alpha, beta, C)
            assert np.array_equal(got, want), (m, k, dd is None)


@pytest.mark.parametrize("path", [ff.FF_PATH_FP64, ff.FF_PATH_INT8], ids=["fp64", "int8"])
def test_paths(path):
    p, m, k = 8388593, 700, 300
    A = synth.residues(synth.seed_for(210, 1), (m, k), p)
    d = synth.residues(synth.seed_for(210, 2), (k,), p)
    d[::7] = 0
    C = synth.residues(synth.seed_for(210, 3), (m, m), p)
    for dd in (None, d):
        got = gpu_aat(p, A, dd, 5, 2, C, path=path)
        assert np.array_equal(got, oracle.aat(p, A, dd, 5, 2, C))


def test_long_k_runs_block_rows_as_separate_products():
    # k past one int32 pass of the INT8 path (43690 for 3 8-bit digits)
    p, m, k = 8388593, 40, 44000
    A = synth.residues(synth.seed_for(211, 1), (m, k), p)
    C = np.zeros((m, m), np.uint32)
    got = gpu_aat(p, A, None, 1, 0, C, path=ff.FF_PATH_INT8)
    assert np.array_equal(got, oracle.aat(p, A))


def test_quick_returns_and_upper_triangle_ignored():
    p, m, k = 65521, 90, 40
    A = synth.residues(synth.seed_for(212, 1), (m, k), p)
    C = synth.residues(synth.seed_for(212, 3), (m, m), p)
    # alpha = 0 and k = 0: C <- beta C on the lower triangle, mirrored
    want = oracle.aat(p, A, None, 0, 7, C)
    assert np.array_equal(gpu_aat(p, A, None, 0, 7, C), want)
    Z = np.zeros((m, 0), np.uint32)
    dC = to_dev(C)
    assert ff.ff_faat(p, m, 0, 1, 0, 1, None, 7, dC, m) == ff.FF_OK
    assert np.array_equal(from_dev(dC), want)
    # the strict upper triangle of C on entry does not change the result
    C2 = C.copy()
    C2[np.triu_indices(m, 1)] = 1
    assert np.array_equal(gpu_aat(p, A, None, 2, 3, C2), gpu_aat(p, A, None, 2, 3, C))
    # bad arguments
    assert ff.ff_faat(p, m, k, 1, to_dev(A), k - 1, None, 0, dC, m) == ff.FF_EINVAL
    assert ff.ff_faat(p, m, k, 1, to_dev(A), k, None, 0, dC, m - 1) == ff.FF_EINVAL


def test_full_size_sampled():
    # m = k = 4096, p = 8388593, D given: the benchmark's configuration
    p, m, k = 8388593, 4096, 4096
    A = synth.residues(synth.seed_for(213, 1), (m, k), p)
    d = synth.residues(synth.seed_for(213, 2), (k,), p)
    C = np.zeros((m, m), np.uint32)
    got = gpu_aat(p, A, d, 1, 0, C)
    assert np.array_equal(got, got.T)
    AD = (A.astype(np.uint64) * d.astype(np.uint64)[None, :] % p).astype(np.uint32)
    rng = np.random.default_rng(9)
    rows = rng.integers(0, m, 500)
    cols = (rng.random(500) * (rows + 1)).astype(np.int64)  # lower triangle
    want = oracle.fgemm_entries(p, A, AD, rows, cols, transB=True)
    assert np.array_equal(got[rows, cols], want)
