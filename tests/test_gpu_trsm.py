"""Parity of the HIP triangular solve with the CPU oracle (bit-exact).

op(T) X = alpha B (mod p) has exactly one solution when T's diagonal is
invertible, so the comparison is element by element with the oracle's plain
substitution; at the full size, sampled entries of op(T) X are computed by
the oracle one by one and compared with alpha B.
"""
import itertools

import numpy as np
import pytest

import oracle
from gpu_util import from_dev, to_dev
from paper_cs_0601133_amd import ffgemm as ff
from paper_cs_0601133_amd import synth

pytestmark = pytest.mark.gpu


def tri(p, m, seed):
    """m x m residues with a nonzero diagonal (a unit for prime p); both
    triangles hold data, the solve must read only the one it is told."""
    T = synth.residues(synth.seed_for(seed, 1), (m, m), p)
    for i in range(m):
        T[i, i] = 1 + T[i, i] % (p - 1)
    return T


def solve_gpu(p, T, B, alpha, lower, trans, unit, **opts):
    dT, dB = to_dev(T), to_dev(B)
    ff.ftrsm(p, dT, dB, alpha, lower, trans, unit, opts=ff.make_opts(**opts))
    return from_dev(dB)


PRIMES = [7, 65521, 8388593, 2147483647]
SHAPES = [(1, 1), (5, 3), (64, 17), (65, 40), (130, 33), (300, 100)]


@pytest.mark.parametrize("lower,trans,unit", list(itertools.product((0, 1), repeat=3)))
@pytest.mark.parametrize("p", PRIMES)
def test_trsm_matches_oracle(p, lower, trans, unit):
    for si, (m, n) in enumerate(SHAPES):
        T = tri(p, m, 90 + si)
        B = synth.residues(synth.seed_for(91 + si, 2), (m, n), p)
        alpha = (3 + si) % p
        got = solve_gpu(p, T, B, alpha, lower, trans, unit)
        want = oracle.ftrsm(p, T, B, alpha, lower, trans, unit)
        assert np.array_equal(got, want), (m, n)


@pytest.mark.parametrize("path", [ff.FF_PATH_FP64, ff.FF_PATH_INT8], ids=["fp64", "int8"])
def test_trsm_update_paths(path):
    # the updates between diagonal blocks follow opts.path; m = 700 gives
    # several levels of the recursion and a ragged last block
    p, m, n = 8388593, 700, 90
    for lower in (0, 1):
        T = tri(p, m, 93 + lower)
        B = synth.residues(synth.seed_for(94, 2), (m, n), p)
        got = solve_gpu(p, T, B, 11, lower, 0, 0, path=path)
        assert np.array_equal(got, oracle.ftrsm(p, T, B, 11, lower)), lower


def test_trsm_quick_returns_and_leading_dimensions():
    import torch
    p, m, n = 65521, 50, 30
    T = tri(p, m, 95)
    B = synth.residues(synth.seed_for(96, 2), (m, n), p)
    # alpha = 0: X = 0
    assert not solve_gpu(p, T, B, 0, 0, 0, 0).any()
    # wider buffers: ldt = m + 7, ldb = n + 5; the padding is not touched
    Tw = np.zeros((m, m + 7), np.uint32); Tw[:, :m] = T
    Bw = np.full((m, n + 5), 9, np.uint32); Bw[:, :n] = B
    dT, dB = to_dev(Tw), to_dev(Bw)
    ff.ftrsm(p, dT[:, :m], dB[:, :n], 4, lower=True)
    got = from_dev(dB)
    assert np.array_equal(got[:, :n], oracle.ftrsm(p, T, B, 4, lower=True))
    assert np.all(got[:, n:] == 9)
    # m = 0 / n = 0: nothing happens
    assert ff.ff_ftrsm(p, 0, 0, 0, 0, n, 1, dT, m + 7, dB, n + 5) == ff.FF_OK
    torch.cuda.synchronize()


def test_trsm_validate_rejects_a_singular_diagonal():
    p, m, n = 7, 9, 4
    T = tri(p, m, 97)
    T[4, 4] = 0
    B = synth.residues(synth.seed_for(98, 2), (m, n), p)
    dT, dB = to_dev(T), to_dev(B)
    rc = ff.ff_ftrsm_ex(p, 0, 0, 0, m, n, 1, dT, m, dB, n, ff.make_opts(validate=1))
    assert rc == ff.FF_EINVAL
    assert np.array_equal(from_dev(dB), B)  # nothing written
    # unit diagonal: the stored zero is not read
    got = solve_gpu(p, T, B, 1, 0, 0, 1, validate=1)
    assert np.array_equal(got, oracle.ftrsm(p, T, B, 1, unit=True))
    # bad arguments
    assert ff.ff_ftrsm(p, 2, 0, 0, m, n, 1, dT, m, dB, n) == ff.FF_EINVAL
    assert ff.ff_ftrsm(p, 0, 0, 0, m, n, 1, dT, m - 1, dB, n) == ff.FF_EINVAL


@pytest.mark.parametrize("lower", [0, 1], ids=["upper", "lower"])
def test_trsm_full_size_sampled(lower):
    # m = n = 3000, p = 8388593: sampled entries of op(T) X against alpha B
    p, m, n, alpha = 8388593, 3000, 3000, 5
    T = tri(p, m, 99)
    B = synth.residues(synth.seed_for(100, 2), (m, n), p)
    X = solve_gpu(p, T, B, alpha, lower, 0, 0)
    Te = np.ascontiguousarray(np.tril(T) if lower else np.triu(T))
    rng = np.random.default_rng(11)
    rows, cols = rng.integers(0, m, 400), rng.integers(0, n, 400)
    lhs = oracle.fgemm_entries(p, Te, X, rows, cols)
    rhs = (alpha * B[rows, cols].astype(np.int64) % p).astype(np.uint32)
    assert np.array_equal(lhs, rhs)


@pytest.mark.parametrize("leaf", ["64", "192", "512"])
@pytest.mark.parametrize("p", [8388593, 2147483647], ids=["binary64", "split"])
def test_trsm_leaf_sizes(monkeypatch, p, leaf):
    # FF_TRSM_LEAF sets the rows per leaf launch (1 to 8 sub-blocks of 64);
    # m = 1100 leaves a ragged last sub-block in every leaf size
    monkeypatch.setenv("FF_TRSM_LEAF", leaf)
    m, n = 1100, 70
    for lower in (0, 1):
        T = tri(p, m, 101 + lower)
        B = synth.residues(synth.seed_for(102, 2), (m, n), p)
        got = solve_gpu(p, T, B, 7, lower, 1, 0)
        assert np.array_equal(got, oracle.ftrsm(p, T, B, 7, lower, trans=True)), lower


@pytest.mark.parametrize("p", [65521, 2147483647], ids=["binary64", "split"])
def test_trsm_single_block_read_in_place(p):
    # m <= 64: the inverse of the one diagonal block is formed straight from
    # op(T) (no normalised copy); T sits in a wider buffer (ldt = m + 3) and
    # is read transposed, upper and lower, unit and not
    m, n = 37, 50
    T = tri(p, m, 103)
    Tw = np.full((m, m + 3), p - 1, np.uint32); Tw[:, :m] = T
    B = synth.residues(synth.seed_for(104, 2), (m, n), p)
    for lower, unit in itertools.product((0, 1), (0, 1)):
        dT, dB = to_dev(Tw), to_dev(B)
        ff.ftrsm(p, dT[:, :m], dB, 6, lower, True, unit)
        want = oracle.ftrsm(p, T, B, 6, lower, True, unit)
        assert np.array_equal(from_dev(dB), want), (lower, unit)


@pytest.mark.parametrize("p", [7, 65521, 8388593])
def test_trsm_small_system_many_columns(p):
    # m <= 64 rows (one diagonal block) with many columns: several leaf
    # workgroups of columns (the last one ragged), B inside a wider buffer
    # (ldb = n + 5), every uplo/trans/diag and a non-trivial alpha
    for si, (m, n) in enumerate([(64, 700), (1, 300), (33, 257), (63, 1)]):
        T = tri(p, m, 110 + si)
        B = synth.residues(synth.seed_for(111 + si, 2), (m, n), p)
        for lower, trans, unit in itertools.product((0, 1), repeat=3):
            Bw = np.full((m, n + 5), p - 1, np.uint32); Bw[:, :n] = B
            dT, dB = to_dev(T), to_dev(Bw)
            ff.ftrsm(p, dT, dB[:, :n], (5 + si) % p, lower, trans, unit)
            got = from_dev(dB)
            want = oracle.ftrsm(p, T, B, (5 + si) % p, lower, trans, unit)
            assert np.array_equal(got[:, :n], want), (m, n, lower, trans, unit)
            assert np.all(got[:, n:] == p - 1), "wrote outside B"
