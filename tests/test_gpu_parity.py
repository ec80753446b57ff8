"""Parity of the HIP fgemm paths with the CPU oracle (bit-exact).

Every result is unique (reduction mod p is a ring homomorphism), so the
comparison is element by element with no tolerance: the full product where
the oracle is fast enough, and at the full workload sizes sampled entries
computed one by one plus Freivalds' random-vector check on all of C.
"""
import itertools

import numpy as np
import pytest

import oracle
from gpu_util import check_sampled, from_dev, to_dev
from paper_cs_0601133_amd import ffgemm as ff
from paper_cs_0601133_amd import synth

pytestmark = pytest.mark.gpu

FP64, INT8 = ff.FF_PATH_FP64, ff.FF_PATH_INT8


def run(p, A, B, C0, alpha, beta, transA=False, transB=False, **kw):
    dA, dB, dC = to_dev(A), to_dev(B), to_dev(C0)
    kw.setdefault("winograd_levels", 0)
    ff.fgemm(p, dA, dB, dC, alpha, beta, transA, transB, ff.make_opts(**kw))
    return from_dev(dC)


def inputs(p, m, n, k, seed, transA=False, transB=False):
    A = synth.residues(synth.seed_for(seed, 1), (k, m) if transA else (m, k), p)
    B = synth.residues(synth.seed_for(seed, 2), (n, k) if transB else (k, n), p)
    C = synth.residues(synth.seed_for(seed, 3), (m, n), p)
    return A, B, C


PATHS = [dict(path=FP64), dict(path=INT8, digit_bits=7), dict(path=INT8, digit_bits=8)]


@pytest.mark.parametrize("opts", PATHS, ids=["fp64", "int8d7", "int8d8"])
def test_small_config_full_oracle(opts):
    # m = n = k = 256, p = 65521, alpha = 1, beta = 0
    p = 65521
    A, B, C = inputs(p, 256, 256, 256, 1)
    got = run(p, A, B, C, 1, 0, **opts)
    want = oracle.fgemm(p, A, B, None, 1, 0)
    assert np.array_equal(got, want)


SHAPES = [(1, 1, 1), (2, 3, 1), (3, 2, 5), (63, 65, 127), (65, 63, 129), (127, 129, 65),
          (129, 127, 300), (200, 33, 513)]


@pytest.mark.parametrize("opts", PATHS, ids=["fp64", "int8d7", "int8d8"])
@pytest.mark.parametrize("p", [2, 3, 251, 65521, 8388593])
def test_edge_shapes(opts, p):
    for si, (m, n, k) in enumerate(SHAPES):
        for tA, tB in itertools.product((False, True), repeat=2):
            A, B, C = inputs(p, m, n, k, 100 + si, tA, tB)
            alpha, beta = [(1, 0), (p - 1, 1), (3 % p, (p - 1))][(si + tA + 2 * tB) % 3]
            got = run(p, A, B, C, alpha, beta, tA, tB, **opts)
            want = oracle.fgemm(p, A, B, C, alpha, beta, tA, tB)
            assert np.array_equal(got, want), (m, n, k, tA, tB, alpha, beta)


@pytest.mark.parametrize("opts", PATHS, ids=["fp64", "int8d7", "int8d8"])
def test_leading_dimensions_larger_than_rows(opts):
    import torch
    p = 8388593
    m, n, k = 70, 90, 150
    A, B, C = inputs(p, m, n, k, 7)
    # embed in wider buffers: lda = k + 13, ldb = n + 5, ldc = n + 9
    Aw = np.zeros((m, k + 13), np.uint32); Aw[:, :k] = A
    Bw = np.zeros((k, n + 5), np.uint32); Bw[:, :n] = B
    Cw = np.full((m, n + 9), 7, np.uint32); Cw[:, :n] = C
    dA, dB, dC = to_dev(Aw), to_dev(Bw), to_dev(Cw)
    ff.fgemm(p, dA[:, :k], dB[:, :n], dC[:, :n], 3, 5, opts=ff.make_opts(winograd_levels=0,
                                                                         **opts))
    got = from_dev(dC)
    want = oracle.fgemm(p, A, B, C, 3, 5)
    assert np.array_equal(got[:, :n], want)
    assert np.all(got[:, n:] == 7)  # padding untouched


@pytest.mark.parametrize("opts", PATHS, ids=["fp64", "int8d7", "int8d8"])
def test_quick_returns(opts):
    p = 65521
    A, B, C = inputs(p, 40, 30, 20, 9)
    # alpha = 0: C <- beta C
    got = run(p, A, B, C, 0, 7, **opts)
    assert np.array_equal(got, (7 * C.astype(np.int64) % p).astype(np.uint32))
    # beta = 0 with garbage in C: C is write-only
    garbage = np.full_like(C, 0xFFFFFFFF)
    got = run(p, A, B, garbage, 5, 0, **opts)
    assert np.array_equal(got, oracle.fgemm(p, A, B, None, 5, 0))
    # k = 0
    dC = to_dev(C)
    rc = ff.ff_fgemm_ex(p, 0, 0, 40, 30, 0, 1, to_dev(A), 20, to_dev(B), 30, 3, dC, 30,
                        ff.make_opts(winograd_levels=0, **opts))
    assert rc == ff.FF_OK
    assert np.array_equal(from_dev(dC), (3 * C.astype(np.int64) % p).astype(np.uint32))


def test_fp64_folds_every_kblock():
    # p = 8388593: the FP64 path reduces every 512 products; k = 1500 crosses
    # two reductions and a ragged tail
    p = 8388593
    A, B, C = inputs(p, 96, 80, 1500, 11)
    got = run(p, A, B, C, 3, 5, path=FP64)
    assert np.array_equal(got, oracle.fgemm(p, A, B, C, 3, 5))


@pytest.mark.parametrize("p", [33554393, 47499979, 94906249])
def test_fp64_large_moduli_reduction_schedule(p):
    # K-blocks 32 (a reduction every two K stages), 15 and 4 (a reduction
    # after every matrix-core step): random operands, then every product at
    # the largest magnitude with one sign, where a late reduction overflows
    # 2^53 and loses exactness
    A, B, C = inputs(p, 130, 150, 700, 13)
    got = run(p, A, B, C, 3, 5, path=FP64)
    assert np.array_equal(got, oracle.fgemm(p, A, B, C, 3, 5))
    m, n, k = 64, 80, 1000
    A = np.full((m, k), p // 2, np.uint32)          # centered (p - 1)/2
    B = np.full((k, n), (p + 1) // 2, np.uint32)    # centered -(p - 1)/2
    got = run(p, A, B, np.zeros((m, n), np.uint32), 1, 0, path=FP64)
    assert np.array_equal(got, oracle.fgemm(p, A, B, None, 1, 0))


@pytest.mark.parametrize("p,opts", [(2147483647, dict(path=INT8, digit_bits=7)),
                                     (2147483629, dict(path=INT8, digit_bits=8)),
                                     (94906249, dict(path=FP64)),
                                     (3, dict(path=FP64)), (2, dict(path=INT8, digit_bits=7))],
                         ids=["p2^31-1-int8d7", "p2147483629-int8d8", "p94906249-fp64",
                              "p3-fp64", "p2-int8d7"])
def test_epilogue_products_at_the_largest_residues(p, opts):
    # alpha, beta and C near p - 1: the epilogue's products mod p (alpha*r,
    # beta*c) at their largest operands; then every residue p - 1
    m, n, k = 70, 130, 190
    A, B, C = inputs(p, m, n, k, 14)
    alpha, beta = (p - 2) % p, (p - 3) % p
    got = run(p, A, B, C, alpha, beta, **opts)
    assert np.array_equal(got, oracle.fgemm(p, A, B, C, alpha, beta))
    full = np.full((m, k), p - 1, np.uint32), np.full((k, n), p - 1, np.uint32)
    Cf = np.full((m, n), p - 1, np.uint32)
    got = run(p, full[0], full[1], Cf, p - 1, p - 1, **opts)
    assert np.array_equal(got, oracle.fgemm(p, full[0], full[1], Cf, p - 1, p - 1))


@pytest.mark.parametrize("opts", PATHS, ids=["fp64", "int8d7", "int8d8"])
def test_long_k_tiny_output(opts):
    # k = 1000003 with a 3 x 5 output: FP64 splits K 512 ways with
    # reductions inside every split; INT8 runs 8 (7-bit) or 23 (8-bit)
    # int32 K-passes chained with beta = 1
    p = 8388593
    A, B, C = inputs(p, 3, 5, 1000003, 15)
    got = run(p, A, B, C, 7, 11, **opts)
    assert np.array_equal(got, oracle.fgemm(p, A, B, C, 7, 11))


def test_int8_k_split_beyond_int32_block():
    # p = 251 direct plane: one int32 pass is exact up to k = 137438, so
    # k = 140000 takes two passes chained with beta = 1
    p = 251
    A, B, C = inputs(p, 64, 48, 140000, 12)
    got = run(p, A, B, C, 2, 3, path=INT8)
    assert np.array_equal(got, oracle.fgemm(p, A, B, C, 2, 3))


def test_extreme_values():
    # all entries at the ends of the centered range: the accumulation bound
    # is reached with equality in sign
    for p in (65521, 8388593, 2147483647):
        m = n = 64
        k = 2048
        A = np.full((m, k), p // 2, np.uint32)            # most positive
        B = np.full((k, n), (p + 1) // 2, np.uint32)      # most negative
        for opts in ([dict(path=FP64)] if p < (1 << 24) else []) + \
                [dict(path=INT8, digit_bits=7), dict(path=INT8, digit_bits=8)]:
            try:
                got = run(p, A, B, np.zeros((m, n), np.uint32), 1, 0, **opts)
            except ff.FFError as e:
                assert e.status == ff.FF_EUNSUPPORTED
                continue
            want = oracle.fgemm(p, A, B, None, 1, 0)
            assert np.array_equal(got, want), (p, opts)


def test_validate_rejects_out_of_range():
    p = 251
    A, B, C = inputs(p, 16, 16, 16, 13)
    A[3, 4] = 251
    dA, dB, dC = to_dev(A), to_dev(B), to_dev(C)
    before = from_dev(dC).copy()
    with pytest.raises(ff.FFError) as e:
        ff.fgemm(p, dA, dB, dC, 1, 1, opts=ff.make_opts(validate=1, winograd_levels=0))
    assert e.value.status == ff.FF_EINVAL
    assert np.array_equal(from_dev(dC), before)


def test_deterministic_and_paths_agree():
    p = 8388593
    A, B, C = inputs(p, 300, 260, 700, 14)
    outs = [run(p, A, B, C, 3, 5, **o) for o in PATHS + PATHS]
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])
    assert np.array_equal(outs[0], oracle.fgemm(p, A, B, C, 3, 5))


_FULL_4096 = {}


def _full_4096():
    """Inputs of the 4096^3 workload and the oracle's whole product, computed
    once per session."""
    if not _FULL_4096:
        p = 8388593
        A, B, C = inputs(p, 4096, 4096, 4096, 2)
        _FULL_4096["args"] = (p, A, B, C)
        _FULL_4096["want"] = oracle.fgemm(p, A, B, C, 3, 5)
    return _FULL_4096["args"], _FULL_4096["want"]


@pytest.mark.parametrize("opts", PATHS + [dict(path=INT8, digit_bits=7, winograd_levels=1),
                                          dict(path=INT8, digit_pairing=1)],
                         ids=["fp64", "int8d7", "int8d8", "int8d7_winograd1", "int8d7_pairing"])
def test_full_size_4096(opts):
    # m = n = k = 4096, p = 8388593, alpha = 3, beta = 5 (the benchmark's
    # workload and launch configuration): every entry against the oracle
    (p, A, B, C), want = _full_4096()
    got = run(p, A, B, C, 3, 5, **opts)
    bad = np.argwhere(got != want)
    assert bad.size == 0, f"{len(bad)} entries differ, first at {tuple(bad[0])}"


def test_full_size_8192_p251():
    # m = n = k = 8192, p = 251, one direct int8 plane
    p = 251
    A, B, _ = inputs(p, 8192, 8192, 8192, 3)
    C = np.zeros((8192, 8192), np.uint32)
    got = run(p, A, B, C, 1, 0, path=INT8)
    err = check_sampled(p, A, B, C, got, 1, 0, count=256, seed=3, trials=2)
    assert err is None, err
