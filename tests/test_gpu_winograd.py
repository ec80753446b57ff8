"""Winograd levels (Section 3.2) on both paths: bit-exact vs the oracle.

Covers 1 and 2 levels, delayed (unreduced) and reduced pre-additions,
dimensions that are not multiples of 2^l (peeling), alpha/beta and
transposes, the last pre-addition level fused into the digit slicing (INT8)
or the binary64 packing (FP64) of the leaves (the default) and kept apart
(FF_WINO_FUSED=0), and the 8192^3 product at p = 8388593 (sampled +
Freivalds).
"""
import numpy as np
import pytest

import oracle
from gpu_util import check_sampled, from_dev, to_dev
from paper_cs_0601133_amd import ffgemm as ff
from paper_cs_0601133_amd import synth

pytestmark = pytest.mark.gpu

CASES = [
    (8388593, 256, 256, 256, 1), (8388593, 320, 288, 352, 2), (65521, 257, 301, 263, 1),
    (65521, 130, 190, 517, 2), (251, 96, 64, 128, 2), (2147483647, 128, 128, 128, 1),
]


@pytest.mark.parametrize("path,bits,fused", [(ff.FF_PATH_INT8, 7, "1"), (ff.FF_PATH_INT8, 8, "1"),
                                             (ff.FF_PATH_INT8, 7, "0"), (ff.FF_PATH_INT8, 8, "0"),
                                             (ff.FF_PATH_FP64, 0, "1"), (ff.FF_PATH_FP64, 0, "0")],
                         ids=["int8d7", "int8d8", "int8d7_apart", "int8d8_apart", "fp64",
                              "fp64_apart"])
@pytest.mark.parametrize("mode", [1, 2], ids=["delayed", "reduced"])
def test_winograd_levels(path, bits, fused, mode, monkeypatch):
    monkeypatch.setenv("FF_WINO_FUSED", fused)
    for ci, (p, m, n, k, L) in enumerate(CASES):
        tA, tB = bool(ci & 1), bool(ci & 2)
        A = synth.residues(synth.seed_for(60 + ci, 1), (k, m) if tA else (m, k), p)
        B = synth.residues(synth.seed_for(60 + ci, 2), (n, k) if tB else (k, n), p)
        C = synth.residues(synth.seed_for(60 + ci, 3), (m, n), p)
        o = ff.make_opts(path=path, digit_bits=bits, winograd_levels=L, preadd_mode=mode)
        try:
            info = ff.ff_plan_query(p, int(tA), int(tB), m, n, k, o)
        except ff.FFError as e:
            assert e.status == ff.FF_EUNSUPPORTED
            continue
        assert info.winograd_levels == L
        dA, dB, dC = to_dev(A), to_dev(B), to_dev(C)
        ff.fgemm(p, dA, dB, dC, 3, 5, tA, tB, opts=o)
        want = oracle.fgemm(p, A, B, C, 3, 5, tA, tB)
        assert np.array_equal(from_dev(dC), want), (p, m, n, k, L, tA, tB)


@pytest.mark.parametrize("L", [1, 2])
@pytest.mark.parametrize("path,bits", [(ff.FF_PATH_INT8, 7), (ff.FF_PATH_INT8, 8),
                                       (ff.FF_PATH_FP64, 0)], ids=["int8d7", "int8d8", "fp64"])
def test_winograd_full_size_8192(L, path, bits):
    p = 8388593
    A = synth.residues(synth.seed_for(3, 1), (8192, 8192), p)
    B = synth.residues(synth.seed_for(3, 2), (8192, 8192), p)
    C = np.zeros((8192, 8192), np.uint32)
    dA, dB, dC = to_dev(A), to_dev(B), to_dev(C)
    ff.fgemm(p, dA, dB, dC, 1, 0, opts=ff.make_opts(path=path, digit_bits=bits,
                                                    winograd_levels=L))
    err = check_sampled(p, A, B, C, from_dev(dC), 1, 0, count=256, seed=L, trials=2)
    assert err is None, err


def test_winograd_rows_beyond_one_launch():
    # FP64 leaves with two levels at m = 131076: the first level's
    # pre-additions (65538 quadrant rows) and both levels' post-additions
    # (32769 and 65538 rows) are split into launches of at most 32768 rows
    # (the grid's y extent); 131077 rows also peel a last row
    for m in (131076, 131077):
        p, n, k = 65521, 64, 64
        A = synth.residues(synth.seed_for(80, 1), (m, k), p)
        B = synth.residues(synth.seed_for(80, 2), (k, n), p)
        C = synth.residues(synth.seed_for(80, 3), (m, n), p)
        o = ff.make_opts(path=ff.FF_PATH_FP64, winograd_levels=2)
        assert ff.ff_plan_query(p, 0, 0, m, n, k, o).winograd_levels == 2
        dA, dB, dC = to_dev(A), to_dev(B), to_dev(C)
        ff.fgemm(p, dA, dB, dC, 2, 7, opts=o)
        want = oracle.fgemm(p, A, B, C, 2, 7)
        assert np.array_equal(from_dev(dC), want), m


@pytest.mark.parametrize("path,bits,fused", [(ff.FF_PATH_INT8, 7, "1"), (ff.FF_PATH_INT8, 8, "1"),
                                             (ff.FF_PATH_INT8, 8, "0"), (ff.FF_PATH_FP64, 0, "1"),
                                             (ff.FF_PATH_FP64, 0, "0")],
                         ids=["int8d7", "int8d8", "int8d8_apart", "fp64", "fp64_apart"])
def test_winograd_three_levels(path, bits, fused, monkeypatch):
    # three levels: the two stored levels of pre-additions alternate between
    # the workspace's buffers without a level writing the one it reads (the
    # fused path stores levels 1 and 2, the unfused one all three); odd
    # sizes peel at every dimension, leaves stay >= 16
    monkeypatch.setenv("FF_WINO_FUSED", fused)
    for ci, (p, m, n, k) in enumerate([(8388593, 256, 256, 256), (65521, 300, 270, 333),
                                       (251, 136, 200, 168)]):
        tA, tB = bool(ci & 1), bool(ci & 2)
        A = synth.residues(synth.seed_for(70 + ci, 1), (k, m) if tA else (m, k), p)
        B = synth.residues(synth.seed_for(70 + ci, 2), (n, k) if tB else (k, n), p)
        C = synth.residues(synth.seed_for(70 + ci, 3), (m, n), p)
        o = ff.make_opts(path=path, digit_bits=bits, winograd_levels=3)
        try:
            info = ff.ff_plan_query(p, int(tA), int(tB), m, n, k, o)
        except ff.FFError as e:
            assert e.status == ff.FF_EUNSUPPORTED
            continue
        assert info.winograd_levels == 3
        dA, dB, dC = to_dev(A), to_dev(B), to_dev(C)
        ff.fgemm(p, dA, dB, dC, 6, 2, tA, tB, opts=o)
        want = oracle.fgemm(p, A, B, C, 6, 2, tA, tB)
        assert np.array_equal(from_dev(dC), want), (p, m, n, k, tA, tB)
