"""Digit pairing on the GPU (7-bit digits, products of digit sums for the
cross terms) against the oracle, bit for bit.

Moduli give 2, 3, 4 and 5 digits; shapes span several 128 x 64 (64 x 64 at
five digits) tiles with ragged tails, with transposes and alpha/beta; K past
one int32 pass; the benchmark's 4096^3 product is compared whole in
test_gpu_parity.py, and five digits at p = 2^31 - 1 at 2048^3 here by
sampled entries and Freivalds.
"""
import itertools

import numpy as np
import pytest

import oracle
from gpu_util import check_sampled, from_dev, to_dev
from paper_cs_0601133_amd import ffgemm as ff
from paper_cs_0601133_amd import synth

pytestmark = pytest.mark.gpu

PAIR = dict(path=ff.FF_PATH_INT8, digit_pairing=1)


def run(p, A, B, C0, alpha, beta, transA=False, transB=False):
    dA, dB, dC = to_dev(A), to_dev(B), to_dev(C0)
    ff.fgemm(p, dA, dB, dC, alpha, beta, transA, transB, ff.make_opts(**PAIR))
    return from_dev(dC)


def inputs(p, m, n, k, seed, transA=False, transB=False):
    A = synth.residues(synth.seed_for(seed, 1), (k, m) if transA else (m, k), p)
    B = synth.residues(synth.seed_for(seed, 2), (n, k) if transB else (k, n), p)
    C = synth.residues(synth.seed_for(seed, 3), (m, n), p)
    return A, B, C


SHAPES = [(1, 1, 1), (3, 2, 5), (63, 65, 127), (129, 127, 300), (200, 33, 513),
          (300, 260, 700)]


@pytest.mark.parametrize("p,S", [(8191, 2), (65521, 3), (8388593, 4), (2147483647, 5)])
def test_pairing_matches_the_oracle(p, S):
    info = ff.ff_plan_query(p, 0, 0, 300, 260, 700, ff.make_opts(**PAIR))
    assert info.slices == S and info.digit_products == S * (S + 1) // 2
    for si, (m, n, k) in enumerate(SHAPES):
        for tA, tB in itertools.product((False, True), repeat=2):
            A, B, C = inputs(p, m, n, k, 1300 + 10 * S + si, tA, tB)
            alpha, beta = [(1, 0), (p - 1, 1), (3, p - 1)][(si + tA + 2 * tB) % 3]
            got = run(p, A, B, C, alpha, beta, tA, tB)
            want = oracle.fgemm(p, A, B, C, alpha, beta, tA, tB)
            assert np.array_equal(got, want), (p, m, n, k, tA, tB)


def test_pairing_extreme_values_and_long_k():
    # every entry p - 1 or (p - 1) / 2 (largest centered magnitudes), and K
    # past one int32 pass (65535 at four digits)
    p = 8388593
    for fill in (p - 1, (p - 1) // 2, (p + 1) // 2):
        A = np.full((70, 300), fill, np.uint32)
        B = np.full((300, 90), fill, np.uint32)
        got = run(p, A, B, np.zeros((70, 90), np.uint32), 1, 0)
        assert np.array_equal(got, oracle.fgemm(p, A, B, None, 1, 0)), fill
    k = 70000
    A, B, C = inputs(p, 9, 17, k, 1390)
    assert ff.ff_plan_query(p, 0, 0, 9, 17, k, ff.make_opts(**PAIR)).kblock < k
    assert np.array_equal(run(p, A, B, C, 5, 7), oracle.fgemm(p, A, B, C, 5, 7))


def test_pairing_five_digits_at_2048():
    p = 2147483647
    A, B, C = inputs(p, 2048, 2048, 2048, 1395)
    got = run(p, A, B, C, 3, 5)
    err = check_sampled(p, A, B, C, got, 3, 5, count=256, seed=1395)
    assert err is None, err
