"""The one-launch FP64 kernel for small products, bit-exact vs the oracle.

The kernel reads the residues in place (all four transpose combinations),
centers them on the way into LDS, delays the reduction by the plan's
K-block (folds every 2 steps at p = 2^26 - 5, never at p = 65521 for these
depths) and applies alpha and beta in the epilogue.  Ragged shapes cover
partial 32 x 32 tiles and partial 64-deep K stages.  The general FP64 path
(packing, K split, split reduction) is checked on the same shapes with
FF_F64_SMALL=0, and both paths must agree.
"""
import numpy as np
import pytest

import oracle
from gpu_util import from_dev, to_dev
from paper_cs_0601133_amd import ffgemm as ff
from paper_cs_0601133_amd import synth

pytestmark = pytest.mark.gpu

SHAPES = [(1, 1, 1), (31, 33, 65), (32, 32, 64), (256, 256, 256), (300, 200, 2048),
          (5, 700, 130), (512, 512, 67)]
PRIMES = [2, 3, 251, 65521, 8388593, 67108859]


def run(p, A, B, C, alpha, beta, tA, tB):
    dA, dB, dC = to_dev(A), to_dev(B), to_dev(C)
    ff.fgemm(p, dA, dB, dC, alpha, beta, tA, tB,
             ff.make_opts(path=ff.FF_PATH_FP64, winograd_levels=0))
    return from_dev(dC)


@pytest.mark.parametrize("mode", ["1", "0"], ids=["one_launch", "general"])
def test_small_fp64_products(mode, monkeypatch):
    monkeypatch.setenv("FF_F64_SMALL", mode)
    for si, (m, n, k) in enumerate(SHAPES):
        for pi, p in enumerate(PRIMES):
            tA, tB = bool((si + pi) & 1), bool((si + pi) & 2)
            seed = 900 + 10 * si + pi
            A = synth.residues(synth.seed_for(seed, 1), (k, m) if tA else (m, k), p)
            B = synth.residues(synth.seed_for(seed, 2), (n, k) if tB else (k, n), p)
            C = synth.residues(synth.seed_for(seed, 3), (m, n), p)
            alpha, beta = (p - 1) % p, 3 % p
            got = run(p, A, B, C, alpha, beta, tA, tB)
            want = oracle.fgemm(p, A, B, C, alpha, beta, tA, tB)
            assert np.array_equal(got, want), (mode, m, n, k, p, tA, tB)


def test_small_fp64_beta_zero_and_extreme_residues(monkeypatch):
    # all entries p - 1 (centered -1) and (p - 1) / 2 (the largest centered
    # value): the K-block bound is met with equality patterns; beta = 0
    # must not read C (filled with values >= p here)
    monkeypatch.setenv("FF_F64_SMALL", "1")
    for p in (8388593, 67108859):
        for fill in (p - 1, (p - 1) // 2):
            m, n, k = 64, 96, 2048
            A = np.full((m, k), fill, np.uint32)
            B = np.full((k, n), fill, np.uint32)
            C = np.full((m, n), 0xFFFFFFFF, np.uint32)
            got = run(p, A, B, C, 1, 0, False, False)
            want = oracle.fgemm(p, A, B, np.zeros((m, n), np.uint32), 1, 0, False, False)
            assert np.array_equal(got, want), (p, fill)


@pytest.mark.parametrize("mode", ["1", "0"], ids=["one_launch", "general"])
def test_small_fp64_transposed_views_in_wider_buffers(mode, monkeypatch):
    # op(A) = A^T and op(B) = B^T read from column-sliced views of wider
    # buffers (lda = m + 11, ldb = k + 3, ldc = n + 6); the padding of C is
    # not touched
    monkeypatch.setenv("FF_F64_SMALL", mode)
    p, m, n, k = 65521, 45, 70, 133
    A = synth.residues(synth.seed_for(950, 1), (k, m), p)  # op(A) = A^T is m x k
    B = synth.residues(synth.seed_for(950, 2), (n, k), p)
    C = synth.residues(synth.seed_for(950, 3), (m, n), p)
    Aw = np.zeros((k, m + 11), np.uint32); Aw[:, :m] = A
    Bw = np.zeros((n, k + 3), np.uint32); Bw[:, :k] = B
    Cw = np.full((m, n + 6), 5, np.uint32); Cw[:, :n] = C
    dA, dB, dC = to_dev(Aw), to_dev(Bw), to_dev(Cw)
    ff.fgemm(p, dA[:, :m], dB[:, :k], dC[:, :n], 9, 4, True, True,
             ff.make_opts(path=ff.FF_PATH_FP64, winograd_levels=0))
    got = from_dev(dC)
    assert np.array_equal(got[:, :n], oracle.fgemm(p, A, B, C, 9, 4, True, True))
    assert np.all(got[:, n:] == 5)


@pytest.mark.parametrize("mode", ["1", "0"], ids=["one_launch", "general"])
def test_small_fp64_fold_after_every_step(mode, monkeypatch):
    # p = 89999999: (p/2)^2 > 2^50, so the FP64 K-block holds 4..7 products
    # and the accumulators are reduced after every 4-product matrix-core step
    monkeypatch.setenv("FF_F64_SMALL", mode)
    p = 89999999
    o = ff.make_opts(path=ff.FF_PATH_FP64, winograd_levels=0)
    assert 4 <= ff.ff_plan_query(p, 0, 0, 64, 64, 64, o).kblock < 8
    for si, (m, n, k) in enumerate([(31, 33, 65), (256, 256, 256), (70, 40, 700)]):
        A = synth.residues(synth.seed_for(960 + si, 1), (m, k), p)
        B = synth.residues(synth.seed_for(960 + si, 2), (k, n), p)
        C = synth.residues(synth.seed_for(960 + si, 3), (m, n), p)
        got = run(p, A, B, C, 5, 3, False, False)
        assert np.array_equal(got, oracle.fgemm(p, A, B, C, 5, 3)), (m, n, k)
