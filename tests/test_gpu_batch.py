"""Batched persistent launches, HIP graphs and the multi-modular workload.

A multi-modular product: one integer matrix pair with entries uniform in
[-2^30, 2^30] is reduced modulo many primes just below 2^20 (host-side input
preparation), all the modular products run as one batch, every job is
checked against the oracle, and Chinese remaindering of the residues gives
back the exact integer product computed by the oracle in 128-bit integers.
"""
import numpy as np
import pytest

import oracle
from gpu_util import from_dev, to_dev
from paper_cs_0601133_amd import ffgemm as ff
from paper_cs_0601133_amd import synth

pytestmark = pytest.mark.gpu


def reduce_mod(X, p):
    return np.mod(X, p).astype(np.uint32)


def multimodular(n_max, sizes, nprimes, seed):
    A = synth.signed_ints(synth.seed_for(seed, 1), (n_max, n_max), 1 << 30)
    B = synth.signed_ints(synth.seed_for(seed, 2), (n_max, n_max), 1 << 30)
    primes = synth.primes_below(1 << 20, nprimes)
    # balanced assignment of sizes to primes, seeded shuffle
    order = np.random.default_rng(seed).permutation(nprimes)
    jobs = []
    for idx, pi in enumerate(order):
        n = sizes[idx % len(sizes)]
        jobs.append((primes[pi], n))
    return A, B, jobs


@pytest.mark.parametrize("path", [ff.FF_PATH_INT8, ff.FF_PATH_FP64], ids=["int8", "fp64"])
def test_multimodular_batch_small(path):
    A, B, jobs = multimodular(256, [64, 128, 192, 256], 16, 40)
    dev = []
    abi = []
    for (p, n) in jobs:
        Ap = reduce_mod(A[:n, :n], p)
        Bp = reduce_mod(B[:n, :n], p)
        dA, dB = to_dev(Ap), to_dev(Bp)
        dC = to_dev(np.zeros((n, n), np.uint32))
        dev.append((p, n, Ap, Bp, dA, dB, dC))
        abi.append(ff.job(p, dA, dB, dC))
    ff.ff_set_stream(None)
    import torch
    torch.cuda.synchronize()
    rc = ff.ff_fgemm_batched(abi, ff.make_opts(path=path))
    assert rc == ff.FF_OK, ff.ff_last_error()
    results = {}
    for (p, n, Ap, Bp, dA, dB, dC) in dev:
        got = from_dev(dC)
        assert np.array_equal(got, oracle.fgemm(p, Ap, Bp)), (p, n)
        results.setdefault(n, []).append((p, got))
    # Chinese remaindering per size vs the exact integer product
    for n, lst in results.items():
        primes = [p for p, _ in lst[:4]]
        lo, hi = oracle.crt(primes, [g for _, g in lst[:4]])
        elo, ehi = oracle.int_matmul(A[:n, :n], B[:n, :n])
        assert np.array_equal(lo, elo) and np.array_equal(hi, ehi), n


def test_batch_mixed_moduli_transposes_and_quick_jobs():
    # different slice counts in one launch (p = 251, 65521, 8388593), beta,
    # transposes, a k = 0 job and an alpha = 0 job
    rng_seed = 50
    specs = [(251, 70, 90, 33, 1, 0, False, False), (65521, 128, 64, 200, 3, 5, True, False),
             (8388593, 100, 130, 257, 7, 1, False, True), (8388593, 64, 64, 0, 1, 2, False, False),
             (65521, 40, 50, 60, 0, 9, False, False), (2, 33, 17, 129, 1, 1, True, True)]
    items = []
    for i, (p, m, n, k, al, be, tA, tB) in enumerate(specs):
        Ap = synth.residues(synth.seed_for(rng_seed + i, 1), (k, m) if tA else (m, k), p)
        Bp = synth.residues(synth.seed_for(rng_seed + i, 2), (n, k) if tB else (k, n), p)
        Cp = synth.residues(synth.seed_for(rng_seed + i, 3), (m, n), p)
        dA, dB, dC = to_dev(Ap), to_dev(Bp), to_dev(Cp)
        items.append((p, Ap, Bp, Cp, al, be, tA, tB, dA, dB, dC, k))
    abi = []
    for (p, Ap, Bp, Cp, al, be, tA, tB, dA, dB, dC, k) in items:
        j = ff.job(p, dA, dB, dC, al, be, tA, tB)
        if k == 0:
            j.k = 0
        abi.append(j)
    for path in (ff.FF_PATH_INT8, ff.FF_PATH_FP64):
        for it, j in zip(items, abi):
            it[10].copy_(to_dev(it[3]))
        rc = ff.ff_fgemm_batched(abi, ff.make_opts(path=path))
        assert rc == ff.FF_OK, ff.ff_last_error()
        for (p, Ap, Bp, Cp, al, be, tA, tB, dA, dB, dC, k) in items:
            if k == 0:
                want = (be * Cp.astype(np.int64) % p).astype(np.uint32)
            else:
                want = oracle.fgemm(p, Ap, Bp, Cp, al, be, tA, tB)
            assert np.array_equal(from_dev(dC), want), (path, p)


def test_fp64_batch_mixes_reduction_schedules():
    # FP64 jobs reduced every few K stages and jobs reduced after every
    # matrix-core step (p above about 4.7e7) run as two persistent launches
    specs = [(65521, 96, 80, 300, False, False), (94906249, 70, 130, 257, True, False),
             (8388593, 129, 65, 1100, False, True), (47499979, 33, 200, 64, True, True),
             (33554393, 256, 256, 640, False, False), (94906249, 1, 1, 1, False, False)]
    items, abi = [], []
    for i, (p, m, n, k, tA, tB) in enumerate(specs):
        Ap = synth.residues(synth.seed_for(60 + i, 1), (k, m) if tA else (m, k), p)
        Bp = synth.residues(synth.seed_for(60 + i, 2), (n, k) if tB else (k, n), p)
        Cp = synth.residues(synth.seed_for(60 + i, 3), (m, n), p)
        dA, dB, dC = to_dev(Ap), to_dev(Bp), to_dev(Cp)
        items.append((p, Ap, Bp, Cp, tA, tB, dA, dB, dC))
        abi.append(ff.job(p, dA, dB, dC, 5, 7, tA, tB))
    rc = ff.ff_fgemm_batched(abi, ff.make_opts(path=ff.FF_PATH_FP64))
    assert rc == ff.FF_OK, ff.ff_last_error()
    for (p, Ap, Bp, Cp, tA, tB, dA, dB, dC) in items:
        want = oracle.fgemm(p, Ap, Bp, Cp, 5, 7, tA, tB)
        assert np.array_equal(from_dev(dC), want), p


@pytest.mark.parametrize("path", [ff.FF_PATH_INT8, ff.FF_PATH_FP64], ids=["int8", "fp64"])
def test_batch_graph_replays(path):
    import torch
    A, B, jobs = multimodular(192, [64, 128, 192], 6, 41)
    dev, abi, keep = [], [], []
    for (p, n) in jobs:
        Ap, Bp = reduce_mod(A[:n, :n], p), reduce_mod(B[:n, :n], p)
        dA, dB = to_dev(Ap), to_dev(Bp)
        dC = to_dev(np.zeros((n, n), np.uint32))
        keep.append((dA, dB))  # the graph reads these: keep them alive
        dev.append((p, Ap, Bp, dC))
        abi.append(ff.job(p, dA, dB, dC, 3, 0))
    wants = [oracle.fgemm(p, Ap, Bp, None, 3, 0) for (p, Ap, Bp, _) in dev]
    g = ff.ff_batch_graph_create(abi, ff.make_opts(path=path))
    try:
        stream = torch.cuda.current_stream()
        for replay in range(4):
            for (_, _, _, dC) in dev:          # eager work between replays
                dC.fill_(-1)
            torch.cuda.synchronize()
            ff.ff_batch_graph_launch(g, stream.cuda_stream)
            torch.cuda.synchronize()
            for (p, Ap, Bp, dC), want in zip(dev, wants):
                assert np.array_equal(from_dev(dC), want), (replay, p)
    finally:
        ff.ff_batch_graph_destroy(g)


@pytest.mark.parametrize("path", [ff.FF_PATH_INT8, ff.FF_PATH_FP64], ids=["int8", "fp64"])
def test_multimodular_full_size_crt(path):
    # 64 jobs of n in {512, 1024, 1536, 2048}, the 64 largest primes below
    # 2^20, one persistent launch; Chinese remaindering of 4 primes per size
    # on a sample of entries vs the exact 128-bit product of those entries
    import torch
    A, B, jobs = multimodular(2048, [512, 1024, 1536, 2048], 64, 42)
    dev, abi, keep = [], [], []
    for (p, n) in jobs:
        Ap, Bp = reduce_mod(A[:n, :n], p), reduce_mod(B[:n, :n], p)
        dA, dB = to_dev(Ap), to_dev(Bp)
        dC = to_dev(np.zeros((n, n), np.uint32))
        keep.append((dA, dB))  # device operands must outlive the launch
        dev.append((p, n, Ap, Bp, dC))
        abi.append(ff.job(p, dA, dB, dC))
    torch.cuda.synchronize()
    assert ff.ff_fgemm_batched(abi, ff.make_opts(path=path)) == ff.FF_OK
    rng = np.random.default_rng(7)
    by_size = {}
    for (p, n, Ap, Bp, dC) in dev:
        by_size.setdefault(n, []).append((p, Ap, Bp, from_dev(dC)))
    for n, lst in by_size.items():
        rows = rng.integers(0, n, 24)
        cols = rng.integers(0, n, 24)
        elo, ehi = oracle.int_matmul(A[rows, :n], B[:n, cols])
        primes = [p for p, _, _, _ in lst[:4]]
        res = [got[np.ix_(rows, cols)] for _, _, _, got in lst[:4]]
        lo, hi = oracle.crt(primes, res)
        assert np.array_equal(lo, elo) and np.array_equal(hi, ehi), n
        # every job: sampled entries vs the oracle
        for p, Ap, Bp, got in lst:
            r2, c2 = rng.integers(0, n, 64), rng.integers(0, n, 64)
            want = oracle.fgemm_entries(p, Ap, Bp, r2, c2)
            assert np.array_equal(got[r2, c2], want), (n, p)


def test_multimodular_full_size_graph_replays():
    # The 64-job configuration as one captured persistent launch, replayed
    # three times with eager work in between: after every replay, Chinese
    # remaindering of 4 primes per size on sampled entries against the exact
    # integer product, sampled entries of every job, and (first replay) the
    # whole output of one job per size against the oracle.
    import torch
    A, B, jobs = multimodular(2048, [512, 1024, 1536, 2048], 64, 43)
    dev, abi, keep = [], [], []
    for (p, n) in jobs:
        Ap, Bp = reduce_mod(A[:n, :n], p), reduce_mod(B[:n, :n], p)
        dA, dB = to_dev(Ap), to_dev(Bp)
        dC = to_dev(np.zeros((n, n), np.uint32))
        keep.append((dA, dB))
        dev.append((p, n, Ap, Bp, dC))
        abi.append(ff.job(p, dA, dB, dC))
    torch.cuda.synchronize()
    g = ff.ff_batch_graph_create(abi, ff.make_opts(path=ff.FF_PATH_INT8))
    rng = np.random.default_rng(8)
    try:
        stream = torch.cuda.current_stream()
        for replay in range(3):
            for (_, _, _, _, dC) in dev:
                dC.fill_(-1)
            torch.cuda.synchronize()
            ff.ff_batch_graph_launch(g, stream.cuda_stream)
            torch.cuda.synchronize()
            by_size = {}
            for (p, n, Ap, Bp, dC) in dev:
                by_size.setdefault(n, []).append((p, Ap, Bp, from_dev(dC)))
            for n, lst in by_size.items():
                rows, cols = rng.integers(0, n, 16), rng.integers(0, n, 16)
                elo, ehi = oracle.int_matmul(A[rows, :n], B[:n, cols])
                lo, hi = oracle.crt([q for q, _, _, _ in lst[:4]],
                                    [got[np.ix_(rows, cols)] for _, _, _, got in lst[:4]])
                assert np.array_equal(lo, elo) and np.array_equal(hi, ehi), (replay, n)
                for p, Ap, Bp, got in lst:
                    r2, c2 = rng.integers(0, n, 32), rng.integers(0, n, 32)
                    assert np.array_equal(got[r2, c2], oracle.fgemm_entries(p, Ap, Bp, r2, c2)), \
                        (replay, n, p)
                if replay == 0:
                    p, Ap, Bp, got = lst[0]
                    assert np.array_equal(got, oracle.fgemm(p, Ap, Bp)), (n, p)
    finally:
        ff.ff_batch_graph_destroy(g)
