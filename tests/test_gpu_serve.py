"""Serving loop: continuous batching, admission by HBM footprint.

Every result is bit-exact vs the oracle and identical to the same request
computed alone; a small budget forces queueing; a request that can never fit
is refused with FF_EBUSY.
"""
import time

import numpy as np
import pytest

import oracle
from gpu_util import from_dev, to_dev
from paper_cs_0601133_amd import ffgemm as ff
from paper_cs_0601133_amd import synth

pytestmark = pytest.mark.gpu

PRIMES = [251, 65521, 8388593]


def make_requests(count, lo, hi, seed):
    rng = np.random.default_rng(seed)
    reqs = []
    for r in range(count):
        m, n, k = (int(round(np.exp(rng.uniform(np.log(lo), np.log(hi))))) for _ in range(3))
        p = PRIMES[int(rng.integers(0, 3))]
        A = synth.residues(synth.request_seed(r, 1), (m, k), p)
        B = synth.residues(synth.request_seed(r, 2), (k, n), p)
        C = synth.residues(synth.request_seed(r, 3), (m, n), p)
        reqs.append((p, A, B, C))
    return reqs


def submit_all(srv, reqs, gap_s=0.0):
    handles = []
    for (p, A, B, C) in reqs:
        dA, dB, dC = to_dev(A), to_dev(B), to_dev(C)
        import torch
        torch.cuda.synchronize()
        rid = ff.ff_server_submit(srv, ff.job(p, dA, dB, dC, 3, 5))
        handles.append((rid, dA, dB, dC))
        if gap_s:
            time.sleep(gap_s)
    return handles


def test_server_results_alone_and_in_the_mix():
    reqs = make_requests(48, 64, 512, 70)
    srv = ff.ff_server_create(1 << 30)
    try:
        handles = submit_all(srv, reqs, gap_s=0.0005)
        for rid, *_ in handles:
            ff.ff_server_wait(srv, rid)
        st = ff.ff_server_stats(srv)
        assert st["completed"] == len(reqs)
        assert st["p99_ms"] >= st["p50_ms"] > 0
        mixed = [from_dev(h[3]) for h in handles]
    finally:
        ff.ff_server_destroy(srv)
    for (p, A, B, C), got in zip(reqs, mixed):
        # alone: the same request through the single-call entry point
        dA, dB, dC = to_dev(A), to_dev(B), to_dev(C)
        ff.fgemm(p, dA, dB, dC, 3, 5)
        alone = from_dev(dC)
        assert np.array_equal(got, alone)
        assert np.array_equal(got, oracle.fgemm(p, A, B, C, 3, 5))


def test_server_admission_under_small_budget():
    reqs = make_requests(12, 128, 384, 71)
    # room for about two requests at a time
    budget = 6 * 4 * 384 * 384 * 2 + 2 * 4 * 3 * 512 * 512
    srv = ff.ff_server_create(budget)
    try:
        handles = submit_all(srv, reqs)
        for rid, *_ in handles:
            ff.ff_server_wait(srv, rid)
        st = ff.ff_server_stats(srv)
        assert st["completed"] == len(reqs)
        assert st["max_inflight"] < len(reqs)
        for (p, A, B, C), h in zip(reqs, handles):
            assert np.array_equal(from_dev(h[3]), oracle.fgemm(p, A, B, C, 3, 5))
        # a request that can never fit
        big = 4096
        dA = to_dev(np.zeros((big, big), np.uint32))
        with pytest.raises(ff.FFError) as e:
            ff.ff_server_submit(srv, ff.job(251, dA, dA, dA))
        assert e.value.status == ff.FF_EBUSY
    finally:
        ff.ff_server_destroy(srv)


def test_server_unknown_id():
    srv = ff.ff_server_create(1 << 24)
    try:
        with pytest.raises(ff.FFError) as e:
            ff.ff_server_poll(srv, 12345)
        assert e.value.status == ff.FF_ENOTFOUND
    finally:
        ff.ff_server_destroy(srv)
