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
    """Device copies of every request first, then the submits back to back
    (with an optional gap), so that requests arrive while others run."""
    import torch
    dev = [(to_dev(A), to_dev(B), to_dev(C)) for (_, A, B, C) in reqs]
    torch.cuda.synchronize()
    handles = []
    for (p, A, B, C), (dA, dB, dC) in zip(reqs, dev):
        rid = ff.ff_server_submit(srv, ff.job(p, dA, dB, dC, 3, 5))
        handles.append((rid, dA, dB, dC))
        if gap_s:
            time.sleep(gap_s)
    return handles


def test_server_results_alone_and_in_the_mix():
    # a long request first, then a burst of small ones that arrive while it
    # runs (each of those alone finishes in microseconds)
    p0 = 65521
    big = (p0, synth.residues(synth.request_seed(999, 1), (2048, 2048), p0),
           synth.residues(synth.request_seed(999, 2), (2048, 2048), p0),
           synth.residues(synth.request_seed(999, 3), (2048, 2048), p0))
    reqs = [big] + make_requests(47, 64, 512, 70)
    srv = ff.ff_server_create(1 << 30)
    try:
        handles = submit_all(srv, reqs)
        for rid, *_ in handles:
            ff.ff_server_wait(srv, rid)
        st = ff.ff_server_stats(srv)
        assert st["completed"] == len(reqs)
        assert st["p99_ms"] >= st["p50_ms"] > 0
        info = ff.ff_server_query(srv)
        # the requests were mixed: merged into shared launches or on the
        # device together
        assert info.max_batch_requests >= 2 or info.max_inflight >= 2
        assert 1 <= info.batches <= len(reqs)
        assert info.last_i8_tile >= 0 and info.failed == 0
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


def _check_request(p, A, B, C0, got, alpha, beta, seed):
    m, k = A.shape
    n = B.shape[1]
    if m * n * k <= 1 << 28:
        want = oracle.fgemm(p, A, B, C0, alpha, beta)
        return np.array_equal(got, want)
    rng = np.random.default_rng(seed)
    rows, cols = rng.integers(0, m, 64), rng.integers(0, n, 64)
    want = oracle.fgemm_entries(p, A, B, rows, cols, C0[rows, cols], alpha, beta)
    if not np.array_equal(got[rows, cols], want):
        return False
    X = rng.integers(0, p, (2, n), dtype=np.uint32)
    return oracle.freivalds(p, A, B, C0, got, X, alpha, beta) == 0


def test_server_poisson_stream_at_the_configured_sizes():
    # m, n, k log-uniform in [64, 4096], p from {251, 65521, 8388593},
    # seeded inputs per request, seeded Poisson arrivals (mean gap 0.5 ms).
    # Each request's operands are written by a copy kernel enqueued on the
    # submitting stream just before the submit (no synchronisation): the
    # server must order its launch after them.  Every result is checked:
    # the whole output where the oracle is quick, sampled entries and
    # Freivalds otherwise.
    import torch
    count = 40
    reqs = make_requests(count, 64, 4096, 72)
    gaps = np.random.default_rng(73).exponential(0.0005, count)
    src = [(to_dev(A), to_dev(B), to_dev(C)) for (_, A, B, C) in reqs]
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    srv = ff.ff_server_create(24 << 30, ff.make_opts(stream=stream.cuda_stream))
    try:
        handles = []
        for (p, A, B, C), (sA, sB, sC), gap in zip(reqs, src, gaps):
            dA, dB, dC = sA.clone(), sB.clone(), sC.clone()   # enqueued, not waited on
            handles.append((ff.ff_server_submit(srv, ff.job(p, dA, dB, dC, 3, 5)), dA, dB, dC))
            time.sleep(gap)
        for rid, *_ in handles:
            ff.ff_server_wait(srv, rid)
        info = ff.ff_server_query(srv)
        assert info.completed == count and info.failed == 0
        assert info.max_batch_requests >= 2 or info.max_inflight >= 2
        outs = [from_dev(h[3]) for h in handles]
    finally:
        ff.ff_server_destroy(srv)
    for i, ((p, A, B, C), got) in enumerate(zip(reqs, outs)):
        assert _check_request(p, A, B, C, got, 3, 5, 900 + i), (i, p, A.shape, B.shape)


def test_server_create_failure_releases_everything():
    # an arena the device cannot hold: FF_ENOMEM, nothing left behind (a
    # second server is created and used normally afterwards)
    with pytest.raises(ff.FFError) as e:
        ff.ff_server_create(1 << 52)
    assert e.value.status == ff.FF_ENOMEM
    reqs = make_requests(3, 64, 128, 74)
    srv = ff.ff_server_create(1 << 26)
    try:
        handles = submit_all(srv, reqs)
        for rid, *_ in handles:
            ff.ff_server_wait(srv, rid)
        for (p, A, B, C), h in zip(reqs, handles):
            assert np.array_equal(from_dev(h[3]), oracle.fgemm(p, A, B, C, 3, 5))
    finally:
        ff.ff_server_destroy(srv)
