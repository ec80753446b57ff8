"""Parity of the HIP LQUP factorisation, rank and determinant with the CPU
oracle (bit-exact).

Under the pivoting rule both sides follow (rows in order, first nonzero
column not yet used) the compressed factorisation, the pivot rows and the
column permutation are unique, so they are compared element by element.
At 2048 and 4096 (the benchmark's size) the whole factored matrix is
compared too; the inverse there is checked on sampled rows of X A.
"""
import numpy as np
import pytest

import oracle
from gpu_util import from_dev, to_dev
from paper_cs_0601133_amd import ffgemm as ff
from paper_cs_0601133_amd import synth

pytestmark = pytest.mark.gpu

PRIMES = [2, 3, 7, 65521, 8388593, 2147483647]


def gpu_lqup(p, A, **opts):
    dA = to_dev(A)
    r, piv, perm = ff.lqup(p, dA, opts=ff.make_opts(**opts))
    return from_dev(dA), r, piv, perm


def assert_same(p, A, **opts):
    F, r, piv, perm = gpu_lqup(p, A, **opts)
    F0, r0, piv0, perm0 = oracle.lqup(p, A)
    assert r == r0, (A.shape, r, r0)
    assert np.array_equal(perm, perm0), A.shape
    assert np.array_equal(piv, piv0), A.shape
    assert np.array_equal(F, F0), A.shape
    return r


def known_rank(p, m, n, r, seed):
    # X = [I_r; R1] (rows shuffled) times Y = [I_r R2] (columns shuffled)
    rng = np.random.default_rng(seed)
    X = np.zeros((m, r), np.uint32)
    Y = np.zeros((r, n), np.uint32)
    X[:r] = np.eye(r, dtype=np.uint32)
    X[r:] = synth.residues(synth.seed_for(seed, 1), (m - r, r), p)
    Y[:, :r] = np.eye(r, dtype=np.uint32)
    Y[:, r:] = synth.residues(synth.seed_for(seed, 2), (r, n - r), p)
    return oracle.fgemm(p, np.ascontiguousarray(X[rng.permutation(m)]),
                        np.ascontiguousarray(Y[:, rng.permutation(n)]))


@pytest.mark.parametrize("p", PRIMES)
def test_random_matrices_match_the_oracle(p):
    # shapes spanning several panels, ragged ones, and windows narrower
    # than the remaining columns
    for si, (m, n) in enumerate([(1, 1), (5, 3), (3, 5), (64, 64), (65, 70), (130, 100),
                                  (100, 300), (300, 290)]):
        A = synth.residues(synth.seed_for(140 + si, 1), (m, n), p)
        assert_same(p, A)


@pytest.mark.parametrize("p", [7, 8388593, 2147483647])
def test_constructed_ranks_match_the_oracle(p):
    for si, (m, n, r) in enumerate([(100, 80, 0), (100, 80, 1), (100, 80, 37), (200, 600, 30),
                                     (150, 150, 149), (300, 120, 120)]):
        A = known_rank(p, m, n, r, 150 + si)
        assert assert_same(p, A) == r, (m, n, r)


def test_pivots_past_the_window():
    # row i has its only nonzero at column 400 + 3i: every panel row must
    # search past the 256-column window; rows 7 and 8 repeat rows 1 and 2
    p, m, n = 65521, 12, 600
    A = np.zeros((m, n), np.uint32)
    for i in range(m):
        A[i, 400 + 3 * i] = 1 + i
    A[7] = 2 * A[1] % p
    A[8] = 5 * A[2] % p
    assert_same(p, A)
    # a dense block below such rows
    B = np.vstack([A, synth.residues(synth.seed_for(160, 1), (70, n), p)])
    assert_same(p, B)


def test_update_paths():
    p, m, n = 8388593, 260, 300
    A = synth.residues(synth.seed_for(161, 1), (m, n), p)
    assert_same(p, A, path=ff.FF_PATH_FP64)
    assert_same(p, A, path=ff.FF_PATH_INT8)


def test_rank_and_det():
    import torch
    for p in (7, 65521, 2147483647):
        for si, n in enumerate((1, 2, 17, 130)):
            A = synth.residues(synth.seed_for(170 + si, 1), (n, n), p)
            d = ff.det(p, to_dev(A))
            assert d == oracle.det(p, A), (p, n)
        S = known_rank(p, 90, 90, 89, 175)
        assert ff.det(p, to_dev(S)) == 0
        rank = np.zeros(1, np.int64)
        R = known_rank(p, 90, 140, 61, 176)
        dR = to_dev(R)
        assert ff.ff_frank(p, 90, 140, dR, 140, rank) == ff.FF_OK and rank[0] == 61
    d = np.zeros(1, np.uint32)
    assert ff.ff_fdet(7, 0, to_dev(np.zeros((1, 1), np.uint32)), 1, d) == ff.FF_OK and d[0] == 1
    torch.cuda.synchronize()


def test_arguments_and_empty_shapes():
    p = 7
    rank = np.zeros(1, np.int64)
    piv = np.zeros(4, np.int64)
    perm = np.zeros(4, np.int64)
    dA = to_dev(np.ones((4, 4), np.uint32))
    assert ff.ff_flqup(p, 4, 4, dA, 3, rank, piv, perm) == ff.FF_EINVAL   # lda < n
    assert ff.ff_flqup(1, 4, 4, dA, 4, rank, piv, perm) == ff.FF_EINVAL   # p < 2
    assert ff.ff_flqup(p, 0, 4, dA, 4, rank, piv, perm) == ff.FF_OK and rank[0] == 0
    assert list(perm) == [0, 1, 2, 3]
    # validate rejects entries >= p and writes nothing
    bad = np.ones((4, 4), np.uint32)
    bad[2, 3] = p
    dB = to_dev(bad)
    assert ff.ff_flqup(p, 4, 4, dB, 4, rank, piv, perm, ff.make_opts(validate=1)) == ff.FF_EINVAL
    assert np.array_equal(from_dev(dB), bad)


def check_certificate(p, A, F, r, piv, perm, samples, seed):
    m, n = A.shape
    assert sorted(piv) == list(range(m)) and sorted(perm) == list(range(n))
    is_piv = np.zeros(m, bool)
    is_piv[piv[:r]] = True
    above = np.concatenate(([0], np.cumsum(is_piv)[:-1]))
    for i in range(m):
        ka = int(above[i])
        if is_piv[i]:
            assert F[i, ka] != 0, i
        else:
            assert not F[i, ka:].any(), i
    L, QU = oracle.lqup_factors(p, F, r, piv)
    rng = np.random.default_rng(seed)
    rows = rng.integers(0, m, samples)
    cols = rng.integers(0, n, samples)
    lhs = oracle.fgemm_entries(p, L, QU, rows, cols)
    assert np.array_equal(lhs, A[:, perm][rows, cols])


@pytest.mark.parametrize("n", [2048, 4096])
def test_full_size_whole_output(n):
    # m = n = 4096, p = 8388593 is the benchmark's launch configuration;
    # the whole factored matrix, pivots and permutation against the oracle
    p = 8388593
    A = synth.residues(synth.seed_for(180 + n, 1), (n, n), p)
    assert assert_same(p, A) == n
    # rank deficient at full width: rank n / 2
    if n == 2048:
        R = known_rank(p, n, n, n // 2, 181)
        assert assert_same(p, R) == n // 2
        F, r, piv, perm = gpu_lqup(p, R)
        check_certificate(p, R, F, r, piv, perm, 600, 6)


def gpu_inv(p, A, in_place=False, **opts):
    n = A.shape[0]
    dA = to_dev(A)
    dX = dA if in_place else to_dev(np.full((n, n), 0xABCD, np.uint32))
    ok = ff.inv(p, dA, dX, opts=ff.make_opts(**opts))
    return ok, from_dev(dX)


@pytest.mark.parametrize("path", ["auto", "int8", "fp64"])
def test_inverse_matches_the_oracle(path):
    # the inverse is unique: bit-exact against Gauss-Jordan; singular
    # matrices report it and leave X as it was
    kw = {} if path == "auto" else {"path": ff.FF_PATH_INT8 if path == "int8" else ff.FF_PATH_FP64}
    primes = [3, 7, 65521, 8388593] + ([2147483647] if path != "fp64" else [])
    for pi, p in enumerate(primes):
        for si, n in enumerate([1, 2, 64, 65, 130, 300]):
            A = synth.residues(synth.seed_for(1900 + 10 * pi + si, 1), (n, n), p)
            want = oracle.inv(p, A)
            ok, X = gpu_inv(p, A, in_place=bool(si & 1), **kw)
            if want is None:
                assert not ok, (p, n)
                if not si & 1:
                    assert np.all(X == 0xABCD), (p, n)
            else:
                assert ok and np.array_equal(X, want), (path, p, n)


def test_inverse_of_singular_and_special_matrices():
    p = 65521
    for si, (n, r) in enumerate([(80, 79), (80, 0), (200, 100)]):
        A = known_rank(p, n, n, r, 1950 + si)
        ok, X = gpu_inv(p, A)
        assert not ok and np.all(X == 0xABCD), (n, r)
    perm = np.random.default_rng(1960).permutation(150)
    P = np.ascontiguousarray(np.eye(150, dtype=np.uint32)[perm])
    ok, X = gpu_inv(p, P)
    assert ok and np.array_equal(X, P.T)
    inv_ok = np.zeros(1, np.int32)
    assert ff.ff_finv(p, 0, 0, 1, 0, 1, inv_ok) == ff.FF_OK and inv_ok[0] == 1
    # validate rejects entries >= p and writes neither A nor X
    bad = synth.residues(synth.seed_for(1965, 1), (20, 20), p)
    bad[7, 11] = p
    dB, dX = to_dev(bad), to_dev(np.full((20, 20), 0xABCD, np.uint32))
    rc = ff.ff_finv(p, 20, dB, 20, dX, 20, inv_ok, ff.make_opts(validate=1))
    assert rc == ff.FF_EINVAL
    assert np.array_equal(from_dev(dB), bad) and np.all(from_dev(dX) == 0xABCD)


@pytest.mark.parametrize("n", [2048, 4096])
def test_inverse_full_size_sampled_rows(n):
    # sampled rows of X A against the identity through the fgemm oracle
    p = 8388593
    A = synth.residues(synth.seed_for(1970 + n, 1), (n, n), p)
    ok, X = gpu_inv(p, A)
    assert ok
    rows = np.random.default_rng(n).choice(n, 6, replace=False)
    XA = oracle.fgemm(p, np.ascontiguousarray(X[rows]), A, np.zeros((6, n), np.uint32))
    assert np.array_equal(XA, np.eye(n, dtype=np.uint32)[rows])


def test_concurrent_factorisations_on_two_streams():
    # two host threads factor different matrices at once, each on a torch
    # stream of its own: every call borrows its own second stream (the
    # panels' solves past the window run there) and per-stream workspace,
    # so the results must be those of the oracle, every repetition
    import threading
    import torch
    p = 8388593
    shapes = [(256, 300), (320, 320)]          # m <= n: the full-rank fast path
    mats = [synth.residues(synth.seed_for(170 + i, 1), s, p) for i, s in enumerate(shapes)]
    want = [oracle.lqup(p, A) for A in mats]
    errors = []

    def work(i):
        try:
            s = torch.cuda.Stream()
            with torch.cuda.stream(s):
                for rep in range(4):
                    dA = torch.from_numpy(mats[i].view(np.int32)).to("cuda", non_blocking=False)
                    r, piv, perm = ff.lqup(p, dA)
                    s.synchronize()
                    F = dA.cpu().numpy().view(np.uint32)
                    F0, r0, piv0, perm0 = want[i]
                    if not (r == r0 and np.array_equal(F, F0) and np.array_equal(piv, piv0)
                            and np.array_equal(perm, perm0)):
                        errors.append((i, rep))
        except Exception as e:  # reported below, on the test's thread
            errors.append((i, repr(e)))

    threads = [threading.Thread(target=work, args=(i,), daemon=True) for i in range(2)]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=120)
    assert not any(t.is_alive() for t in threads), "a factorisation did not return"
    assert not errors, errors


@pytest.mark.parametrize("block", ["64", "128", "576", "4096"])
def test_fast_path_node_sizes(block, monkeypatch):
    # The full-rank fast path factors nodes of up to FF_LQUP_BLOCK rows panel
    # by panel, each panel launch also solving G T = X for the node's rows
    # below it (64: never, so the recursion's own solves run; 4096: every
    # row below each panel, more workgroups than one round of CUs for the
    # first panels).  Full rank and rank-deficient inputs (the guess fails
    # and the general path runs), square and wide, ragged last panels.
    monkeypatch.setenv("FF_LQUP_BLOCK", block)
    for si, (p, m, n) in enumerate([(8388593, 1000, 1000), (65521, 700, 1090),
                                     (7, 250, 260)]):
        A = synth.residues(synth.seed_for(190 + si, 1), (m, n), p)
        assert_same(p, A)
    assert_same(65521, known_rank(65521, 600, 640, 590, 191))
