"""Seeded random configurations, bit-exact against the oracle: fgemm, and
the triangular solve, symmetric product and LQUP built on it.

Each case draws a path (automatic, FP64, INT8 with 7- or 8-bit digits),
Winograd levels (-1..3), the pre-addition mode, transposes, a modulus from
2 to 2^31 - 1, alpha and beta, ragged sizes up to a few hundred, and the
FF_WINO_FUSED / FF_F64_SMALL switches; combinations the planner declares
unsupported are skipped.  The draws are fixed by the seed, so a failure
names a reproducible case.
"""
import numpy as np
import pytest

import oracle
from gpu_util import from_dev, to_dev
from paper_cs_0601133_amd import ffgemm as ff
from paper_cs_0601133_amd import synth

pytestmark = pytest.mark.gpu

MODULI = [2, 3, 7, 251, 65521, 1048573, 8388593, 67108859, 89999999, 2147483647]


def cases(seed, count):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        path, bits = [(ff.FF_PATH_AUTO, 0), (ff.FF_PATH_FP64, 0), (ff.FF_PATH_INT8, 7),
                      (ff.FF_PATH_INT8, 8)][rng.integers(4)]
        levels = int(rng.integers(-1, 4))
        lo = 16 << max(levels, 0)  # leaves of at least 16
        m, n, k = (int(rng.integers(lo, lo + 300)) for _ in range(3))
        out.append(dict(p=int(MODULI[rng.integers(len(MODULI))]), path=path, bits=bits,
                        levels=levels, mode=int(rng.integers(3)), m=m, n=n, k=k,
                        tA=bool(rng.integers(2)), tB=bool(rng.integers(2)),
                        alpha=int(rng.integers(1 << 31)), beta=int(rng.integers(1 << 31)),
                        fused=str(rng.integers(2)), small=["", "0", "1"][rng.integers(3)]))
    return out


@pytest.mark.parametrize("block", range(12))
def test_random_configurations(block, monkeypatch):
    ran = 0
    for ci, c in enumerate(cases(1000 + block, 12)):
        monkeypatch.setenv("FF_WINO_FUSED", c["fused"])
        if c["small"]:
            monkeypatch.setenv("FF_F64_SMALL", c["small"])
        else:
            monkeypatch.delenv("FF_F64_SMALL", raising=False)
        p, m, n, k, tA, tB = c["p"], c["m"], c["n"], c["k"], c["tA"], c["tB"]
        o = ff.make_opts(path=c["path"], digit_bits=c["bits"], winograd_levels=c["levels"],
                         preadd_mode=c["mode"])
        try:
            ff.ff_plan_query(p, int(tA), int(tB), m, n, k, o)
        except ff.FFError as e:
            assert e.status == ff.FF_EUNSUPPORTED, c
            continue
        seed = 5000 + 100 * block + ci
        A = synth.residues(synth.seed_for(seed, 1), (k, m) if tA else (m, k), p)
        B = synth.residues(synth.seed_for(seed, 2), (n, k) if tB else (k, n), p)
        C = synth.residues(synth.seed_for(seed, 3), (m, n), p)
        dA, dB, dC = to_dev(A), to_dev(B), to_dev(C)
        ff.fgemm(p, dA, dB, dC, c["alpha"], c["beta"], tA, tB, opts=o)
        want = oracle.fgemm(p, A, B, C, c["alpha"] % p, c["beta"] % p, tA, tB)
        assert np.array_equal(from_dev(dC), want), c
        ran += 1
    assert ran > 0


TRSM_MODULI = [2, 3, 7, 65521, 8388593, 2147483647]


@pytest.mark.parametrize("block", range(4))
def test_random_triangular_solves(block, monkeypatch):
    # op(T) X = alpha B with random uplo/trans/diag, sizes across the 64-row
    # block and the 512-row leaf, and the leaf size switch
    rng = np.random.default_rng(2000 + block)
    for ci in range(8):
        p = int(TRSM_MODULI[rng.integers(len(TRSM_MODULI))])
        m, n = int(rng.integers(1, 700)), int(rng.integers(1, 200))
        lower, trans, unit = (int(rng.integers(2)) for _ in range(3))
        alpha = int(rng.integers(1 << 31)) % p
        monkeypatch.setenv("FF_TRSM_LEAF", str(64 * int(rng.integers(1, 9))))
        seed = 6000 + 100 * block + ci
        T = synth.residues(synth.seed_for(seed, 1), (m, m), p)
        for i in range(m):
            T[i, i] = 1 + T[i, i] % (p - 1)  # a unit for prime p
        B = synth.residues(synth.seed_for(seed, 2), (m, n), p)
        dT, dB = to_dev(T), to_dev(B)
        ff.ftrsm(p, dT, dB, alpha, lower, trans, unit)
        want = oracle.ftrsm(p, T, B, alpha, lower, trans, unit)
        assert np.array_equal(from_dev(dB), want), (p, m, n, lower, trans, unit)


@pytest.mark.parametrize("block", range(2))
def test_random_symmetric_products_and_factorisations(block):
    rng = np.random.default_rng(3000 + block)
    for ci in range(6):
        seed = 7000 + 100 * block + ci
        # A diag(D) A^T on either path, with and without D
        p = int([65521, 8388593, 251][rng.integers(3)])
        m, k = int(rng.integers(1, 400)), int(rng.integers(1, 400))
        A = synth.residues(synth.seed_for(seed, 1), (m, k), p)
        d = synth.residues(synth.seed_for(seed, 2), (k,), p) if rng.integers(2) else None
        C = synth.residues(synth.seed_for(seed, 3), (m, m), p)
        alpha, beta = int(rng.integers(p)), int(rng.integers(p))
        path = [ff.FF_PATH_AUTO, ff.FF_PATH_FP64, ff.FF_PATH_INT8][rng.integers(3)]
        dA, dC = to_dev(A), to_dev(C)
        dD = to_dev(d) if d is not None else None
        ff.aat(p, dA, dC, dD, alpha, beta, opts=ff.make_opts(path=path))
        assert np.array_equal(from_dev(dC), oracle.aat(p, A, d, alpha, beta, C)), (p, m, k)
        # LQUP against the oracle's factorisation (unique under the pivot
        # rule); small moduli make dependent rows likely
        p = int([2, 3, 7, 65521, 8388593][rng.integers(5)])
        m, n = int(rng.integers(1, 300)), int(rng.integers(1, 300))
        A = synth.residues(synth.seed_for(seed, 4), (m, n), p)
        dA = to_dev(A)
        r, piv, perm = ff.lqup(p, dA)
        F0, r0, piv0, perm0 = oracle.lqup(p, A)
        assert r == r0 and np.array_equal(perm, perm0) and np.array_equal(piv, piv0), (p, m, n)
        assert np.array_equal(from_dev(dA), F0), (p, m, n)


@pytest.mark.parametrize("block", range(3))
def test_random_batches(block):
    # one batched launch of jobs with their own modulus, sizes (K = 0 too),
    # transposes, alpha and beta; every job against the oracle
    import torch
    rng = np.random.default_rng(4000 + block)
    path = [ff.FF_PATH_INT8, ff.FF_PATH_FP64, ff.FF_PATH_AUTO][block]
    moduli = [2, 251, 65521, 1048573, 8388593] + ([2147483647] if path != ff.FF_PATH_FP64 else [])
    jobs, abi = [], []
    for ci in range(int(rng.integers(8, 20))):
        p = int(moduli[rng.integers(len(moduli))])
        m, n = int(rng.integers(1, 400)), int(rng.integers(1, 400))
        k = int(rng.integers(0, 400)) if ci % 7 else 0
        tA, tB = bool(rng.integers(2)), bool(rng.integers(2))
        alpha, beta = int(rng.integers(p)), int(rng.integers(p)) if ci % 5 else 0
        seed = 8000 + 100 * block + ci
        A = synth.residues(synth.seed_for(seed, 1), (max(k, 1), m) if tA else (m, max(k, 1)), p)
        B = synth.residues(synth.seed_for(seed, 2), (n, max(k, 1)) if tB else (max(k, 1), n), p)
        C = synth.residues(synth.seed_for(seed, 3), (m, n), p)
        dA, dB, dC = to_dev(A), to_dev(B), to_dev(C)
        j = ff.job(p, dA, dB, dC, alpha, beta, tA, tB)
        if k == 0:
            # the operands stay allocated; the job reads none of them
            j.k = 0
            A = A[:0, :] if tA else A[:, :0]
            B = B[:, :0] if tB else B[:0, :]
        jobs.append((p, A, B, C, alpha, beta, tA, tB, dC, dA, dB))
        abi.append(j)
    ff.ff_set_stream(None)
    torch.cuda.synchronize()
    assert ff.ff_fgemm_batched(abi, ff.make_opts(path=path)) == ff.FF_OK, ff.ff_last_error()
    torch.cuda.synchronize()
    for (p, A, B, C, alpha, beta, tA, tB, dC, _, _) in jobs:
        want = oracle.fgemm(p, A, B, C, alpha, beta, tA, tB)
        assert np.array_equal(from_dev(dC), want), (p, A.shape, B.shape, tA, tB, alpha, beta)


@pytest.mark.parametrize("block", range(3))
def test_random_inverses(block):
    # square matrices of random order, modulus and path, in place or apart;
    # small moduli make singular ones likely (reported, X untouched)
    rng = np.random.default_rng(5000 + block)
    for ci in range(6):
        seed = 9000 + 100 * block + ci
        path = [ff.FF_PATH_AUTO, ff.FF_PATH_FP64, ff.FF_PATH_INT8][rng.integers(3)]
        moduli = [2, 3, 7, 65521, 8388593] + ([2147483647] if path != ff.FF_PATH_FP64 else [])
        p = int(moduli[rng.integers(len(moduli))])
        n = int(rng.integers(1, 300))
        in_place = bool(rng.integers(2))
        A = synth.residues(synth.seed_for(seed, 1), (n, n), p)
        dA = to_dev(A)
        dX = dA if in_place else to_dev(np.full((n, n), 0xABCD, np.uint32))
        ok = ff.inv(p, dA, dX, opts=ff.make_opts(path=path))
        want = oracle.inv(p, A)
        assert ok == (want is not None), (p, n)
        if ok:
            assert np.array_equal(from_dev(dX), want), (path, p, n, in_place)
        elif not in_place:
            assert np.all(from_dev(dX) == 0xABCD), (p, n)
