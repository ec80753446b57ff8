"""Seeded random configurations of fgemm, bit-exact against the oracle.

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
