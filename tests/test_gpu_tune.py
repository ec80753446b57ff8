"""The tile autotuner and the measurement hooks.

ff_autotune times every compiled configuration of a slice count, records the
fastest in its cache file, and later calls of that size class use it: the
results must stay bit-exact with the oracle whichever tile runs.  The
profiling mask brackets only the kernels it names.
"""
import math

import numpy as np
import pytest

import oracle
from gpu_util import from_dev, to_dev
from paper_cs_0601133_amd import ffgemm as ff
from paper_cs_0601133_amd import synth

pytestmark = pytest.mark.gpu


def test_autotune_records_a_tile_and_results_stay_exact(tmp_path, monkeypatch):
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("FF_TUNE_CACHE", str(cache))
    p, m, n, k = 8388593, 384, 320, 448
    best, ms = ff.ff_autotune(4, m, n, k)
    assert best >= 0 and ms > 0
    # one line "S class tile ms" for this size class
    cls = math.floor(math.log2(m * n * k) / 3)
    lines = [l.split() for l in cache.read_text().splitlines()]
    assert ["4", str(cls), str(best)] in [l[:3] for l in lines]
    # the planner now reports the tuned tile for this size class
    o = ff.make_opts(path=ff.FF_PATH_INT8, digit_bits=7, winograd_levels=0)
    assert ff.ff_plan_query(p, 0, 0, m, n, k, o).tile_config == best
    A = synth.residues(synth.seed_for(70, 1), (m, k), p)
    B = synth.residues(synth.seed_for(70, 2), (k, n), p)
    C = synth.residues(synth.seed_for(70, 3), (m, n), p)
    dA, dB, dC = to_dev(A), to_dev(B), to_dev(C)
    ff.fgemm(p, dA, dB, dC, 3, 5, opts=o)
    assert np.array_equal(from_dev(dC), oracle.fgemm(p, A, B, C, 3, 5))


def test_autotune_rejects_bad_arguments():
    for args in ((0, 64, 64, 64), (6, 64, 64, 64), (4, 0, 64, 64)):
        with pytest.raises(ff.FFError) as e:
            ff.ff_autotune(*args)
        assert e.value.status == ff.FF_EINVAL


@pytest.mark.parametrize("path", [ff.FF_PATH_INT8, ff.FF_PATH_FP64], ids=["int8", "fp64"])
def test_profile_mask_selects_kernels(path, monkeypatch):
    import torch
    # the general FP64 path (packing launch + GEMM launch), not the one-launch
    # kernel this size would otherwise take
    monkeypatch.setenv("FF_F64_SMALL", "0")
    p = 65521
    A = synth.residues(synth.seed_for(71, 1), (300, 200), p)
    B = synth.residues(synth.seed_for(71, 2), (200, 260), p)
    dA, dB = to_dev(A), to_dev(B)
    dC = to_dev(np.zeros((300, 260), np.uint32))
    o = ff.make_opts(path=path, winograd_levels=0)
    try:
        ff.ff_profile_enable(ff.FF_PROFILE_GEMM)
        ff.fgemm(p, dA, dB, dC, opts=o)
        g = ff.ff_profile_read()
        ff.ff_profile_enable(ff.FF_PROFILE_PREP)
        ff.fgemm(p, dA, dB, dC, opts=o)
        s = ff.ff_profile_read()
        ff.ff_profile_enable(0)
        ff.fgemm(p, dA, dB, dC, opts=o)
        z = ff.ff_profile_read()
    finally:
        ff.ff_profile_enable(0)
    torch.cuda.synchronize()
    assert g["gemm_launches"] == 1 and g["slice_launches"] == 0 and g["gemm_ms"] > 0
    assert s["gemm_launches"] == 0 and s["slice_launches"] == 1 and s["slice_ms"] > 0
    assert z["gemm_launches"] == 0 and z["slice_launches"] == 0
    assert np.array_equal(from_dev(dC), oracle.fgemm(p, A, B))


def test_profile_one_launch_fp64_small_product(monkeypatch):
    import torch
    monkeypatch.delenv("FF_F64_SMALL", raising=False)
    p = 65521
    A = synth.residues(synth.seed_for(72, 1), (300, 200), p)
    B = synth.residues(synth.seed_for(72, 2), (200, 260), p)
    dA, dB = to_dev(A), to_dev(B)
    dC = to_dev(np.zeros((300, 260), np.uint32))
    o = ff.make_opts(path=ff.FF_PATH_FP64, winograd_levels=0)
    try:
        ff.ff_profile_enable(ff.FF_PROFILE_GEMM | ff.FF_PROFILE_PREP)
        ff.fgemm(p, dA, dB, dC, opts=o)
        g = ff.ff_profile_read()
    finally:
        ff.ff_profile_enable(0)
    torch.cuda.synchronize()
    assert g["gemm_launches"] == 1 and g["slice_launches"] == 0
    assert np.array_equal(from_dev(dC), oracle.fgemm(p, A, B))
