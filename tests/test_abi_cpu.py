"""Host-side checks of the C ABI (no GPU needed, no compute calls).

* libffgemm.so loads and exports every function include/ffgemm.h declares;
* the planner (ff_plan_query, C++) agrees with the oracle's bound
  calculator (Python, exact integers) on K-blocks, slice counts, operand
  ranges and leaf product bounds;
* argument errors come back as status codes with a message, before any
  device is touched.
"""
import os
import re

import numpy as np
import pytest

from oracle import bounds as bd
from paper_cs_0601133_amd import ffgemm as ff

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "ffgemm.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ff_\w+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = ff.load()
    names = declared_functions()
    assert len(names) >= 15
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(names) == ff.EXPORTED


P_LIST = [2, 3, 5, 251, 65521, 1048573, 8388593, 2147483647]


@pytest.mark.parametrize("p", P_LIST)
def test_plan_fp64_kblock_matches_bound(p):
    o = ff.make_opts(path=ff.FF_PATH_FP64, winograd_levels=0)
    lo, hi = bd.centered_range(p)
    M = max(-lo, hi)
    kb = bd.fp64_kblock(M * M, p + 2)
    if kb < 4:
        with pytest.raises(ff.FFError) as e:
            ff.ff_plan_query(p, 0, 0, 64, 64, 64, o)
        assert e.value.status == ff.FF_EUNSUPPORTED
        return
    info = ff.ff_plan_query(p, 0, 0, 64, 64, 64, o)
    assert info.path == ff.FF_PATH_FP64
    assert info.kblock == kb
    assert (info.operand_lo, info.operand_hi) == (lo, hi)
    assert info.max_abs_product == M * M


@pytest.mark.parametrize("p", P_LIST)
@pytest.mark.parametrize("bits", [7, 8])
def test_plan_int8_slices_match_bound(p, bits):
    o = ff.make_opts(path=ff.FF_PATH_INT8, winograd_levels=0, digit_bits=bits)
    lo, hi = bd.centered_range(p)
    s = bd.slices_needed(lo, hi, bits)
    if s > 5:
        with pytest.raises(ff.FFError):
            ff.ff_plan_query(p, 0, 0, 64, 64, 64, o)
        return
    info = ff.ff_plan_query(p, 0, 0, 64, 64, 64, o)
    assert info.slices == s
    d = bd.digit_max_abs(lo, hi, bits, s)
    assert info.kblock == bd.int32_kblock(d, d, s)


@pytest.mark.parametrize("L", [1, 2, 3])
@pytest.mark.parametrize("p", [251, 65521, 8388593])
def test_plan_winograd_leaf_bounds(L, p):
    lo, hi = bd.centered_range(p)
    wl, wh = bd.winograd_leaf_operand_range(lo, hi, lo, hi, L)
    mp = bd.winograd_leaf_max_product(lo, hi, lo, hi, L)
    # delayed (unreduced) pre-additions, FP64 path
    o = ff.make_opts(path=ff.FF_PATH_FP64, winograd_levels=L, preadd_mode=1)
    kb = bd.fp64_kblock(mp, p + 2)
    if kb >= 4:
        info = ff.ff_plan_query(p, 0, 0, 1024, 1024, 1024, o)
        assert info.winograd_levels == L and info.preadds_reduced == 0
        assert (info.operand_lo, info.operand_hi) == (wl, wh)
        assert info.max_abs_product == mp
        assert info.kblock == kb
    # delayed pre-additions, INT8 path, 7-bit digits
    o = ff.make_opts(path=ff.FF_PATH_INT8, winograd_levels=L, preadd_mode=1, digit_bits=7)
    info = ff.ff_plan_query(p, 0, 0, 1024, 1024, 1024, o)
    assert info.slices == bd.slices_needed(wl, wh, 7)
    # reduced pre-additions: leaves are centered residues again
    o = ff.make_opts(path=ff.FF_PATH_INT8, winograd_levels=L, preadd_mode=2, digit_bits=8)
    info = ff.ff_plan_query(p, 0, 0, 1024, 1024, 1024, o)
    assert info.preadds_reduced == 1
    assert info.slices == bd.slices_needed(lo, hi, 8)


def test_plan_configs_of_the_workloads():
    # n = 4096, p = 8388593: FP64 K-block 512; INT8 with 4 signed 7-bit digits
    i = ff.ff_plan_query(8388593, 0, 0, 4096, 4096, 4096,
                         ff.make_opts(path=ff.FF_PATH_FP64, winograd_levels=0))
    assert i.kblock == 512
    i = ff.ff_plan_query(8388593, 0, 0, 4096, 4096, 4096,
                         ff.make_opts(path=ff.FF_PATH_INT8, digit_bits=7, winograd_levels=0))
    assert i.slices == 4 and i.kblock >= 4096
    # p = 251: one direct int8 plane, exact int32 sums up to k = 137438
    i = ff.ff_plan_query(251, 0, 0, 8192, 8192, 8192,
                         ff.make_opts(path=ff.FF_PATH_INT8, winograd_levels=0))
    assert i.slices == 1 and i.kblock == 137438
    # Winograd leaves at p = 8388593: FP64 K-blocks 56 (l = 1) and 6 (l = 2)
    for L, kb in ((1, 56), (2, 6)):
        i = ff.ff_plan_query(8388593, 0, 0, 8192, 8192, 8192,
                             ff.make_opts(path=ff.FF_PATH_FP64, winograd_levels=L,
                                          preadd_mode=1))
        assert i.kblock == kb


def test_plan_direct_plane_tiles(monkeypatch):
    # one-digit products: the 256 x 256 tile (id 21) where its tiles fill
    # whole rounds of one workgroup per CU (256 CUs), else the default two
    # 128 x 128 workgroups per CU (id 20)
    monkeypatch.delenv("FF_I8_TILE", raising=False)
    o = ff.make_opts(path=ff.FF_PATH_INT8, winograd_levels=0)
    for n, tile in ((2048, 20), (3072, 20), (4096, 21), (6144, 20), (8192, 21)):
        assert ff.ff_plan_query(251, 0, 0, n, n, n, o).tile_config == tile, n


def test_plan_fp64_small_products_need_no_workspace(monkeypatch):
    # m * n <= 512^2 and k <= 768: one launch reads the residues in place
    monkeypatch.delenv("FF_F64_SMALL", raising=False)
    o = ff.make_opts(path=ff.FF_PATH_FP64, winograd_levels=0)
    assert ff.ff_plan_query(65521, 0, 0, 256, 256, 256, o).workspace_bytes == 0
    assert ff.ff_plan_query(65521, 0, 0, 512, 512, 768, o).workspace_bytes == 0
    assert ff.ff_plan_query(65521, 0, 0, 512, 512, 769, o).workspace_bytes > 0
    assert ff.ff_plan_query(65521, 0, 0, 513, 512, 64, o).workspace_bytes > 0


def test_plan_automatic_path_for_small_products(monkeypatch):
    # the automatic path takes the one-launch FP64 kernel for small products
    # where the FP64 K-block allows the modulus and no digit width is asked
    # for; INT8 otherwise
    monkeypatch.delenv("FF_F64_SMALL", raising=False)

    def path(p, m, n, k, **kw):
        return ff.ff_plan_query(p, 0, 0, m, n, k, ff.make_opts(**kw)).path

    assert path(65521, 256, 256, 256) == ff.FF_PATH_FP64
    assert path(251, 64, 512, 768) == ff.FF_PATH_FP64
    assert path(65521, 256, 256, 256, digit_bits=7) == ff.FF_PATH_INT8
    assert path(2147483647, 256, 256, 256) == ff.FF_PATH_INT8   # FP64 K-block < 4
    assert path(65521, 1024, 1024, 1024) == ff.FF_PATH_INT8
    assert path(65521, 256, 256, 769) == ff.FF_PATH_INT8


def test_plan_fp64_tiles_and_split_k_workspace(monkeypatch):
    # A single launch with fewer than 256 tiles splits K into
    # min(K stages, 512 / tiles) parts; the workspace is
    # the packed operands (8 bytes per padded element) plus, 256-aligned,
    # one uint32 partial product per split.  (Small products take the
    # one-launch kernel by default; FF_F64_SMALL=0 keeps the general path.)
    monkeypatch.setenv("FF_F64_SMALL", "0")
    monkeypatch.delenv("FF_F64_TILE", raising=False)
    o = ff.make_opts(path=ff.FF_PATH_FP64, winograd_levels=0)
    # the 256 x 128 tile where its tiles fill whole rounds of one workgroup
    # per CU (256 CUs), the 128 x 128 tile otherwise; Winograd leaves count
    # all of a level's products
    for n, tile in ((2048, 2), (3072, 2), (4096, 1), (6144, 2), (8192, 1)):
        assert ff.ff_plan_query(8388593, 0, 0, n, n, n, o).tile_config == tile, n
    for n, L, tile in ((4096, 1, 2), (8192, 1, 1), (8192, 2, 2)):
        wo = ff.make_opts(path=ff.FF_PATH_FP64, winograd_levels=L)
        assert ff.ff_plan_query(8388593, 0, 0, n, n, n, wo).tile_config == tile, (n, L)
    i = ff.ff_plan_query(8388593, 0, 0, 4096, 4096, 4096, o)
    assert i.tile_config == 1
    assert i.workspace_bytes == (4096 + 4096) * 4096 * 8          # 512 tiles: no split
    i = ff.ff_plan_query(65521, 0, 0, 256, 256, 256, o)
    assert i.tile_config == 2
    tiles, stages = 4, 256 // 16
    splits = min(stages, 512 // tiles)                              # 16 splits of 1 stage
    assert i.workspace_bytes == (256 + 256) * 256 * 8 + 256 + splits * 256 * 256 * 4
    i = ff.ff_plan_query(8388593, 0, 0, 3, 5, 1000003, o)
    stages = (1000003 + 15) // 16
    per = -(-stages // 512)
    splits = -(-stages // per)
    assert i.workspace_bytes == (128 + 128) * stages * 16 * 8 + 256 + splits * 3 * 5 * 4


def test_plan_automatic_winograd_levels(monkeypatch):
    # Section 3.2.1 leaves the crossover to experiment.  Automatic levels:
    # a first level at min(m, n, k) >= w_first, one more per halving while
    # the leaf order stays >= w_next.  INT8 with one digit: never; INT8 with
    # more digits: (3072, 12288) below p = 2^30, (8192, 24576) above;
    # FP64: (3072, 3072).  FF_WINOGRAD_W = w is the paper's
    # l = floor(log2(n / w)) + 1.
    monkeypatch.delenv("FF_WINOGRAD_W", raising=False)
    i8, f64 = ff.make_opts(path=ff.FF_PATH_INT8), ff.make_opts(path=ff.FF_PATH_FP64)

    def lv(p, n, o, m=None, k=None):
        return ff.ff_plan_query(p, 0, 0, m or n, n, k or n, o).winograd_levels

    assert lv(251, 32768, i8) == 0
    assert [lv(8388593, n, i8) for n in (3071, 3072, 24575, 24576)] == [0, 1, 1, 2]
    assert lv(8388593, 8192, i8, k=2048) == 0            # the smallest order decides
    assert [lv(2147483647, n, i8) for n in (8191, 8192, 49152)] == [0, 1, 2]
    assert [lv(65521, n, f64) for n in (3071, 3072, 6143, 6144, 12288)] == [0, 1, 1, 2, 3]
    monkeypatch.setenv("FF_WINOGRAD_W", "5000")
    assert [lv(8388593, n, i8) for n in (4999, 5000, 10000, 20000)] == [0, 1, 2, 3]
    assert lv(251, 5000, i8) == 1


def test_plan_int8_winograd_workspace(monkeypatch):
    # INT8 leaves in one int32 pass: the last level's seven int32
    # combinations per side are sliced in registers, so the workspace holds
    # no buffer for them (m = n = k = 4096, one level: 7 leaves of 2048^2
    # int32 per side)
    o = ff.make_opts(path=ff.FF_PATH_INT8, winograd_levels=1)
    monkeypatch.delenv("FF_WINO_FUSED", raising=False)
    fused = ff.ff_plan_query(8388593, 0, 0, 4096, 4096, 4096, o).workspace_bytes
    monkeypatch.setenv("FF_WINO_FUSED", "0")
    apart = ff.ff_plan_query(8388593, 0, 0, 4096, 4096, 4096, o).workspace_bytes
    assert apart - fused == 2 * 7 * 2048 * 2048 * 4
    # from three levels on two sets of int32 combinations are stored either
    # way (levels 1 and 2 alternate), so the workspace is the same
    o3 = ff.make_opts(path=ff.FF_PATH_INT8, winograd_levels=3)
    apart3 = ff.ff_plan_query(8388593, 0, 0, 4096, 4096, 4096, o3).workspace_bytes
    monkeypatch.delenv("FF_WINO_FUSED")
    assert ff.ff_plan_query(8388593, 0, 0, 4096, 4096, 4096, o3).workspace_bytes == apart3


@pytest.mark.parametrize("args,msg", [
    ((1, 0, 0, 4, 4, 4, 1, 8, 4, 8, 4, 0, 8, 4), "p must"),
    ((7, 2, 0, 4, 4, 4, 1, 8, 4, 8, 4, 0, 8, 4), "trans"),
    ((7, 0, 0, -1, 4, 4, 1, 8, 4, 8, 4, 0, 8, 4), "negative"),
    ((7, 0, 0, 4, 4, 4, 1, 8, 3, 8, 4, 0, 8, 4), "lda"),
    ((7, 0, 0, 4, 4, 4, 1, 8, 4, 8, 3, 0, 8, 4), "ldb"),
    ((7, 0, 0, 4, 4, 4, 1, 8, 4, 8, 4, 0, 8, 3), "ldc"),
    ((7, 0, 0, 4, 4, 4, 1, None, 4, 8, 4, 0, 8, 4), "null"),
    ((7, 0, 0, 4, 4, 4, 1, 8, 4, 8, 4, 0, None, 4), "null"),
    ((7, 1, 0, 4, 5, 3, 1, 8, 3, 8, 5, 0, 8, 5), "lda"),
])
def test_argument_errors(args, msg):
    rc = ff.ff_fgemm(*args)
    assert rc == ff.FF_EINVAL
    assert msg in ff.ff_last_error()


def test_empty_product_is_a_no_op_without_device():
    # m == 0 or n == 0 returns before any device call
    assert ff.ff_fgemm(7, 0, 0, 0, 4, 4, 1, None, 4, None, 4, 0, None, 4) == ff.FF_OK
    assert ff.ff_fgemm(7, 0, 0, 4, 0, 4, 1, None, 4, None, 4, 0, None, 4) == ff.FF_OK


def test_inverse_argument_checks_without_device():
    # every check comes before the first device call; n = 0 is invertible
    ok = np.zeros(1, np.int32)
    assert ff.ff_finv(7, 0, None, 1, None, 1, ok) == ff.FF_OK and ok[0] == 1
    for n, ldx, x, msg in ((-1, 4, 8, "negative"), (70000, 70000, 8, "65535"),
                           (4, 3, 8, "ldx"), (4, 4, None, "null")):
        assert ff.ff_finv(7, n, 8, 4, x, ldx, ok) == ff.FF_EINVAL
        assert msg in ff.ff_last_error(), msg
    rc = ff.load().ff_finv(7, 4, 8, 4, 8, 4, None, None)
    assert rc == ff.FF_EINVAL and "null output" in ff.ff_last_error()


def test_bad_options():
    for o in (ff.make_opts(path=5), ff.make_opts(digit_bits=6),
              ff.make_opts(winograd_levels=4), ff.make_opts(preadd_mode=3)):
        with pytest.raises(ff.FFError) as e:
            ff.ff_plan_query(7, 0, 0, 8, 8, 8, o)
        assert e.value.status == ff.FF_EINVAL


def test_plan_digit_pairing():
    # 7-bit digits with products of digit sums for the cross terms: S(S+1)/2
    # digit products, S(S+1)/2 planes per operand, and an int32 K-block from
    # the largest set of sum products sharing one weight (two pairs for
    # S = 4 and 5: 2 * 128^2 per step)
    o = ff.make_opts(path=ff.FF_PATH_INT8, digit_pairing=1)
    for p, S, kb in ((8191, 2, 131071), (65521, 3, 131071), (8388593, 4, 65535),
                     (2147483647, 5, 65535)):
        i = ff.ff_plan_query(p, 0, 0, 4096, 4096, 4096, o)
        assert (i.slices, i.digit_bits, i.digit_products) == (S, 7, S * (S + 1) // 2), p
        assert i.kblock == kb and i.winograd_levels == 0 and i.tile_config == -1, p
        bm = 64 if S == 5 else 128
        assert i.workspace_bytes == S * (S + 1) // 2 * (4096 // bm * bm + 4096) * 4096, p
        plain = ff.ff_plan_query(p, 0, 0, 4096, 4096, 4096,
                                 ff.make_opts(path=ff.FF_PATH_INT8, digit_bits=7,
                                              winograd_levels=0))
        assert plain.digit_products == S * S and plain.slices == S
    # one direct plane: nothing to pair
    i = ff.ff_plan_query(251, 0, 0, 256, 256, 256, o)
    assert i.slices == 1 and i.digit_products == 1
    for bad, status in ((dict(path=ff.FF_PATH_FP64, digit_pairing=1), ff.FF_EUNSUPPORTED),
                        (dict(path=ff.FF_PATH_INT8, digit_bits=8, digit_pairing=1),
                         ff.FF_EUNSUPPORTED),
                        (dict(path=ff.FF_PATH_INT8, winograd_levels=1, digit_pairing=1),
                         ff.FF_EUNSUPPORTED),
                        (dict(digit_pairing=2), ff.FF_EINVAL)):
        with pytest.raises(ff.FFError) as e:
            ff.ff_plan_query(8388593, 0, 0, 512, 512, 512, ff.make_opts(**bad))
        assert e.value.status == status, bad
