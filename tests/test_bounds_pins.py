"""Pins of the oracle's bounds and Winograd algebra against the paper.

* Section 4.3's parameter table: t_update from eq. (1) for three primes.
* Table "tab:winolevel": operation counts of the exact-integer Winograd
  implementation, counted while it runs, against all 25 printed entries, and
  the level rule l = floor(log2(n/w)) + 1 of Section 3.2.1 against the
  printed optima.
* Appendix A's P4 = A22*T4 against the A12 printed in the schedule table of
  Section 3.2.2.
* eq. (1) and eq. (2) of Section 2.1.2: hand values, the factor of two the
  centered representation gains, and a brute-force search over every
  sequence of centered products in a gamma-bit two's-complement register.
* Theorem 3.1: Appendix A's matrices A_l, B_l reach the bound exactly; random
  and extreme inputs never exceed it; Corollaries 3.2/3.3 are its special
  cases; Corollary 3.4's exact threshold is checked by brute force over k.
* The readings the GPU path relies on, checked by brute force where possible:
  digit capacities, the binary64 K-block, the int32 K-block.
"""
import itertools
import math
import random

import pytest

from oracle import bounds as bd
from oracle import winograd as wg
from golden_io import trsm_params, winolevel


def test_t_update_column():
    # (the table's ceil(log2 p) column prints 20 and 23 for primes just above
    # 2^20 and 2^23; it is not used)
    for p, _logp, _tdel, tupd in trsm_params():
        assert bd.t_update(p, 53) == tupd


def test_winolevel_table_counts():
    for n, (vals, best) in winolevel().items():
        for l, want in enumerate(vals):
            A = [[1] * n for _ in range(n)]
            tr = wg.Tracker()
            wg.winograd_mul(A, A, l, tr)
            assert tr.ops == want, (n, l)
        assert min(range(len(vals)), key=vals.__getitem__) == best


@pytest.mark.parametrize("w", [9, 12, 16])
def test_level_rule_matches_printed_optimum(w):
    # The bold optimum of each row equals floor(log2(n/w)) + 1, clamped at 0,
    # for any crossover order w in (8, 16].
    for n, (_vals, best) in winolevel().items():
        l = max(0, math.floor(math.log2(n / w)) + 1)
        assert l == best


def _rand(rows, cols, lo, hi, rnd):
    return [[rnd.randint(lo, hi) for _ in range(cols)] for _ in range(rows)]


def test_winograd_equals_classic_and_peeling():
    rnd = random.Random(5)
    for l in (1, 2, 3):
        n = 8
        A = _rand(n, n, -50, 50, rnd)
        B = _rand(n, n, -50, 50, rnd)
        assert wg.winograd_mul(A, B, l) == wg.classic(A, B)
    for (m, k, n) in [(5, 7, 3), (9, 4, 11), (6, 6, 6), (3, 3, 3)]:
        A = _rand(m, k, -9, 9, rnd)
        B = _rand(k, n, -9, 9, rnd)
        for l in (1, 2):
            assert wg.winograd_mul_peeled(A, B, l) == wg.classic(A, B)


def test_p4_is_a22_times_t4():
    # Appendix A: P4 = A22*T4, and U6 = U3 - P4 is the block C21 of A*B.
    # The alpha/beta schedule table of Section 3.2.2 prints A12 in its P4
    # step; with that operand U6 is not C21 (reading of a misprint).
    rnd = random.Random(7)
    for n in (2, 4, 6):
        A = _rand(n, n, -20, 20, rnd)
        B = _rand(n, n, -20, 20, rnd)
        A11, A12, A21, A22 = wg._split(A)
        B11, B12, B21, B22 = wg._split(B)
        cl = wg.classic
        S1 = wg._add(A21, A22, None)
        S2 = wg._add(S1, A11, None, -1)
        S3 = wg._add(A11, A21, None, -1)
        T1 = wg._add(B12, B11, None, -1)
        T2 = wg._add(B22, T1, None, -1)
        T3 = wg._add(B22, B12, None, -1)
        T4 = wg._add(T2, B21, None, -1)
        U3 = wg._add(wg._add(cl(A11, B11), cl(S2, T2), None), cl(S3, T3), None)
        C21 = wg._add(cl(A21, B11), cl(A22, B21), None)
        assert wg._add(U3, cl(A22, T4), None, -1) == C21
        assert wg._add(U3, cl(A12, T4), None, -1) != C21


@pytest.mark.parametrize("l", [1, 2, 3, 4])
@pytest.mark.parametrize("mM", [(-5, 5), (0, 10), (-3, 7), (-4194296, 4194296)])
def test_theorem31_optimality_construction(l, mM):
    m, M = mM
    A, B = wg.optimal_pair(l, m, M, m, M)
    tr = wg.Tracker()
    C = wg.winograd_mul(A, B, l, tr)
    assert C == wg.classic(A, B)
    assert tr.max_abs == bd.thm31_bound(m, M, m, M, 1 << l, l)


def test_theorem31_never_exceeded():
    rnd = random.Random(11)
    for l in (1, 2):
        for k in (4, 6, 8, 12):
            n = 4 if l == 1 else 8
            if k % (1 << l):
                continue
            for (mA, MA) in [(-6, 6), (0, 9), (-2, 8)]:
                mB, MB = mA, MA
                mC, MC = max(mB, -3), min(MB, 3)
                beta = min(MA, MB, 3)
                A = _rand(n, k, mA, MA, rnd)
                B = _rand(k, n, mB, MB, rnd)
                C = _rand(n, n, mC, MC, rnd)
                tr = wg.Tracker()
                got = wg.winograd_abc_appendix(A, B, C, beta, l, tr)
                want = [[x + beta * c for x, c in zip(r1, r2)]
                        for r1, r2 in zip(wg.classic(A, B), C)]
                assert got == want
                assert tr.max_abs <= bd.thm31_bound(mA, MA, mB, MB, k, l)


def test_corollaries_are_special_cases():
    for p in (5, 251, 65521, 8388593):
        for l in (1, 2, 3):
            for k in (8, 100, 4096):
                assert bd.cor32_positive(p, k, l) == bd.thm31_bound(
                    0, p - 1, 0, p - 1, k, l)
                h = (p - 1) // 2
                assert bd.cor33_balanced(p, k, l) == bd.thm31_bound(
                    -h, h, -h, h, k, l)


def test_cor34_exact_threshold_by_brute_force():
    for gamma in (20, 24, 30):
        for p in (3, 5, 11, 31):
            for l in (1, 2):
                for balanced in (False, True):
                    kw = bd.k_winograd_exact(p, l, gamma, balanced)
                    def bound(k):
                        return (bd.cor33_balanced(p, k, l) if balanced
                                else bd.cor32_positive(p, k, l))
                    assert bound(kw - 1) < (1 << gamma) <= bound(kw)
                    # the closed form of the corollary is the real relaxation
                    assert kw - 1 < bd.k_winograd_paper(p, l, gamma, balanced)


def test_fp64_kblock_values():
    p = 8388593
    M = p // 2
    kb = bd.fp64_kblock(M * M, p)
    assert kb == 512
    assert kb * M * M + p <= 1 << 53 < (kb + 1) * M * M
    assert bd.fp64_kblock(bd.winograd_leaf_max_product(-M, M, -M, M, 1), p) == 56
    assert bd.fp64_kblock(bd.winograd_leaf_max_product(-M, M, -M, M, 2), p) == 6
    # p = 65521: no K-blocking needed at k = 256
    assert bd.fp64_kblock((65521 // 2) ** 2, 65521) > 256


def test_leaf_max_product_is_theorem31_at_k_2l():
    for (m, M) in [(-7, 7), (0, 12), (-3, 9)]:
        for l in (1, 2, 3):
            assert bd.winograd_leaf_max_product(m, M, m, M, l) == \
                bd.thm31_bound(m, M, m, M, 1 << l, l)


def test_leaf_operand_range_by_enumeration():
    # l = 1 over [-M, M]: enumerate every block value combination of the
    # A-side pre-additions (S4 = A12 + A11 - A21 - A22 is the widest).
    M = 3
    vals = range(-M, M + 1)
    widest = 0
    for a11, a12, a21, a22 in itertools.product(vals, repeat=4):
        s1 = a21 + a22
        s2 = s1 - a11
        s3 = a11 - a21
        s4 = a12 - s2
        widest = max(widest, abs(s1), abs(s2), abs(s3), abs(s4))
    lo, hi = bd.winograd_leaf_operand_range(-M, M, -M, M, 1)
    assert (lo, hi) == (-widest, widest) == (-4 * M, 4 * M)


@pytest.mark.parametrize("bits,s", [(3, 1), (3, 2), (3, 3), (4, 2), (2, 4)])
def test_digit_capacity_brute_force(bits, s):
    R = 1 << bits
    digits = range(-(R // 2), R // 2)
    values = {sum(d * R ** i for i, d in enumerate(ds))
              for ds in itertools.product(digits, repeat=s)}
    lo, hi = bd.digit_capacity(bits, s)
    assert min(values) == lo and max(values) == hi
    assert values == set(range(lo, hi + 1))   # every integer in between


def test_slice_counts_and_int32_blocks():
    p = 8388593
    lo, hi = bd.centered_range(p)
    assert bd.slices_needed(lo, hi, 7) == 4
    assert bd.slices_needed(lo, hi, 8) == 3
    assert bd.slices_needed(*bd.centered_range(251), 7) == 1
    assert bd.int32_kblock(125, 125, 1) == 137438      # k < 137000 for p = 251
    assert bd.int32_kblock(64, 64, 4) >= 8192
    assert bd.slices_needed(*bd.centered_range(65521), 7) == 3
    assert bd.slices_needed(*bd.centered_range(1048573), 7) == 3
    # Winograd leaves over [-M, M] at p = 8388593: operands up to 4^l M
    for l, s in ((1, 4), (2, 4), (3, 5)):
        wl, wh = bd.winograd_leaf_operand_range(lo, hi, lo, hi, l)
        assert bd.slices_needed(wl, wh, 7) == s


# --- Section 2.1.2, eq. (1) and eq. (2) -----------------------------------

def test_lambda_hand_values():
    # eq. (1): lambda*(p-1)^2 < 2^gamma; eq. (2): lambda*((p-1)/2)^2 < 2^(gamma-1)
    assert bd.lambda_positive(3, 3) == 1        # 1*4 < 8 <= 2*4
    assert bd.lambda_centered(3, 3) == 3        # 3*1 < 4 <= 4*1
    assert bd.lambda_positive(5, 6) == 3        # 3*16 < 64 <= 4*16
    assert bd.lambda_centered(5, 6) == 7        # 7*4 < 32 <= 8*4
    assert bd.lambda_centered(7, 8) == 14       # 14*9 < 128 <= 15*9
    assert bd.lambda_centered(11, 10) == 20     # 20*25 < 512 <= 21*25


def test_lambda_centered_gains_a_factor_of_two():
    # Section 2.1.2: the centered representation improves lambda by a factor
    # of 2 over eq. (1); exactly, lambda_c is 2*lambda or 2*lambda + 1.
    for p in (3, 5, 7, 11, 101, 251, 65521, 1048573, 8388593, 2147483647):
        for gamma in (24, 31, 32, 53, 64):
            lp = bd.lambda_positive(p, gamma)
            lc = bd.lambda_centered(p, gamma)
            assert lc in (2 * lp, 2 * lp + 1), (p, gamma)


def _wraps(x, gamma):
    """x stored in a gamma-bit two's-complement register reads back as x?"""
    lo, hi = -(1 << (gamma - 1)), (1 << (gamma - 1)) - 1
    return lo <= x <= hi


@pytest.mark.parametrize("p,gamma", [(3, 4), (5, 5), (5, 7), (7, 8), (11, 9)])
def test_lambda_centered_brute_force(p, gamma):
    # Largest lambda such that summing ANY lambda products of centered
    # residues in a gamma-bit signed register never leaves its range:
    # breadth-first over the reachable partial sums.
    h = (p - 1) // 2
    prods = {a * b for a in range(-h, h + 1) for b in range(-h, h + 1)}
    sums = {0}
    lam = 0
    while True:
        nxt = {s + q for s in sums for q in prods}
        if not all(_wraps(x, gamma) for x in nxt):
            break
        sums = nxt
        lam += 1
    assert bd.lambda_centered(p, gamma) == lam
    # and the same search over residues in [0, p-1] with an unsigned gamma-bit
    # register gives eq. (1)
    prods = {a * b for a in range(p) for b in range(p)}
    sums, lam = {0}, 0
    while True:
        nxt = {s + q for s in sums for q in prods}
        if max(nxt) >= 1 << gamma:
            break
        sums = nxt
        lam += 1
    assert bd.lambda_positive(p, gamma) == lam


def test_lambda_centered_and_the_fp64_kblock():
    # Reading A1: a binary64 value holds every integer of magnitude <= 2^53,
    # i.e. it acts as a 54-bit signed register in eq. (2)'s sense, so the
    # K-block of the FP64 path at p = 8388593 is lambda_centered(p, 54) = 512
    # (the configuration's k_max), while gamma = 53 in eq. (2) gives 256.
    p = 8388593
    assert bd.lambda_centered(p, 53) == 256
    assert bd.lambda_centered(p, 54) == 512
    assert bd.fp64_kblock((p // 2) ** 2, p) == bd.lambda_centered(p, 54)
