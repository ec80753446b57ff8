"""Accumulation and growth bounds of the paper, in exact integers.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).  These are the
quantities the GPU planner must reproduce; the planner is C++ and shares no
code with this module.

Notation: for a modulus p, the centered (balanced) residue of u in [0, p) is
u if u <= (p-1)//2 else u - p, so centered values lie in
[-(p//2), (p-1)//2] and M = p//2 bounds their magnitude (Section 2.1.2; for
even p the paper is silent and this is the reading taken).
"""
from fractions import Fraction

TWO53 = 1 << 53
INT32_MAX = (1 << 31) - 1


# --- Section 2.1.2, delayed reduction --------------------------------------

def lambda_positive(p, gamma):
    """eq. (1): the largest lambda with lambda*(p-1)^2 < 2^gamma, i.e. the
    number of products of residues in [0, p-1] that can be summed in a
    gamma-bit integer before a reduction is due."""
    q = (p - 1) ** 2
    return ((1 << gamma) - 1) // q


def lambda_centered(p, gamma):
    """eq. (2): the largest lambda with lambda*((p-1)/2)^2 < 2^(gamma-1),
    for centered residues of an odd modulus."""
    h = (p - 1) // 2
    return ((1 << (gamma - 1)) - 1) // (h * h)


def t_update(p, gamma=53):
    """Section 4.3's table column t_update: lambda - 1 with lambda from
    eq. (1), one product's worth of room being kept for the accumulated
    right-hand side.  The printed value for p = 5 (2 147 483 642) is
    2^31 - 1 - p, i.e. the implementation caps the block at the 32-bit index
    range; the cap is applied here the same way (reading, one data point)."""
    return min(lambda_positive(p, gamma) - 1, INT32_MAX - p)


# --- Section 3.2.3, Theorem 3.1 and its corollaries ------------------------

def t_s(l):
    """t_l = (1+3^l)/2 and s_l = (1-3^l)/2 of Appendix A (both integers)."""
    return (1 + 3 ** l) // 2, (1 - 3 ** l) // 2


def v_series(m, M, l):
    """v_l = t_l*M + s_l*m: the growth series of Appendix A, with u_0 = m <= 0
    and v_0 = M >= 0."""
    t, s = t_s(l)
    return t * M + s * m


def thm31_bound(mA, MA, mB, MB, k, l):
    """Theorem 3.1: every intermediate value of A*B + beta*C computed with l
    levels of Winograd's algorithm (inner dimension k) is bounded in magnitude
    by v_l^A * v_l^B * floor(k / 2^l)."""
    return v_series(mA, MA, l) * v_series(mB, MB, l) * (k >> l)


def cor32_positive(p, k, l):
    """Corollary 3.2: ((1+3^l)/2)^2 * floor(k/2^l) * (p-1)^2."""
    t, _ = t_s(l)
    return t * t * (k >> l) * (p - 1) ** 2


def cor33_balanced(p, k, l):
    """Corollary 3.3: (3^l/2)^2 * floor(k/2^l) * (p-1)^2 (a Fraction in
    general; an integer for odd p)."""
    return Fraction(3 ** l, 2) ** 2 * (k >> l) * (p - 1) ** 2


def k_winograd_paper(p, l, gamma, balanced):
    """Corollary 3.4's closed form (a real number: the printed formula takes
    no floor), positive or balanced representation."""
    c = (3 ** l) if balanced else (1 + 3 ** l)
    return (Fraction(1 << (gamma + 2), (c * (p - 1)) ** 2) + 1) * (1 << l)


def k_winograd_exact(p, l, gamma, balanced):
    """The exact threshold behind Corollary 3.4: the smallest k for which the
    corollary's bound reaches 2^gamma; every k below it is safe."""
    if balanced:
        c = Fraction(3 ** l, 2) ** 2 * (p - 1) ** 2
    else:
        t, _ = t_s(l)
        c = t * t * (p - 1) ** 2
    # bound(k) = c * floor(k / 2^l) < 2^gamma  <=>  floor(k/2^l) <= d with d
    # the largest integer such that c*d < 2^gamma, i.e. ceil(2^gamma/c) - 1.
    q = Fraction(1 << gamma) / c
    d = -((-q.numerator) // q.denominator) - 1
    return (d + 1) << l


# --- the readings used by the GPU path (checked against the above) ---------

def centered_range(p):
    """(lo, hi) of centered residues: [-(p//2), (p-1)//2]."""
    return -(p // 2), (p - 1) // 2


def fp64_kblock(max_abs_product, carry):
    """Largest K-block kb with kb*max_abs_product + carry <= 2^53: every
    partial sum of kb products plus the residue carried over from the previous
    block is then an integer of magnitude <= 2^53, hence exact in binary64
    whatever the summation order."""
    return (TWO53 - carry) // max_abs_product


def digit_capacity(bits, s):
    """Range (lo, hi) covered by s signed digits of the given width, digits
    in [-2^(bits-1), 2^(bits-1) - 1] with base 2^bits."""
    R = 1 << bits
    geo = (R ** s - 1) // (R - 1)
    return -(R // 2) * geo, (R // 2 - 1) * geo


def slices_needed(lo, hi, bits):
    """Smallest number of signed digits that represents every integer in
    [lo, hi]; a range that fits int8 directly takes one plane."""
    if -128 <= lo and hi <= 127:
        return 1
    s = 1
    while True:
        clo, chi = digit_capacity(bits, s)
        if clo <= lo and hi <= chi:
            return s
        s += 1


def digit_max_abs(lo, hi, bits, s):
    """Largest |digit| that occurs: the value itself for one direct plane,
    else the most negative digit."""
    if s == 1 and -128 <= lo and hi <= 127:
        return max(-lo, hi)
    return 1 << (bits - 1)


def int32_kblock(dA, dB, s):
    """Largest K with s * K * dA * dB <= 2^31 - 1: the accumulator of the
    digit-product sums E_t = sum_{i+j=t} A_i B_j takes at most s digit pairs,
    each contributing K products of magnitude <= dA*dB."""
    return INT32_MAX // (s * dA * dB)


# --- Winograd operand growth (Appendix A's pre-additions) ------------------

def _a_side(lo, hi):
    """Ranges of the seven A-side operands of one Winograd level, in product
    order P1..P7: A11, A12, S4, A22, S1, S2, S3."""
    s1 = (2 * lo, 2 * hi)
    s2 = (2 * lo - hi, 2 * hi - lo)
    s3 = (lo - hi, hi - lo)
    s4 = (2 * lo - 2 * hi, 2 * hi - 2 * lo)
    return [(lo, hi), (lo, hi), s4, (lo, hi), s1, s2, s3]


def _b_side(lo, hi):
    """B-side operands in product order P1..P7: B11, B21, B22, T4, T1, T2, T3."""
    t1 = (lo - hi, hi - lo)
    t2 = (2 * lo - hi, 2 * hi - lo)
    t3 = (lo - hi, hi - lo)
    t4 = (2 * lo - 2 * hi, 2 * hi - 2 * lo)
    return [(lo, hi), (lo, hi), (lo, hi), t4, t1, t2, t3]


def winograd_leaf_ranges(loA, hiA, loB, hiB, l):
    """Operand ranges of all 7^l leaf products after l levels of unreduced
    pre-additions: list of ((loA, hiA), (loB, hiB))."""
    leaves = [((loA, hiA), (loB, hiB))]
    for _ in range(l):
        nxt = []
        for ra, rb in leaves:
            for xa, xb in zip(_a_side(*ra), _b_side(*rb)):
                nxt.append((xa, xb))
        leaves = nxt
    return leaves


def winograd_leaf_max_product(loA, hiA, loB, hiB, l):
    """max over leaves of max|a| * max|b|: the per-term bound of a leaf dot
    product (equals v_l^A v_l^B, Theorem 3.1 with k = 2^l)."""
    best = 0
    for (la, ha), (lb, hb) in winograd_leaf_ranges(loA, hiA, loB, hiB, l):
        best = max(best, max(-la, ha) * max(-lb, hb))
    return best


def winograd_leaf_operand_range(loA, hiA, loB, hiB, l):
    """Widest operand range over all leaves (both sides): what the digit
    slicer has to cover."""
    lo, hi = 0, 0
    for (la, ha), (lb, hb) in winograd_leaf_ranges(loA, hiA, loB, hiB, l):
        lo = min(lo, la, lb)
        hi = max(hi, ha, hb)
    return lo, hi


# --- Section 4.2, delayed reductions in a triangular solve -----------------

def trsm_uv(m, M, k):
    """Theorem 4.2: u_k and v_k for a unit upper triangular system whose
    entries (and right-hand side) lie in [m, M], m <= 0 <= M.  The unknown
    x_{n-k} lies in [-u_k, v_k] for even k and [-v_k, u_k] for odd k.
    Returned as exact rationals (the halves cancel for integer inputs of the
    same parity)."""
    u = Fraction(M - m, 2) * (M + 1) ** k - Fraction(M + m, 2) * (M - 1) ** k
    v = Fraction(M - m, 2) * (M + 1) ** k + Fraction(M + m, 2) * (M - 1) ** k
    return u, v


def trsm_bound(m, M, n):
    """Corollary 4.3: |x| <= v_{n-1} for a system of dimension n."""
    return trsm_uv(m, M, n - 1)[1]


def trsm_bound_positive(p, n):
    """Corollary 4.4: entries in [0, p-1]."""
    return Fraction(p - 1, 2) * (p ** (n - 1) + (p - 1) ** (n - 1))


def trsm_bound_balanced(p, n):
    """Corollary 4.5: entries in [-(p-1)/2, (p-1)/2]."""
    return Fraction(p - 1, 2) * Fraction(p + 1, 2) ** (n - 1)


def t_del_positive(p, gamma=53):
    """eq. (trsmboundpos): the largest n with (p-1)/2 (p^(n-1) + (p-1)^(n-1))
    < 2^gamma, the dimension of a unit triangular solve over Z that needs no
    reduction (positive representation)."""
    n = 1
    while trsm_bound_positive(p, n + 1) < (1 << gamma):
        n += 1
    return n


def t_del_balanced(p, gamma=53):
    """eq. (trsmboundcen) as printed: the largest n with
    (p-1)/2 ((p+1)/2)^n < 2^gamma.  The exponent is n where Corollary 4.5
    has n - 1 (reading: the printed, more conservative form, which gives the
    text's 52 for p = 3)."""
    n = 0
    while Fraction(p - 1, 2) * Fraction(p + 1, 2) ** (n + 1) < (1 << gamma):
        n += 1
    return n
