"""Pins of the oracle's triangular solve and of the Section 4.2 bounds.

The solve op(T) X = alpha B (mod p) has exactly one solution when the
diagonal of T is invertible, so the oracle is checked against the defining
equation (through the independently pinned fgemm oracle), against special
cases with closed forms (identity, diagonal T), and against brute force over
Z_3.  The bounds are checked against the paper's printed values (the t_del
column of the Section 4.3 table, the dimensions quoted for Z_3) and against
the optimality construction of Corollary 4.3, solved exactly over Z.
"""
import itertools
from fractions import Fraction

import numpy as np
import pytest

import oracle
from golden_io import trsm_params
from oracle import bounds as bd
from paper_cs_0601133_amd import synth


def tri(p, m, seed, lower):
    """Triangular m x m residues with a nonzero (hence invertible, p prime)
    diagonal; the other triangle holds noise that must not be read."""
    T = synth.residues(synth.seed_for(seed, 1), (m, m), p)
    for i in range(m):
        T[i, i] = 1 + T[i, i] % (p - 1)
    return T


def op_effective(T, lower, trans, unit):
    """op(T) as the triangle the solve uses (other triangle zero)."""
    Te = np.tril(T) if lower else np.triu(T)
    if unit:
        np.fill_diagonal(Te, 1)
    return np.ascontiguousarray(Te.T if trans else Te)


def check_solves(p, T, B, X, alpha, lower, trans, unit, plant=None):
    lhs = oracle.fgemm(p, op_effective(T, lower, trans, unit), X)
    rhs = (alpha * B.astype(np.int64) % p).astype(np.uint32)
    return np.array_equal(lhs, rhs)


@pytest.mark.parametrize("lower,trans,unit", list(itertools.product((0, 1), repeat=3)))
def test_solution_satisfies_the_system(lower, trans, unit):
    for p, m, n in ((7, 9, 5), (65521, 33, 17), (8388593, 40, 3), (2147483647, 12, 6)):
        T = tri(p, m, 80 + m, lower)
        B = synth.residues(synth.seed_for(81 + m, 2), (m, n), p)
        alpha = 5 % p
        X = oracle.ftrsm(p, T, B, alpha, lower, trans, unit)
        assert check_solves(p, T, B, X, alpha, lower, trans, unit), (p, m, n)


def test_identity_and_diagonal_closed_forms():
    p, m, n = 65521, 20, 7
    B = synth.residues(synth.seed_for(82, 2), (m, n), p)
    I = np.eye(m, dtype=np.uint32)
    assert np.array_equal(oracle.ftrsm(p, I, B, 9),
                          (9 * B.astype(np.int64) % p).astype(np.uint32))
    d = [1 + (7 * i * i + 3) % (p - 1) for i in range(m)]
    D = np.diag(np.array(d, dtype=np.uint32))
    want = np.array([[9 * pow(d[i], -1, p) * int(B[i, j]) % p for j in range(n)]
                     for i in range(m)], dtype=np.uint32)
    for lower in (0, 1):
        assert np.array_equal(oracle.ftrsm(p, D, B, 9, lower=lower), want)


def test_brute_force_over_z3():
    # every 2 x 2 upper triangular system over Z_3 with an invertible
    # diagonal: the unique x found by enumeration
    p = 3
    for t00, t01, t11, b0, b1 in itertools.product(range(3), repeat=5):
        if t00 == 0 or t11 == 0:
            continue
        T = np.array([[t00, t01], [0, t11]], np.uint32)
        b = np.array([[b0], [b1]], np.uint32)
        sols = [x for x in itertools.product(range(3), repeat=2)
                if (t00 * x[0] + t01 * x[1]) % 3 == b0 and (t11 * x[1]) % 3 == b1]
        assert len(sols) == 1
        assert tuple(oracle.ftrsm(p, T, b).ravel()) == sols[0]


def test_unit_flag_ignores_the_stored_diagonal():
    p, m, n = 251, 15, 4
    T = tri(p, m, 83, 0)
    B = synth.residues(synth.seed_for(84, 2), (m, n), p)
    T1 = T.copy()
    np.fill_diagonal(T1, 1)
    T0 = T.copy()
    np.fill_diagonal(T0, 0)
    X = oracle.ftrsm(p, T1, B, unit=False)
    assert np.array_equal(oracle.ftrsm(p, T0, B, unit=True), X)
    assert np.array_equal(oracle.ftrsm(p, T, B, unit=True), X)


def test_non_invertible_diagonal_is_reported():
    B = np.ones((3, 2), np.uint32)
    T = np.array([[1, 2, 3], [0, 0, 1], [0, 0, 1]], np.uint32)
    with pytest.raises(ZeroDivisionError):
        oracle.ftrsm(7, T, B)
    # composite modulus: 5 has no inverse modulo 15, 7 has one
    T = np.array([[7, 1], [0, 5]], np.uint32)
    with pytest.raises(ZeroDivisionError):
        oracle.ftrsm(15, T, np.ones((2, 1), np.uint32))
    T[1, 1] = 7
    X = oracle.ftrsm(15, T, np.ones((2, 1), np.uint32))
    assert check_solves(15, T, np.ones((2, 1), np.uint32), X, 1, 0, 0, 0)


def test_planted_mistake_is_caught():
    # plant 6: the division by the diagonal is skipped
    p, m, n = 7, 6, 3
    T = tri(p, m, 85, 0)
    B = synth.residues(synth.seed_for(86, 2), (m, n), p)
    X = oracle.ftrsm(p, T, B, plant=6)
    assert not check_solves(p, T, B, X, 1, 0, 0, 0)


# --- Section 4.2 bounds ----------------------------------------------------

def test_t_del_column_of_the_table():
    # Section 4.3's table: t_del for p = 5, 1048583, 8388617 (the positive
    # representation's bound, eq. (trsmboundpos))
    for p, _logp, tdel, _tupd in trsm_params():
        assert bd.t_del_positive(p) == tdel, p


def test_t_del_values_quoted_in_the_text():
    # Section 4.2: dimension 34 (positive) and 52 (balanced) for Z_3, and
    # n <= 5 for p = 1001 in the positive representation
    assert bd.t_del_positive(3) == 34
    assert bd.t_del_balanced(3) == 52
    assert bd.t_del_positive(1001) == 5


def solve_unit_upper_over_z(T, b):
    n = len(b)
    x = [0] * n
    for i in range(n - 1, -1, -1):
        x[i] = b[i] - sum(T[i][j] * x[j] for j in range(i + 1, n))
    return x


@pytest.mark.parametrize("M,n", [(1, 9), (3, 6), (5, 7), (32760, 4)])
def test_corollary_43_bound_is_attained(M, n):
    # the optimality construction with m = -M (the balanced representation,
    # Corollary 4.5): unit upper T with M on odd and m on even
    # superdiagonals, b alternating M, m from the bottom; then
    # |x_{n-k}| = v_k for every k (Theorem 4.2, Corollary 4.3).  For other
    # ranges the construction falls short of v_k.
    m = -M
    T = [[1 if j == i else (M if (j - i) % 2 else m) if j > i else 0 for j in range(n)]
         for i in range(n)]
    b = [M if (n - 1 - i) % 2 == 0 else m for i in range(n)]
    x = solve_unit_upper_over_z(T, b)
    for k in range(n):
        u, v = bd.trsm_uv(m, M, k)
        assert abs(x[n - 1 - k]) == v, (k, x)
        lo, hi = (-u, v) if k % 2 == 0 else (-v, u)
        assert lo <= x[n - 1 - k] <= hi
    assert max(abs(t) for t in x) == bd.trsm_bound(m, M, n)


def test_theorem_42_holds_on_random_systems():
    # random unit upper systems with entries in [m, M], |m| <= M (the
    # theorem's proof needs -m u_k <= M v_k, which fails for |m| > M): every
    # unknown stays within the theorem's interval
    rng = np.random.default_rng(5)
    for _ in range(300):
        M = int(rng.integers(0, 7))
        m = -int(rng.integers(0, M + 1))
        n = int(rng.integers(1, 8))
        T = [[1 if j == i else int(rng.integers(m, M + 1)) if j > i else 0 for j in range(n)]
             for i in range(n)]
        b = [int(rng.integers(m, M + 1)) for _ in range(n)]
        x = solve_unit_upper_over_z(T, b)
        for k in range(n):
            u, v = bd.trsm_uv(m, M, k)
            lo, hi = (-u, v) if k % 2 == 0 else (-v, u)
            assert lo <= x[n - 1 - k] <= hi, (m, M, T, b, x)


def test_theorem_42_needs_the_range_to_be_balanced_or_positive():
    # with |m| > M the stated interval is wrong: entries in [-4, 1] give
    # x_{n-1} = -4 - (-4)(-4) = -20, outside [-v_1, u_1] = [-5, 5]
    m, M = -4, 1
    x = solve_unit_upper_over_z([[1, m], [0, 1]], [m, m])
    u, v = bd.trsm_uv(m, M, 1)
    assert x[0] == -20 and not (-v <= x[0] <= u)


def test_corollaries_44_45_against_the_theorem():
    for p in (3, 7, 251):
        h = (p - 1) // 2
        for n in range(1, 8):
            # balanced: the theorem at m = -(p-1)/2, M = (p-1)/2
            assert bd.trsm_bound_balanced(p, n) == bd.trsm_bound(-h, h, n)
            # positive: the theorem at m = 0, M = p-1 has (p-2)^(n-1) where
            # the corollary prints (p-1)^(n-1); the printed form is looser
            assert bd.trsm_bound_positive(p, n) >= bd.trsm_bound(0, p - 1, n)
            assert bd.trsm_bound(0, p - 1, n) == \
                Fraction(p - 1, 2) * (p ** (n - 1) + (p - 2) ** (n - 1))
