"""Pins of the oracle's LQUP factorisation, rank and determinant.

LQUP (Section 5.1) is not unique in general; under the pivoting rule the
oracle states (rows in order, first nonzero column not yet used) it is, and
the hand-worked fixtures pin that rule.  Everything else is checked against
what the factorisation must satisfy whatever the implementation: the factors
rebuild the matrix (through the independently pinned fgemm oracle), rank and
determinant agree with brute force (minors, Leibniz) on every small matrix
over Z/2 and Z/3, matrices of constructed rank have that rank, and the
determinant is multiplicative.
"""
import itertools

import numpy as np
import pytest

import oracle
from golden_io import lqup_hand
from paper_cs_0601133_amd import synth


def leibniz(p, A):
    n = A.shape[0]
    d = 0
    for perm in itertools.permutations(range(n)):
        t = oracle.permutation_sign(perm)
        for i in range(n):
            t *= int(A[i, perm[i]])
        d += t
    return d % p


def brute_rank(p, A):
    m, n = A.shape
    for r in range(min(m, n), 0, -1):
        for rows in itertools.combinations(range(m), r):
            for cols in itertools.combinations(range(n), r):
                if leibniz(p, A[np.ix_(rows, cols)]) != 0:
                    return r
    return 0


def check_factorisation(p, A, F, rank, piv, perm):
    """The compressed factors rebuild A and have the stated structure."""
    m, n = A.shape
    assert sorted(piv) == list(range(m)) and sorted(perm) == list(range(n))
    assert list(piv[rank:]) == sorted(piv[rank:])
    assert list(piv[:rank]) == sorted(piv[:rank])
    L, QU = oracle.lqup_factors(p, F, rank, piv)
    k = 0
    for i in range(m):
        if k < rank and piv[k] == i:
            assert F[i, k] != 0            # the pivot
            k += 1
        else:
            assert not F[i, k:].any()       # dependent row: nothing after the multipliers
    return np.array_equal(A[:, perm], oracle.fgemm(p, L, QU))


def test_hand_examples():
    for c in lqup_hand():
        p = c["p"]
        F, r, piv, perm = oracle.lqup(p, c["A"])
        assert np.array_equal(F, c["F"]), p
        assert r == c["rank"] and list(piv) == c["pivrows"] and list(perm) == c["colperm"]
        if "det" in c:
            assert oracle.det(p, c["A"]) == c["det"]


def known_rank(p, m, n, r, seed):
    """A = X Y with X = [I_r; R1] (rows shuffled) and Y = [I_r R2] (columns
    shuffled): X has full column rank and Y full row rank, so rank(A) = r
    exactly (Sylvester's inequality)."""
    rng = np.random.default_rng(seed)
    X = np.zeros((m, r), np.uint32)
    Y = np.zeros((r, n), np.uint32)
    X[:r] = np.eye(r, dtype=np.uint32)
    X[r:] = synth.residues(synth.seed_for(seed, 1), (m - r, r), p)
    Y[:, :r] = np.eye(r, dtype=np.uint32)
    Y[:, r:] = synth.residues(synth.seed_for(seed, 2), (r, n - r), p)
    X = X[rng.permutation(m)]
    Y = Y[:, rng.permutation(n)]
    return oracle.fgemm(p, np.ascontiguousarray(X), np.ascontiguousarray(Y))


@pytest.mark.parametrize("p", [2, 3, 7, 65521, 8388593, 2147483647])
def test_factors_rebuild_the_matrix(p):
    shapes = [(1, 1), (1, 5), (5, 1), (6, 6), (9, 14), (14, 9), (40, 40)]
    for si, (m, n) in enumerate(shapes):
        A = synth.residues(synth.seed_for(110 + si, 1), (m, n), p)
        F, r, piv, perm = oracle.lqup(p, A)
        assert check_factorisation(p, A, F, r, piv, perm), (m, n)
        for rr in sorted({0, 1, min(m, n) // 2, min(m, n)}):
            Ak = known_rank(p, m, n, rr, 120 + si)
            F, r, piv, perm = oracle.lqup(p, Ak)
            assert r == rr, (m, n, rr)
            assert check_factorisation(p, Ak, F, r, piv, perm), (m, n, rr)


def test_zero_and_empty_matrices():
    for m, n in ((3, 4), (4, 3)):
        F, r, piv, perm = oracle.lqup(7, np.zeros((m, n), np.uint32))
        assert r == 0 and list(piv) == list(range(m)) and list(perm) == list(range(n))
        assert not F.any()
    F, r, piv, perm = oracle.lqup(7, np.zeros((0, 3), np.uint32))
    assert r == 0 and F.shape == (0, 3)


@pytest.mark.parametrize("p,m,n", [(2, 2, 2), (3, 2, 2), (2, 2, 3), (2, 3, 3), (3, 3, 3)])
def test_rank_and_det_against_brute_force(p, m, n):
    # every m x n matrix over Z/p (3 x 3 over Z/3: all 19683)
    for vals in itertools.product(range(p), repeat=m * n):
        A = np.array(vals, np.uint32).reshape(m, n)
        F, r, piv, perm = oracle.lqup(p, A)
        assert r == brute_rank(p, A), A
        if m == n:
            assert oracle.det(p, A) == leibniz(p, A), A


def test_det_is_multiplicative():
    p, n = 65521, 40
    A = synth.residues(synth.seed_for(130, 1), (n, n), p)
    B = synth.residues(synth.seed_for(130, 2), (n, n), p)
    dA, dB = oracle.det(p, A), oracle.det(p, B)
    assert dA and dB
    assert oracle.det(p, oracle.fgemm(p, A, B)) == dA * dB % p
    S = known_rank(p, n, n, n - 1, 131)
    assert oracle.det(p, S) == 0
    assert oracle.det(p, oracle.fgemm(p, A, S)) == 0


def test_det_of_triangular_and_permutation_matrices():
    p, n = 8388593, 12
    T = np.triu(synth.residues(synth.seed_for(132, 1), (n, n), p))
    np.fill_diagonal(T, [3 + 5 * i for i in range(n)])
    want = 1
    for i in range(n):
        want = want * (3 + 5 * i) % p
    assert oracle.det(p, T) == want
    assert oracle.det(p, np.ascontiguousarray(T.T)) == want
    for seed in range(5):
        perm = np.random.default_rng(seed).permutation(n)
        Pm = np.eye(n, dtype=np.uint32)[perm]
        assert oracle.det(p, Pm) == (1 if oracle.permutation_sign(perm) > 0 else p - 1)


def test_composite_modulus():
    # modulo 15, a pivot 5 is nonzero but not a unit
    with pytest.raises(ZeroDivisionError):
        oracle.lqup(15, np.array([[5, 1], [1, 1]], np.uint32))
    A = np.array([[7, 1, 3], [2, 4, 1]], np.uint32)
    F, r, piv, perm = oracle.lqup(15, A)
    assert r == 2 and check_factorisation(15, A, F, r, piv, perm)


def test_planted_mistake_is_caught():
    # plant 7: the column right after each pivot is not reduced
    p = 7
    A = synth.residues(synth.seed_for(133, 1), (8, 8), p)
    F, r, piv, perm = oracle.lqup(p, A, plant=7)
    assert not check_factorisation(p, A, F, r, piv, perm)


def test_inverse_of_every_2x2_over_z5_is_the_adjugate_over_the_determinant():
    # the closed form [[d, -b], [-c, a]] / (ad - bc); singular exactly when
    # ad - bc = 0 (mod 5)
    p = 5
    for a, b, c, d in itertools.product(range(p), repeat=4):
        X = oracle.inv(p, [[a, b], [c, d]])
        dt = (a * d - b * c) % p
        if dt == 0:
            assert X is None, (a, b, c, d)
            continue
        s = pow(dt, p - 2, p)
        want = np.array([[d * s % p, (-b) * s % p], [(-c) * s % p, a * s % p]], np.uint32)
        assert np.array_equal(X, want), (a, b, c, d)


@pytest.mark.parametrize("p", [2, 3, 65521, 8388593, 2147483647])
def test_inverse_is_two_sided_and_an_involution(p):
    # A X = X A = I through the fgemm oracle, inv(inv(A)) = A; A with a zero
    # leading entry needs a row exchange
    n = 37
    for s in range(4):
        A = synth.residues(synth.seed_for(700 + s, p % 1000), (n, n), p)
        A[0, 0] = 0
        X = oracle.inv(p, A)
        if X is None:
            assert oracle.lqup(p, A)[1] < n
            continue
        Z = np.zeros((n, n), np.uint32)
        eye = np.eye(n, dtype=np.uint32)
        assert np.array_equal(oracle.fgemm(p, A, X, Z), eye)
        assert np.array_equal(oracle.fgemm(p, X, A, Z), eye)
        assert np.array_equal(oracle.inv(p, X), A)


def test_inverse_special_cases():
    p = 65521
    # permutation matrix: the transpose
    perm = np.random.default_rng(3).permutation(9)
    P = np.eye(9, dtype=np.uint32)[perm]
    assert np.array_equal(oracle.inv(p, P), P.T)
    # diagonal: the entrywise inverses
    d = np.array([1, 2, 3, p - 1, 40000], np.int64)
    want = np.diag([pow(int(x), p - 2, p) for x in d]).astype(np.uint32)
    assert np.array_equal(oracle.inv(p, np.diag(d)), want)
    # singular: equal rows, a zero column, the zero matrix; 1 x 1
    A = synth.residues(synth.seed_for(710, 1), (6, 6), p)
    A[4] = A[1]
    assert oracle.inv(p, A) is None
    A = synth.residues(synth.seed_for(711, 1), (6, 6), p)
    A[:, 2] = 0
    assert oracle.inv(p, A) is None
    assert oracle.inv(p, np.zeros((3, 3), np.uint32)) is None
    assert oracle.inv(p, [[7]])[0, 0] * 7 % p == 1
