"""Pins of the oracle's symmetric product alpha A diag(d) A^T + beta C
(Section 6: the symmetric product A x A^T with a diagonal D between the factors).

Checked against the definition evaluated in Python integers (no fgemm), the
block identity the paper's recursion rests on (splitting A's columns and d
splits the product into a sum), closed forms and symmetry.
"""
import numpy as np
import pytest

import oracle
from paper_cs_0601133_amd import synth


def exact(p, A, d, alpha, beta, C):
    m, k = A.shape
    R = np.zeros((m, m), np.uint32)
    for i in range(m):
        for j in range(i + 1):
            s = sum(int(A[i, l]) * int(d[l]) * int(A[j, l]) for l in range(k))
            v = (alpha * s + beta * int(C[i, j])) % p
            R[i, j] = R[j, i] = v
    return R


@pytest.mark.parametrize("p", [2, 7, 65521, 8388593, 2147483647])
def test_definition_in_python_integers(p):
    for si, (m, k) in enumerate([(1, 1), (3, 5), (7, 2), (12, 9)]):
        A = synth.residues(synth.seed_for(190 + si, 1), (m, k), p)
        d = synth.residues(synth.seed_for(190 + si, 2), (k,), p)
        C = synth.residues(synth.seed_for(190 + si, 3), (m, m), p)
        alpha, beta = 3 % p, (p - 1) % p
        got = oracle.aat(p, A, d, alpha, beta, C)
        assert np.array_equal(got, exact(p, A, d, alpha, beta, C)), (m, k)
        # without a diagonal: d = 1
        assert np.array_equal(oracle.aat(p, A, None, alpha), exact(p, A, [1] * k, alpha, 0,
                                                                   np.zeros((m, m), np.uint32)))


def test_block_identity_of_the_recursion():
    # [A1 A2] diag(d1, d2) [A1 A2]^T = A1 d1 A1^T + A2 d2 A2^T
    p, m, k1, k2 = 65521, 20, 13, 8
    A = synth.residues(synth.seed_for(195, 1), (m, k1 + k2), p)
    d = synth.residues(synth.seed_for(195, 2), (k1 + k2,), p)
    whole = oracle.aat(p, A, d)
    part1 = oracle.aat(p, np.ascontiguousarray(A[:, :k1]), d[:k1])
    part2 = oracle.aat(p, np.ascontiguousarray(A[:, k1:]), d[k1:])
    assert np.array_equal(whole, ((part1.astype(np.int64) + part2) % p).astype(np.uint32))


def test_closed_forms():
    p = 8388593
    A = synth.residues(synth.seed_for(196, 1), (9, 6), p)
    d = synth.residues(synth.seed_for(196, 2), (6,), p)
    R = oracle.aat(p, A, d, 5)
    assert np.array_equal(R, R.T)
    for i in range(9):
        s = sum(int(d[l]) * int(A[i, l]) ** 2 for l in range(6))
        assert R[i, i] == 5 * s % p
    # rows of the identity: A A^T = I; a zero diagonal gives 0
    E = np.eye(4, 7, dtype=np.uint32)
    assert np.array_equal(oracle.aat(p, E), np.eye(4, dtype=np.uint32))
    assert not oracle.aat(p, A, np.zeros(6, np.uint32)).any()
    # the upper triangle of C on entry does not matter
    C = synth.residues(synth.seed_for(196, 3), (9, 9), p)
    C2 = C.copy()
    C2[np.triu_indices(9, 1)] = 0
    assert np.array_equal(oracle.aat(p, A, d, 2, 3, C), oracle.aat(p, A, d, 2, 3, C2))
