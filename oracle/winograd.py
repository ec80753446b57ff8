"""Winograd's variant of Strassen's algorithm in exact Python integers.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).  Small sizes only
(pure-Python loops).  Every function works on lists of lists of ints and, if
given a ``Tracker``, counts scalar field operations and records the largest
magnitude of every intermediate value, so that Table "tab:winolevel" and
Theorem 3.1 (with its optimality construction) can be checked.

Two evaluation orders are provided, both from Appendix A's definitions:
* ``winograd_mul``: C = A*B through the seven products and fifteen block
  additions S1..S4, T1..T4, P1..P7, U1..U7.
* ``winograd_abc_appendix``: A*B + beta*C with the beta*C terms folded into
  four of the products, the evaluation Theorem 3.1 bounds.
Appendix A defines P4 as A22*T4; the alpha/beta schedule table of Section
3.2.2 prints A12 in that step, which a test shows cannot be right.
"""


class Tracker:
    def __init__(self):
        self.ops = 0
        self.max_abs = 0

    def see(self, x):
        a = abs(x)
        if a > self.max_abs:
            self.max_abs = a
        return x


def _shape(X):
    return len(X), (len(X[0]) if X else 0)


def _block(X, r0, r1, c0, c1):
    return [row[c0:c1] for row in X[r0:r1]]


def _add(X, Y, tr, sign=1):
    out = []
    for rx, ry in zip(X, Y):
        row = []
        for a, b in zip(rx, ry):
            v = a + b if sign > 0 else a - b
            if tr:
                tr.ops += 1
                tr.see(v)
            row.append(v)
        out.append(row)
    return out


def _scale(X, s, tr):
    out = []
    for rx in X:
        row = []
        for a in rx:
            v = s * a
            if tr:
                tr.ops += 1
                tr.see(v)
            row.append(v)
        out.append(row)
    return out


def classic(A, B, tr=None):
    """Classic product: each entry is a dot product summed left to right
    (n multiplications and n-1 additions per entry)."""
    m, k = _shape(A)
    n = len(B[0]) if B else 0
    C = []
    for i in range(m):
        row = []
        for j in range(n):
            acc = A[i][0] * B[0][j] if k else 0
            if tr and k:
                tr.ops += 1
                tr.see(acc)
            for l in range(1, k):
                acc = acc + A[i][l] * B[l][j]
                if tr:
                    tr.ops += 2
                    tr.see(A[i][l] * B[l][j])
                    tr.see(acc)
            row.append(acc)
        C.append(row)
    return C


def _split(X):
    r, c = _shape(X)
    h, w = r // 2, c // 2
    return (_block(X, 0, h, 0, w), _block(X, 0, h, w, c),
            _block(X, h, r, 0, w), _block(X, h, r, w, c))


def _join(C11, C12, C21, C22):
    return [a + b for a, b in zip(C11, C12)] + [a + b for a, b in zip(C21, C22)]


def winograd_mul(A, B, l, tr=None):
    """C = A*B with l recursive levels of Winograd's algorithm (even
    dimensions at every level are required; see ``winograd_mul_peeled``)."""
    m, k = _shape(A)
    n = len(B[0]) if B else 0
    if l == 0:
        return classic(A, B, tr)
    if m % 2 or k % 2 or n % 2:
        raise ValueError("odd dimension; use winograd_mul_peeled")
    A11, A12, A21, A22 = _split(A)
    B11, B12, B21, B22 = _split(B)
    S1 = _add(A21, A22, tr)
    S2 = _add(S1, A11, tr, -1)
    S3 = _add(A11, A21, tr, -1)
    S4 = _add(A12, S2, tr, -1)
    T1 = _add(B12, B11, tr, -1)
    T2 = _add(B22, T1, tr, -1)
    T3 = _add(B22, B12, tr, -1)
    T4 = _add(T2, B21, tr, -1)
    P1 = winograd_mul(A11, B11, l - 1, tr)
    P2 = winograd_mul(A12, B21, l - 1, tr)
    P3 = winograd_mul(S4, B22, l - 1, tr)
    P4 = winograd_mul(A22, T4, l - 1, tr)
    P5 = winograd_mul(S1, T1, l - 1, tr)
    P6 = winograd_mul(S2, T2, l - 1, tr)
    P7 = winograd_mul(S3, T3, l - 1, tr)
    U1 = _add(P1, P2, tr)
    U2 = _add(P1, P6, tr)
    U3 = _add(U2, P7, tr)
    U4 = _add(U2, P5, tr)
    U5 = _add(U4, P3, tr)
    U6 = _add(U3, P4, tr, -1)
    U7 = _add(U3, P5, tr)
    return _join(U1, U5, U6, U7)


def winograd_mul_peeled(A, B, l, tr=None):
    """Dynamic peeling (Appendix A, case of an arbitrary k): at each level the
    largest even top-left blocks go through Winograd's algorithm and the odd
    leftovers are added by thin products (a rank-one update for an odd k, a
    row and a column for odd m and n)."""
    m, k = _shape(A)
    n = len(B[0]) if B else 0
    if l == 0 or m < 2 or k < 2 or n < 2:
        return classic(A, B, tr)
    me, ke, ne = m - m % 2, k - k % 2, n - n % 2
    Ae = _block(A, 0, me, 0, ke)
    Be = _block(B, 0, ke, 0, ne)
    # recurse with peeling inside the Winograd step
    A11, A12, A21, A22 = _split(Ae)
    B11, B12, B21, B22 = _split(Be)
    S1 = _add(A21, A22, tr)
    S2 = _add(S1, A11, tr, -1)
    S3 = _add(A11, A21, tr, -1)
    S4 = _add(A12, S2, tr, -1)
    T1 = _add(B12, B11, tr, -1)
    T2 = _add(B22, T1, tr, -1)
    T3 = _add(B22, B12, tr, -1)
    T4 = _add(T2, B21, tr, -1)
    rec = winograd_mul_peeled
    P1 = rec(A11, B11, l - 1, tr)
    P2 = rec(A12, B21, l - 1, tr)
    P3 = rec(S4, B22, l - 1, tr)
    P4 = rec(A22, T4, l - 1, tr)
    P5 = rec(S1, T1, l - 1, tr)
    P6 = rec(S2, T2, l - 1, tr)
    P7 = rec(S3, T3, l - 1, tr)
    U1 = _add(P1, P2, tr)
    U2 = _add(P1, P6, tr)
    U3 = _add(U2, P7, tr)
    U4 = _add(U2, P5, tr)
    U5 = _add(U4, P3, tr)
    U6 = _add(U3, P4, tr, -1)
    U7 = _add(U3, P5, tr)
    Ce = _join(U1, U5, U6, U7)
    if k != ke:   # rank-one update with the last column of A / row of B
        R1 = classic(_block(A, 0, me, ke, k), _block(B, ke, k, 0, ne), tr)
        Ce = _add(Ce, R1, tr)
    C = [row + [0] * (n - ne) for row in Ce] + [[0] * n for _ in range(m - me)]
    if n != ne:   # last column of C
        col = classic(_block(A, 0, me, 0, k), _block(B, 0, k, ne, n), tr)
        for i in range(me):
            C[i][ne] = col[i][0]
    if m != me:   # last row of C
        row = classic(_block(A, me, m, 0, k), B, tr)
        C[me] = row[0]
    return C


def winograd_abc_appendix(A, B, C, beta, l, tr=None):
    """A*B + beta*C with l levels, the beta*C terms folded into the products
    P2, P4, P5, P7 as in Appendix A's list of intermediate computations; this
    is the evaluation Theorem 3.1 bounds.  At l = 0 the classic product plus
    beta*C."""
    m, k = _shape(A)
    n = len(B[0]) if B else 0
    if l == 0:
        P = classic(A, B, tr)
        return _add(P, _scale(C, beta, tr), tr)
    A11, A12, A21, A22 = _split(A)
    B11, B12, B21, B22 = _split(B)
    C11, C12, C21, C22 = _split(C)
    z = [[0] * (n // 2) for _ in range(m // 2)]
    S1 = _add(A21, A22, tr)
    S2 = _add(S1, A11, tr, -1)
    S3 = _add(A11, A21, tr, -1)
    S4 = _add(A12, S2, tr, -1)
    T1 = _add(B12, B11, tr, -1)
    T2 = _add(B22, T1, tr, -1)
    T3 = _add(B22, B12, tr, -1)
    T4 = _add(T2, B21, tr, -1)
    c4 = _add(_add(C22, C12, tr, -1), C21, tr, -1)
    c7 = _add(C22, C12, tr, -1)
    rec = winograd_abc_appendix
    P1 = rec(A11, B11, z, 0, l - 1, tr)
    P2 = rec(A12, B21, C11, beta, l - 1, tr)
    P3 = rec(S4, B22, z, 0, l - 1, tr)
    P4 = rec(A22, T4, c4, beta, l - 1, tr)
    P5 = rec(S1, T1, C12, beta, l - 1, tr)
    P6 = rec(S2, T2, z, 0, l - 1, tr)
    P7 = rec(S3, T3, c7, beta, l - 1, tr)
    U1 = _add(P1, P2, tr)
    U2 = _add(P1, P6, tr)
    U3 = _add(U2, P7, tr)
    U4 = _add(U2, P5, tr)
    U5 = _add(U4, P3, tr)
    U6 = _add(U3, P4, tr, -1)
    U7 = _add(U3, P5, tr)
    return _join(U1, U5, U6, U7)


def optimal_pair(l, mA, MA, mB, MB):
    """The matrices A_l, B_l of order 2^l from Appendix A ("Optimality of the
    bound"): A_1 = [[mA, 0], [MA, MA]], B_1 = [[MB, mB], [0, MB]],
    A_{l+1} = [[bar(A_l), 0], [A_l, A_l]], B_{l+1} = [[B_l, bar(B_l)], [0, B_l]]
    with bar(x) = M + m - x."""
    A = [[mA, 0], [MA, MA]]
    B = [[MB, mB], [0, MB]]
    for _ in range(l - 1):
        h = len(A)
        Abar = [[MA + mA - x for x in row] for row in A]
        Bbar = [[MB + mB - x for x in row] for row in B]
        Z = [[0] * h for _ in range(h)]
        A = _join(Abar, Z, A, A)
        B = _join(B, Bbar, Z, B)
    return A, B
