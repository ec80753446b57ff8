"""CPU oracle for fgemm -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It shares no code with the HIP implementation and never
imports it.

Contents
--------
* ``fgemm`` / ``fgemm_entries`` / ``freivalds`` / ``int_matmul`` / ``crt``:
  ctypes wrappers around ``oracle.c`` (the plain definition of
  C <- alpha*A*B + beta*C mod p, Section 3; 128-bit accumulation with a
  reduction after every multiply-add).
* ``ftrsm``: the triangular solve op(T) X = alpha B mod p of Section 4 by
  plain substitution, every multiply-add reduced.
* ``aat``: the symmetric product alpha A diag(d) A^T + beta C of Section 6
  (lower triangle, mirrored), as the definition through ``fgemm``.
* ``lqup`` / ``lqup_factors`` / ``det``: the LQUP factorisation of Section
  5.1 by plain row-by-row elimination (first nonzero column as pivot), its
  explicit factors, and the determinant read off U (Section 6).
* ``inv``: the inverse over Z/p (Section 6 lists it among the routines
  built on LQUP) as its plain definition, the unique X with A X = I,
  found by Gauss-Jordan elimination on [A | I]; None when A is singular.
* ``oracle.bounds``: the paper's accumulation and growth bounds (eq. (1),
  eq. (2), Theorem 3.1, Corollaries 3.2-3.4) in exact Python integers.
* ``oracle.winograd``: Winograd's variant in exact Python integers (the
  App. A formulas and the schedule table "tab:schedule:ABC"), with operation
  counting and intermediate-magnitude tracking.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_libs = {}

_u32p = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_u64p = np.ctypeslib.ndpointer(dtype=np.uint64, flags="C_CONTIGUOUS")
_I64 = ctypes.c_int64
_U32 = ctypes.c_uint32
_INT = ctypes.c_int


def _load(plant=None):
    key = plant
    if key in _libs:
        return _libs[key]
    path = _build.lib_path(plant)
    src = _build.SRC
    if (not os.path.exists(path)) or os.path.getmtime(path) < os.path.getmtime(src):
        _build.build(plant)
    lib = ctypes.CDLL(path)
    lib.oracle_fgemm.argtypes = [_U32, _INT, _INT, _I64, _I64, _I64, _U32,
                                 ctypes.c_void_p, _I64, ctypes.c_void_p, _I64,
                                 _U32, ctypes.c_void_p, _I64]
    lib.oracle_fgemm.restype = _INT
    lib.oracle_fgemm_entries.argtypes = [_U32, _INT, _INT, _I64, _U32,
                                         ctypes.c_void_p, _I64, ctypes.c_void_p,
                                         _I64, _U32, _I64, _i64p, _i64p, _u32p,
                                         _u32p]
    lib.oracle_fgemm_entries.restype = _INT
    lib.oracle_freivalds.argtypes = [_U32, _INT, _INT, _I64, _I64, _I64, _U32,
                                     ctypes.c_void_p, _I64, ctypes.c_void_p,
                                     _I64, _U32, ctypes.c_void_p, _I64,
                                     ctypes.c_void_p, _I64, _INT, _u32p, _u32p]
    lib.oracle_freivalds.restype = _INT
    lib.oracle_int_matmul.argtypes = [_I64, _I64, _I64, _i64p, _I64, _i64p,
                                      _I64, _u64p, _i64p, _I64]
    lib.oracle_int_matmul.restype = _INT
    lib.oracle_crt.argtypes = [_INT, _u32p, _I64, _u32p, _u64p, _i64p]
    lib.oracle_crt.restype = _INT
    lib.oracle_ftrsm.argtypes = [_U32, _INT, _INT, _INT, _I64, _I64, _U32, ctypes.c_void_p,
                                 _I64, ctypes.c_void_p, _I64]
    lib.oracle_ftrsm.restype = _INT
    lib.oracle_lqup.argtypes = [_U32, _I64, _I64, ctypes.c_void_p, _I64, ctypes.c_void_p,
                                ctypes.c_void_p, ctypes.c_void_p]
    lib.oracle_lqup.restype = _INT
    _libs[key] = lib
    return lib


def _ptr(a):
    if a is None:
        return None
    assert a.dtype == np.uint32 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.c_void_p)


def _dims(trans, X, rows_op, cols_op):
    """Leading dimension of X for op(X) of shape rows_op x cols_op."""
    if X is None or X.size == 0:
        return max(1, cols_op if not trans else rows_op)
    return X.shape[1]


def fgemm(p, A, B, C=None, alpha=1, beta=0, transA=False, transB=False,
          plant=None):
    """Return alpha*op(A)*op(B) + beta*C mod p as a new uint32 array.

    A, B, C are 2-D uint32 arrays of residues in [0, p) (C may be None when
    beta is 0).  op(X) = X.T when trans is set.
    """
    A = np.ascontiguousarray(A, dtype=np.uint32)
    B = np.ascontiguousarray(B, dtype=np.uint32)
    m = A.shape[1] if transA else A.shape[0]
    k = A.shape[0] if transA else A.shape[1]
    kb = B.shape[1] if transB else B.shape[0]
    n = B.shape[0] if transB else B.shape[1]
    if kb != k:
        raise ValueError("inner dimensions differ")
    if C is None:
        out = np.zeros((m, n), dtype=np.uint32)
    else:
        out = np.array(C, dtype=np.uint32, copy=True, order="C")
        if out.shape != (m, n):
            raise ValueError("C has the wrong shape")
    lda = max(1, A.shape[1]) if A.ndim == 2 else 1
    ldb = max(1, B.shape[1]) if B.ndim == 2 else 1
    rc = _load(plant).oracle_fgemm(int(p), int(bool(transA)), int(bool(transB)),
                                   m, n, k, int(alpha) % int(p), _ptr(A), lda,
                                   _ptr(B), ldb, int(beta) % int(p), _ptr(out),
                                   max(1, n))
    if rc != 0:
        raise ValueError(f"oracle_fgemm rejected its arguments ({rc})")
    return out


def fgemm_entries(p, A, B, rows, cols, cin=None, alpha=1, beta=0,
                  transA=False, transB=False):
    """Sampled entries (rows[t], cols[t]) of alpha*op(A)*op(B) + beta*C mod p.

    ``cin[t]`` is C at that position before the product (zeros if None)."""
    A = np.ascontiguousarray(A, dtype=np.uint32)
    B = np.ascontiguousarray(B, dtype=np.uint32)
    k = A.shape[0] if transA else A.shape[1]
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    cols = np.ascontiguousarray(cols, dtype=np.int64)
    if cin is None:
        cin = np.zeros(rows.shape[0], dtype=np.uint32)
    cin = np.ascontiguousarray(cin, dtype=np.uint32)
    out = np.zeros(rows.shape[0], dtype=np.uint32)
    rc = _load().oracle_fgemm_entries(int(p), int(bool(transA)),
                                      int(bool(transB)), k, int(alpha) % int(p),
                                      _ptr(A), A.shape[1], _ptr(B), B.shape[1],
                                      int(beta) % int(p), rows.shape[0], rows,
                                      cols, cin, out)
    if rc != 0:
        raise ValueError("oracle_fgemm_entries rejected its arguments")
    return out


def freivalds(p, A, B, C0, C1, X, alpha=1, beta=0, transA=False,
              transB=False):
    """Number of Freivalds trials (rows of X) on which C1 disagrees with
    alpha*op(A)*op(B) + beta*C0 mod p.  0 means consistent."""
    A = np.ascontiguousarray(A, dtype=np.uint32)
    B = np.ascontiguousarray(B, dtype=np.uint32)
    C0 = np.ascontiguousarray(C0, dtype=np.uint32)
    C1 = np.ascontiguousarray(C1, dtype=np.uint32)
    X = np.ascontiguousarray(X, dtype=np.uint32)
    m = A.shape[1] if transA else A.shape[0]
    k = A.shape[0] if transA else A.shape[1]
    n = B.shape[0] if transB else B.shape[1]
    work = np.zeros(k + 2 * m + 1, dtype=np.uint32)
    rc = _load().oracle_freivalds(int(p), int(bool(transA)), int(bool(transB)),
                                  m, n, k, int(alpha) % int(p), _ptr(A),
                                  A.shape[1], _ptr(B), B.shape[1],
                                  int(beta) % int(p), _ptr(C0), C0.shape[1],
                                  _ptr(C1), C1.shape[1], X.shape[0], X, work)
    if rc < 0:
        raise ValueError("oracle_freivalds rejected its arguments")
    return rc


def int_matmul(A, B):
    """Exact integer product of int64 matrices, as (lo uint64, hi int64)."""
    A = np.ascontiguousarray(A, dtype=np.int64)
    B = np.ascontiguousarray(B, dtype=np.int64)
    m, k = A.shape
    n = B.shape[1]
    lo = np.zeros((m, n), dtype=np.uint64)
    hi = np.zeros((m, n), dtype=np.int64)
    rc = _load().oracle_int_matmul(m, n, k, A, k, B, n, lo, hi, n)
    if rc != 0:
        raise ValueError("oracle_int_matmul rejected its arguments")
    return lo, hi


def crt(primes, residues):
    """Chinese remaindering of residue planes (list of equal-shape uint32
    arrays, one per prime) into symmetric integers, as (lo, hi) words."""
    primes = np.ascontiguousarray(primes, dtype=np.uint32)
    shape = residues[0].shape
    R = np.ascontiguousarray(np.stack([np.asarray(r, dtype=np.uint32).ravel()
                                       for r in residues]))
    count = R.shape[1]
    lo = np.zeros(count, dtype=np.uint64)
    hi = np.zeros(count, dtype=np.int64)
    rc = _load().oracle_crt(len(primes), primes, count, R.ravel(), lo, hi)
    if rc != 0:
        raise ValueError("oracle_crt rejected its arguments")
    return lo.reshape(shape), hi.reshape(shape)


def ftrsm(p, T, B, alpha=1, lower=False, trans=False, unit=False, plant=None):
    """X with op(T) X = alpha B (mod p), T m x m triangular (upper unless
    `lower`; op(T) = T^T if `trans`; `unit`: unit diagonal, not read), B m x n.
    Returns X (a new array).  Raises ZeroDivisionError when a diagonal entry
    has no inverse modulo p."""
    T = np.ascontiguousarray(T, dtype=np.uint32)
    X = np.array(B, dtype=np.uint32, order="C", copy=True)
    m, n = X.shape
    assert T.shape == (m, m)
    rc = _load(plant).oracle_ftrsm(p, int(lower), int(trans), int(unit), m, n, alpha,
                                    _ptr(T), max(m, 1), _ptr(X), max(n, 1))
    if rc == -2:
        raise ZeroDivisionError("a diagonal entry of T is not invertible modulo p")
    if rc != 0:
        raise ValueError("oracle_ftrsm rejected its arguments")
    return X


def lqup(p, A, plant=None):
    """LQUP of A over Z/p (Section 5.1) in the compressed in-place form
    written out in oracle.c.  Returns (F, rank, pivrows, colperm): F the
    factored matrix (a new array), pivrows the pivot rows in order followed
    by the dependent rows, colperm[j] the input column at position j.
    Raises ZeroDivisionError when a nonzero pivot has no inverse modulo p."""
    F = np.array(A, dtype=np.uint32, order="C", copy=True)
    m, n = F.shape
    rank = np.zeros(1, dtype=np.int64)
    piv = np.zeros(max(m, 1), dtype=np.int64)
    perm = np.zeros(max(n, 1), dtype=np.int64)
    rc = _load(plant).oracle_lqup(p, m, n, _ptr(F), max(n, 1), rank.ctypes.data,
                                  piv.ctypes.data, perm.ctypes.data)
    if rc == -2:
        raise ZeroDivisionError("a nonzero pivot has no inverse modulo p")
    if rc != 0:
        raise ValueError("oracle_lqup rejected its arguments")
    return F, int(rank[0]), piv[:m].copy(), perm[:n].copy()


def lqup_factors(p, F, rank, pivrows):
    """Explicit factors from the compressed form: L (m x m unit lower
    triangular, original row order) and QU (m x n: U's row k at row
    pivrows[k], zero rows elsewhere), with A[:, colperm] = L QU mod p."""
    m, n = F.shape
    L = np.eye(m, dtype=np.uint32)
    QU = np.zeros((m, n), dtype=np.uint32)
    is_piv = np.zeros(m, dtype=bool)
    is_piv[pivrows[:rank]] = True
    # pivots in the rows above row i
    above = np.concatenate(([0], np.cumsum(is_piv)[:-1]))
    prow = np.asarray(pivrows[:rank])
    for i in range(m):
        ka = int(above[i])
        L[i, prow[:ka]] = F[i, :ka]
        if is_piv[i]:
            QU[i, ka:] = F[i, ka:]
    return L, QU


def permutation_sign(perm):
    """+1 or -1: the parity of a permutation given as an index array."""
    perm = list(perm)
    seen = [False] * len(perm)
    sign = 1
    for i in range(len(perm)):
        if seen[i]:
            continue
        j, length = i, 0
        while not seen[j]:
            seen[j] = True
            j = perm[j]
            length += 1
        if length % 2 == 0:
            sign = -sign
    return sign


def det(p, A, plant=None):
    """Determinant of a square A over Z/p (Section 6): 0 below full rank,
    else the product of U's diagonal times the sign of the column
    permutation (every row is then a pivot row, in order)."""
    F, r, piv, perm = lqup(p, A, plant)
    n = F.shape[0]
    if r < n:
        return 0
    d = 1
    for k in range(n):
        d = d * int(F[k, k]) % p
    return d if permutation_sign(perm) > 0 else (p - d) % p


def inv(p, A):
    """A^-1 over Z/p for a square A (p prime), or None when A is singular.
    Gauss-Jordan on [A | I]: for each column take the first row at or below
    the diagonal with a nonzero entry, exchange it into place, scale it to a
    unit pivot and clear the column in every other row.  This is not the
    LQUP route the library takes; only the result (unique) is shared."""
    A = np.asarray(A, dtype=np.int64) % p
    n = A.shape[0]
    if A.shape != (n, n):
        raise ValueError("square matrix expected")
    M = np.concatenate([A, np.eye(n, dtype=np.int64)], axis=1)
    for c in range(n):
        nz = np.nonzero(M[c:, c])[0]
        if nz.size == 0:
            return None
        r = c + int(nz[0])
        if r != c:
            M[[c, r]] = M[[r, c]]
        M[c] = M[c] * pow(int(M[c, c]), p - 2, p) % p
        f = M[:, c].copy()
        f[c] = 0
        # entries < p < 2^31, so every product fits in int64
        M = (M - (f[:, None] * M[c][None, :]) % p) % p
    return M[:, n:].astype(np.uint32)


def aat(p, A, d=None, alpha=1, beta=0, C=None):
    """Symmetric product of Section 6: the lower triangle (i >= j) of
    alpha A diag(d) A^T + beta C mod p, mirrored into the upper triangle
    (d None: the identity; C None: zeros).  Written as the definition
    through fgemm with op(B) = (A diag(d))^T."""
    A = np.ascontiguousarray(A, dtype=np.uint32)
    m, k = A.shape
    if d is None:
        AD = A
    else:
        dd = np.asarray(d, dtype=np.uint64).reshape(1, k)
        AD = np.ascontiguousarray((A.astype(np.uint64) * dd % p).astype(np.uint32))
    C0 = np.zeros((m, m), np.uint32) if C is None else np.array(C, dtype=np.uint32)
    R = fgemm(p, A, AD, C0, alpha, beta, transB=True)
    return np.tril(R) + np.tril(R, -1).T
