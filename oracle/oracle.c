/*
 * oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * The reference against which the GPU fgemm is checked.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load this
 * library; the product path never does.  It shares no code, header or table
 * with the HIP implementation.
 *
 * What it computes is the plain definition of the operation the paper builds
 * its kernel around (Section 3, the extended product C <- alpha*A*B + beta*C
 * over Z/pZ, as in the Winograd schedule table "tab:schedule:ABC"):
 *
 *     C'[i][j] = ( alpha * sum_{l<k} a[i][l] * b[l][j]  +  beta * C[i][j] ) mod p
 *
 * with a = op(A), b = op(B) given as residues in [0, p).  Reduction modulo p
 * is a ring homomorphism from Z onto Z/pZ (Section 2.1.2), so this value is
 * unique: every correct algorithm, delayed reductions and Winograd included,
 * must return exactly these words.
 *
 * The loop takes the slow, obviously safe route: a 128-bit accumulator and a
 * reduction after every single multiply-add (no delayed reduction at all).
 * OpenMP splits the rows of C between threads; nothing else is reordered.
 *
 * Layout: row-major.  op(A) is m x k; A is m x k (lda >= k) when transA == 0,
 * k x m (lda >= m) when transA == 1.  Likewise for B (op(B) is k x n).
 * C is m x n with ldc >= n.  Return 0 on success, -1 on a bad argument.
 */
#include <stdint.h>
#include <stddef.h>

typedef unsigned __int128 u128;
typedef __int128 i128;

#ifdef ORACLE_PLANT
/* Planted-mistake builds exist only so that the test suite can show that its
 * pins catch a wrong oracle.  Each value of ORACLE_PLANT injects one mistake. */
#define PLANT(x) (ORACLE_PLANT == (x))
#else
#define PLANT(x) 0
#endif

static inline uint32_t op_elem(const uint32_t *X, int64_t ld, int trans,
                               int64_t r, int64_t c)
{
    /* element (r, c) of op(X) */
    if (PLANT(3)) trans = !trans; /* planted: transpose flag ignored/inverted */
    return trans ? X[c * ld + r] : X[r * ld + c];
}

int oracle_fgemm(uint32_t p, int transA, int transB,
                 int64_t m, int64_t n, int64_t k,
                 uint32_t alpha, const uint32_t *A, int64_t lda,
                 const uint32_t *B, int64_t ldb,
                 uint32_t beta, uint32_t *C, int64_t ldc)
{
    if (p < 2 || m < 0 || n < 0 || k < 0) return -1;
    if (m == 0 || n == 0) return 0;
    if (ldc < n) return -1;
    if (k > 0) {
        if (lda < (transA ? m : k)) return -1;
        if (ldb < (transB ? k : n)) return -1;
    }
    const u128 P = p;
    const u128 al = alpha % p, be = beta % p;

#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < m; ++i) {
        for (int64_t j = 0; j < n; ++j) {
            u128 acc = 0;
            int64_t kend = PLANT(1) ? k - 1 : k; /* planted: last term dropped */
            for (int64_t l = 0; l < kend; ++l) {
                u128 a = op_elem(A, lda, transA, i, l);
                u128 b = op_elem(B, ldb, transB, l, j);
                if (PLANT(4)) b = op_elem(B, ldb, transB, l, (j + 1) % n); /* planted: wrong column index */
                acc = (acc + a * b) % P;
            }
            u128 c = C[i * ldc + j];
            u128 r;
            if (PLANT(2))      r = (al * acc + P * P - (be * c) % P) % P; /* planted: wrong sign */
            else if (PLANT(5)) r = (acc + be * c) % P;                   /* planted: alpha dropped */
            else               r = (al * acc + be * c) % P;
            C[i * ldc + j] = (uint32_t)r;
        }
    }
    return 0;
}

/*
 * Sampled entries of the same definition, computed one by one.  Used where a
 * full product is too slow for the CPU: entry t is row ii[t], column jj[t];
 * cin[t] is the value of C at that position before the call.
 */
int oracle_fgemm_entries(uint32_t p, int transA, int transB, int64_t k,
                         uint32_t alpha, const uint32_t *A, int64_t lda,
                         const uint32_t *B, int64_t ldb, uint32_t beta,
                         int64_t nsamp, const int64_t *ii, const int64_t *jj,
                         const uint32_t *cin, uint32_t *out)
{
    if (p < 2 || k < 0 || nsamp < 0) return -1;
    const u128 P = p;
    const u128 al = alpha % p, be = beta % p;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t t = 0; t < nsamp; ++t) {
        u128 acc = 0;
        for (int64_t l = 0; l < k; ++l) {
            u128 a = op_elem(A, lda, transA, ii[t], l);
            u128 b = op_elem(B, ldb, transB, l, jj[t]);
            acc = (acc + a * b) % P;
        }
        out[t] = (uint32_t)((al * acc + be * (u128)cin[t]) % P);
    }
    return 0;
}

/*
 * Freivalds' probabilistic check of C1 == alpha*op(A)*op(B) + beta*C0 (mod p).
 * For each of the ntrials vectors x (row t of X, n residues supplied by the
 * caller) it compares C1*x with alpha*op(A)*(op(B)*x) + beta*C0*x, all mod p.
 * A wrong C1 survives one trial with probability at most 1/p.  Returns the
 * number of trials that disagree (0 = consistent), or -1 on a bad argument.
 * Cost: O(ntrials * (m*k + k*n + 2*m*n)).
 */
int oracle_freivalds(uint32_t p, int transA, int transB,
                     int64_t m, int64_t n, int64_t k,
                     uint32_t alpha, const uint32_t *A, int64_t lda,
                     const uint32_t *B, int64_t ldb, uint32_t beta,
                     const uint32_t *C0, int64_t ldc0,
                     const uint32_t *C1, int64_t ldc1,
                     int ntrials, const uint32_t *X,
                     uint32_t *work /* k + 2*m words */)
{
    if (p < 2 || m < 0 || n < 0 || k < 0 || ntrials < 0) return -1;
    const u128 P = p;
    const u128 al = alpha % p, be = beta % p;
    int bad = 0;
    uint32_t *bx = work, *y1 = work + k, *y2 = work + k + m;
    for (int t = 0; t < ntrials; ++t) {
        const uint32_t *x = X + (int64_t)t * n;
#pragma omp parallel for
        for (int64_t l = 0; l < k; ++l) {
            u128 acc = 0;
            for (int64_t j = 0; j < n; ++j)
                acc = (acc + (u128)op_elem(B, ldb, transB, l, j) * x[j]) % P;
            bx[l] = (uint32_t)acc;
        }
#pragma omp parallel for
        for (int64_t i = 0; i < m; ++i) {
            u128 s1 = 0, s0 = 0, sa = 0;
            for (int64_t j = 0; j < n; ++j) {
                s1 = (s1 + (u128)C1[i * ldc1 + j] * x[j]) % P;
                s0 = (s0 + (u128)C0[i * ldc0 + j] * x[j]) % P;
            }
            for (int64_t l = 0; l < k; ++l)
                sa = (sa + (u128)op_elem(A, lda, transA, i, l) * bx[l]) % P;
            y1[i] = (uint32_t)s1;
            y2[i] = (uint32_t)((al * sa + be * s0) % P);
        }
        for (int64_t i = 0; i < m; ++i)
            if (y1[i] != y2[i]) { ++bad; break; }
    }
    return bad;
}

/*
 * Exact integer product D = A * B of signed matrices (row-major, no
 * transposes), entries of D returned as 128-bit two's complement split in
 * (lo, hi) 64-bit words.  With |a|, |b| <= 2^30 and k <= 2^11 every sum fits
 * in 2^71, far inside 128 bits.  This is the "exact big-integer CPU product"
 * against which multi-modular results are checked after Chinese remaindering.
 */
int oracle_int_matmul(int64_t m, int64_t n, int64_t k,
                      const int64_t *A, int64_t lda,
                      const int64_t *B, int64_t ldb,
                      uint64_t *Dlo, int64_t *Dhi, int64_t ldd)
{
    if (m < 0 || n < 0 || k < 0) return -1;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < m; ++i)
        for (int64_t j = 0; j < n; ++j) {
            i128 acc = 0;
            for (int64_t l = 0; l < k; ++l)
                acc += (i128)A[i * lda + l] * (i128)B[l * ldb + j];
            Dlo[i * ldd + j] = (uint64_t)(u128)acc;
            Dhi[i * ldd + j] = (int64_t)(acc >> 64);
        }
    return 0;
}

/*
 * Chinese remaindering (Garner's mixed-radix form) of nprime residue planes
 * into the symmetric integer range (-P/2, P/2], P = prod of the primes, which
 * must stay below 2^126.  R holds nprime planes of count words each; the
 * integer of element e is returned as (lo, hi) 128-bit words.
 */
static uint64_t inv_mod(uint64_t a, uint64_t p)
{
    /* a^(p-2) mod p by square-and-multiply (p prime) */
    u128 r = 1, b = a % p;
    uint64_t e = p - 2;
    while (e) {
        if (e & 1) r = (r * b) % p;
        b = (b * b) % p;
        e >>= 1;
    }
    return (uint64_t)r;
}

int oracle_crt(int nprime, const uint32_t *primes, int64_t count,
               const uint32_t *R, uint64_t *lo, int64_t *hi)
{
    if (nprime < 1 || nprime > 6 || count < 0) return -1;
    u128 Ptot = 1;
    for (int a = 0; a < nprime; ++a) Ptot *= primes[a];
#pragma omp parallel for
    for (int64_t e = 0; e < count; ++e) {
        /* mixed-radix digits v_a with x = v_0 + v_1 p_0 + v_2 p_0 p_1 + ... */
        uint64_t v[6];
        for (int a = 0; a < nprime; ++a) {
            uint64_t pa = primes[a];
            /* value of the partial mixed-radix number modulo p_a */
            u128 t = 0, w = 1;
            for (int b = 0; b < a; ++b) {
                t = (t + (u128)v[b] * w) % pa;
                w = (w * primes[b]) % pa;
            }
            uint64_t ra = R[(int64_t)a * count + e] % pa;
            uint64_t diff = (uint64_t)((ra + pa - (uint64_t)t) % pa);
            v[a] = (uint64_t)(((u128)diff * inv_mod((uint64_t)w, pa)) % pa);
        }
        u128 x = 0, w = 1;
        for (int a = 0; a < nprime; ++a) {
            x += (u128)v[a] * w;
            w *= primes[a];
        }
        i128 s = (x > Ptot / 2) ? (i128)x - (i128)Ptot : (i128)x;
        lo[e] = (uint64_t)(u128)s;
        hi[e] = (int64_t)(s >> 64);
    }
    return 0;
}

/*
 * Triangular system with matrix right-hand side (Section 4): X such that
 *     op(T) X = alpha B   (mod p),
 * T m x m triangular (uplo 0: upper, 1: lower; trans 1: op(T) = T^T; diag 1:
 * unit diagonal, the stored diagonal is not read), B m x n, overwritten by X.
 * Plain substitution, row by row in the order the triangle allows, every
 * multiply-add reduced:
 *     x_i = (alpha b_i - sum_{l solved} op(T)_il x_l) * op(T)_ii^(-1)  mod p.
 * The inverse comes from the extended Euclidean algorithm, so any modulus
 * works as long as the diagonal entries are units.  Columns of B are
 * independent (OpenMP over them).  Returns 0, -1 on a bad argument, -2 when a
 * diagonal entry has no inverse modulo p.
 */
static int64_t inv_euclid(uint64_t a, uint64_t p)
{
    int64_t r0 = (int64_t)p, r1 = (int64_t)(a % p), s0 = 0, s1 = 1;
    while (r1 != 0) {
        const int64_t q = r0 / r1, r2 = r0 - q * r1, s2 = s0 - q * s1;
        r0 = r1; r1 = r2; s0 = s1; s1 = s2;
    }
    if (r0 != 1) return -1;
    return s0 < 0 ? s0 + (int64_t)p : s0;
}

int oracle_ftrsm(uint32_t p, int uplo, int trans, int diag, int64_t m, int64_t n,
                 uint32_t alpha, const uint32_t *T, int64_t ldt, uint32_t *B, int64_t ldb)
{
    if (p < 2 || m < 0 || n < 0) return -1;
    if ((uplo != 0 && uplo != 1) || (trans != 0 && trans != 1) || (diag != 0 && diag != 1))
        return -1;
    if (m == 0 || n == 0) return 0;
    if (ldt < m || ldb < n) return -1;
    const u128 P = p;
    /* op(T) is lower triangular when exactly one of (lower, transposed) holds */
    const int lower = uplo ^ trans;
    int64_t bad = 0;
    if (!diag) {
        for (int64_t i = 0; i < m; ++i)
            if (inv_euclid(T[i * ldt + i], p) < 0) bad = 1;
        if (bad) return -2;
    }
    const u128 al = alpha % p;
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < n; ++j) {
        for (int64_t s = 0; s < m; ++s) {
            const int64_t i = lower ? s : m - 1 - s;
            u128 acc = (al * B[i * ldb + j]) % P;
            for (int64_t t = 0; t < s; ++t) {
                const int64_t l = lower ? t : m - 1 - t;
                const u128 til = op_elem(T, ldt, trans, i, l) % P;
                acc = (acc + (P - til) * B[l * ldb + j]) % P;
            }
            if (!diag && !PLANT(6)) /* planted: diagonal division skipped */
                acc = (acc * (u128)inv_euclid(op_elem(T, ldt, trans, i, i), p)) % P;
            B[i * ldb + j] = (uint32_t)acc;
        }
    }
    return 0;
}

/* LQUP factorisation (Section 5.1, the triangularisation of Ibarra, Moran
 * and Hui): A = L Q U P with L m x m unit lower triangular, Q and P
 * permutations and U m x n upper triangular whose first r = rank(A) rows are
 * nonzero.  Section 6 reads the rank off U (its nonzero rows) and the
 * determinant as the product of U's diagonal.
 *
 * Pivots are taken row by row, in order.  Row i, already reduced by every
 * pivot found above it, pivots on its first nonzero entry among the columns
 * not used by a pivot yet; that column is brought to position k (the index
 * of the new pivot) by exchanging two whole columns.  The rows below are then
 * reduced: row i2 gets the multiplier f = A[i2][k] / A[i][k], stored at
 * A[i2][k], and loses f times row i on the columns after k.  A row with no
 * nonzero entry left is dependent: it takes no pivot.
 *
 * Storage (compressed, in place, as the paper's implementation keeps L): row
 * i keeps its position; with k_i pivots found above it, A[i][j] for j < k_i
 * is row i's multiplier on pivot j, and A[i][j] for j >= k_i holds U's row
 * (pivot rows, the pivot itself at j = k_i) or 0 (dependent rows), columns in
 * the permuted order.  pivrows[0..r) lists the pivot rows in order and
 * pivrows[r..m) the dependent rows in increasing order; colperm[j] is the
 * input column now at position j.  With both, A[:, colperm] = L * (QU) where
 * (QU)[pivrows[k]] = U's row k.
 *
 * Returns 0; -1 on a bad argument; -2 when a nonzero pivot has no inverse
 * modulo p (p not prime).
 */
int oracle_lqup(uint32_t p, int64_t m, int64_t n, uint32_t *A, int64_t lda, int64_t *rank,
                int64_t *pivrows, int64_t *colperm)
{
    if (p < 2 || m < 0 || n < 0 || (m > 0 && n > 0 && lda < n)) return -1;
    const u128 P = p;
    for (int64_t j = 0; j < n; ++j) colperm[j] = j;
    int64_t k = 0;
    for (int64_t i = 0; i < m; ++i) {
        uint32_t *ri = A + i * lda;
        int64_t c = -1;
        for (int64_t j = k; j < n; ++j)
            if (ri[j]) { c = j; break; }
        if (c < 0) continue; /* dependent row */
        if (c != k) {
            for (int64_t r = 0; r < m; ++r) {
                uint32_t *row = A + r * lda;
                const uint32_t t = row[k]; row[k] = row[c]; row[c] = t;
            }
            const int64_t t = colperm[k]; colperm[k] = colperm[c]; colperm[c] = t;
        }
        const int64_t inv = inv_euclid(ri[k], p);
        if (inv < 0) return -2;
        /* the rows below the pivot are updated independently of each other */
#pragma omp parallel for schedule(static) if ((m - i) * (n - k) > (1 << 16))
        for (int64_t i2 = i + 1; i2 < m; ++i2) {
            uint32_t *r2 = A + i2 * lda;
            const u128 f = ((u128)r2[k] * (u128)inv) % P;
            r2[k] = (uint32_t)f;
            if (f == 0) continue;
            /* planted: the column right after the pivot is not reduced */
            for (int64_t j = PLANT(7) ? k + 2 : k + 1; j < n; ++j)
                r2[j] = (uint32_t)((r2[j] + (P - f) * ri[j]) % P);
        }
        pivrows[k++] = i;
    }
    *rank = k;
    /* dependent rows, in increasing order, after the pivot rows */
    int64_t d = k;
    for (int64_t i = 0, q = 0; i < m; ++i) {
        if (q < k && pivrows[q] == i) { ++q; continue; }
        pivrows[d++] = i;
    }
    return 0;
}
