/*
 * ffgemm.h -- C ABI of an MI355X (gfx950) library for exact matrix
 * multiplication over Z/pZ with word-size moduli.
 *
 * The operation is the extended product of Dumas, Giorgi and Pernet,
 * "Dense Linear Algebra over Word-Size Prime Fields: the FFLAS and FFPACK
 * packages", Section 3 (the problem C <- alpha*A*B + beta*C of the Winograd
 * schedule table "tab:schedule:ABC"):
 *
 *     C <- ( alpha * op(A) * op(B) + beta * C ) mod p.
 *
 * It is computed exactly: products are accumulated in machine arithmetic
 * (binary64 on FP64 matrix cores, or int32 on INT8 matrix cores after a
 * split of the residues into signed digits) and the reduction modulo p is
 * delayed for as long as the accumulation bound of Section 2.1.2 (eq. (1),
 * eq. (2)) allows; Winograd's variant (Section 3.2) may be applied on top,
 * within the growth bound of Theorem 3.1.  Reduction modulo p is a ring
 * homomorphism, so the result is unique and every path returns the same
 * words.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Matrices are row-major.  op(A) is m x k: with transA == FF_NOTRANS, A is
 * m x k with leading dimension lda >= k; with FF_TRANS it is k x m with
 * lda >= m.  Likewise op(B) is k x n (B is k x n, ldb >= n, or n x k,
 * ldb >= k).  C is m x n with ldc >= n.  Elements are uint32 residues in
 * [0, p); outputs are canonical residues in [0, p).  2 <= p < 2^31; p need
 * not be prime (only ring operations are used).
 *
 * A, B and C are device pointers owned by the caller (for instance the
 * storage of torch tensors); the library never frees them.  Input entries
 * must be < p: this is not checked unless ff_opts.validate is set (then an
 * out-of-range entry yields FF_EINVAL and nothing is written).  When
 * beta == 0 (mod p) C is write-only and may hold anything.
 *
 * Calls are asynchronous: the work is enqueued on a HIP stream (the one of
 * ff_set_stream, or ff_opts.stream) and the call returns; completion is
 * observed through that stream.  Work enqueued on one stream runs in order;
 * two calls on different streams must not share output memory.
 *
 * Errors are returned as ff_status codes; no entry point aborts or exits,
 * and on error nothing is enqueued.  ff_last_error() gives a description of
 * the last failure of the calling thread.
 */
#ifndef FFGEMM_H
#define FFGEMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FF_OK = 0,
    FF_EINVAL = -1,        /* bad argument (dimension, leading dimension, p, null pointer, entry >= p) */
    FF_EUNSUPPORTED = -2,  /* valid, but the requested path cannot compute it exactly */
    FF_ENOMEM = -3,        /* workspace allocation failed */
    FF_EHIP = -4,          /* a HIP runtime call failed */
    FF_EBUSY = -5,         /* a server request can never fit its memory budget */
    FF_ENOTFOUND = -6      /* unknown request id */
} ff_status;

enum { FF_NOTRANS = 0, FF_TRANS = 1 };
enum { FF_UPPER = 0, FF_LOWER = 1 };   /* triangle of T that ff_ftrsm reads  */
enum { FF_NONUNIT = 0, FF_UNIT = 1 };  /* diagonal of T: stored, or all ones */

/* Arithmetic path.  FP64: centered residues as doubles on FP64 matrix
 * cores, reduction every kblock products (Section 2.1.2, eq. (2), read with
 * the binary64 exactness limit 2^53).  INT8: centered residues split into
 * signed digits, digit products on INT8 matrix cores with int32 sums,
 * recombined modulo p in the epilogue. */
enum { FF_PATH_AUTO = 0, FF_PATH_FP64 = 1, FF_PATH_INT8 = 2 };

/* Environment (read per call; none is needed):
 *   FF_WINOGRAD_W   single crossover order for the automatic Winograd levels
 *   FF_WINO_FUSED   0: keep the last level of pre-additions apart from the
 *                   leaves' slicing/packing
 *   FF_F64_SMALL    0: never, 1: always use the one-launch FP64 kernel (else
 *                   by size)
 *   FF_I8_TILE, FF_F64_TILE   force an INT8 / FP64 tile configuration id
 *   FF_TRSM_LEAF    rows per ftrsm leaf launch (64..512, a multiple of 64)
 *   FF_LQUP_BLOCK   rows of the recursion nodes that ff_flqup's full-rank
 *                   path factors panel by panel (a multiple of 64; default:
 *                   the largest whose first panel launch fits the CUs)
 *   FF_TUNE_CACHE   autotuner cache file (see ff_autotune)
 * Every setting gives the same results; only speed changes. */

typedef struct ff_opts {
    int path;            /* FF_PATH_*.  FF_PATH_AUTO takes INT8, except that a
                            single product small enough for the one-launch FP64
                            kernel (m*n <= 512^2, k <= 768; FF_F64_SMALL=0 never,
                            =1 always) runs on FP64 when no digit width is set
                            and the FP64 K-block allows p                          */
    int winograd_levels; /* 0..3 recursive levels of Winograd's variant (Section
                            3.2); -1: automatic, Section 3.2.1's rule with measured
                            crossover orders: a first level at min(m, n, k) >=
                            w_first and one more per halving while the leaf order
                            stays >= w_next, by path and digit count (INT8, one
                            digit: none; INT8 below p = 2^30: 3072, 12288; INT8
                            above: 8192, 24576; FP64: 3072, 3072).  FF_WINOGRAD_W=w
                            sets w_first = w_next = w, i.e. the paper's
                            l = floor(log2(n/w)) + 1 clamped at 0.  The last level
                            of pre-additions is fused into the leaves' operand
                            preparation (FF_WINO_FUSED=0 keeps them apart)         */
    int digit_bits;      /* INT8 path digit width, 7 or 8; 0: automatic            */
    int validate;        /* nonzero: check that inputs are residues < p first
                            (makes the call synchronous)                           */
    int preadd_mode;     /* Winograd pre-additions: 0 automatic; 1 delayed (kept as
                            unreduced integers, the form Theorem 3.1 bounds); 2
                            reduced to centered residues at the leaves             */
    void *stream;        /* hipStream_t to enqueue on; NULL: the ff_set_stream one */
    int digit_pairing;   /* INT8 path with 7-bit digits, plain products (no
                            Winograd level; automatic levels become none): the
                            cross terms a_i b_j + a_j b_i come from one product
                            of digit sums, (a_i + a_j)(b_i + b_j) - a_i b_i
                            - a_j b_j (Karatsuba's identity per pair of digits;
                            sums of two 7-bit digits fit int8), so S(S+1)/2
                            digit products replace S^2 at the cost of S(S+1)/2
                            planes per operand instead of S.  0: off           */
} ff_opts;

/* What a call will do (ff_plan_query).  Host-only; no device is touched. */
typedef struct ff_plan_info {
    int path;                /* FF_PATH_FP64 or FF_PATH_INT8                        */
    int winograd_levels;     /* levels actually applied                             */
    int preadds_reduced;     /* 1 if Winograd leaf operands are reduced mod p       */
    int digit_bits;          /* INT8: 7 or 8; FP64: 0                               */
    int slices;              /* INT8: digits per operand; FP64: 0                   */
    int64_t operand_lo;      /* range of the values entering the products: the      */
    int64_t operand_hi;      /*  centered residues, widened by Winograd pre-additions */
    int64_t max_abs_product; /* bound on one product term |a*b| at the leaves       */
    int64_t kblock;          /* FP64: products summed between two reductions;
                                INT8: largest K of one exact int32 pass             */
    int64_t workspace_bytes; /* device workspace the call needs                     */
    int tile_config;         /* kernel tile configuration id (-1: the digit-pairing
                                kernel, which has one configuration per S)          */
    int digit_products;      /* INT8: digit-plane products per K step (S^2, or
                                S(S+1)/2 with digit pairing); FP64: 0               */
} ff_plan_info;

/* One fgemm of a batch or a server request: same meaning as the arguments
 * of ff_fgemm. */
typedef struct ff_job {
    uint32_t p;
    int transA, transB;
    int64_t m, n, k;
    uint32_t alpha, beta;
    const uint32_t *A;
    int64_t lda;
    const uint32_t *B;
    int64_t ldb;
    uint32_t *C;
    int64_t ldc;
} ff_job;

/* Checks that a gfx950 device is current and sets up per-device state,
 * including the device address of ff_fgemm_noalloc's scratch array.
 * Optional: every entry point initialises lazily. */
int ff_init(void);

/* Releases the library's device workspaces and cached plans. */
int ff_finalize(void);

/* Sets the stream later calls enqueue on (hipStream_t; NULL = null stream),
 * for the calling thread. */
int ff_set_stream(void *hip_stream);

/* C <- (alpha*op(A)*op(B) + beta*C) mod p, automatic path (Section 3).
 * BLAS quick returns: m == 0 or n == 0 does nothing; k == 0 or
 * alpha == 0 (mod p) gives C <- beta*C mod p. */
int ff_fgemm(uint32_t p, int transA, int transB,
             int64_t m, int64_t n, int64_t k,
             uint32_t alpha, const uint32_t *A, int64_t lda,
             const uint32_t *B, int64_t ldb,
             uint32_t beta, uint32_t *C, int64_t ldc);

/* Same, with explicit options (NULL opts = automatic). */
int ff_fgemm_ex(uint32_t p, int transA, int transB,
                int64_t m, int64_t n, int64_t k,
                uint32_t alpha, const uint32_t *A, int64_t lda,
                const uint32_t *B, int64_t ldb,
                uint32_t beta, uint32_t *C, int64_t ldc,
                const ff_opts *opts);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the plain
 * product of ff_fgemm_ex, same arguments, semantics and results, with its
 * scratch (digit planes of the INT8 path, packed operands and split-K
 * partials of the FP64 path, the validate counter) in a static device array
 * of FF_NOALLOC_SCRATCH_BYTES instead of library-allocated workspace.  Each
 * device holds its own copy of the array from its first use (ff_init on
 * that device, else the first call there) until the process ends.  No
 * hipMalloc, hipFree or allocating library call is made.
 * Limits: no Winograd levels (automatic means none; opts->winograd_levels
 * > 0 returns FF_EUNSUPPORTED); a product whose workspace exceeds the array
 * (ff_plan_query with winograd_levels = 0 reports workspace_bytes; e.g.
 * 4096^3 fits on the INT8 path, not on the FP64 path) returns FF_EINVAL and
 * enqueues nothing.  Every call on one device shares that device's array
 * and leaves its contents behind: calls on one stream are ordered and safe,
 * calls that overlap on one device (other streams, other threads) race and
 * give wrong results.  Call ff_init on each device first so that no call
 * loads the array. */
#define FF_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)
int ff_fgemm_noalloc(uint32_t p, int transA, int transB,
                     int64_t m, int64_t n, int64_t k,
                     uint32_t alpha, const uint32_t *A, int64_t lda,
                     const uint32_t *B, int64_t ldb,
                     uint32_t beta, uint32_t *C, int64_t ldc,
                     const ff_opts *opts);

/* Triangular system with matrix right-hand side (Section 4):
 *
 *     B <- X  with  op(T) X = alpha B   (mod p).
 *
 * T is m x m with leading dimension ldt >= m; only the triangle named by
 * uplo (FF_UPPER or FF_LOWER) is read, and with diag == FF_UNIT not its
 * diagonal either (taken as ones).  op(T) = T (FF_NOTRANS) or T^T
 * (FF_TRANS).  B is m x n with ldb >= n and is overwritten by X; T and B
 * are device pointers owned by the caller and must not overlap.  With
 * FF_NONUNIT every diagonal entry must be invertible modulo p (any unit
 * when p is prime): otherwise the result is unspecified, unless
 * opts->validate is set, which checks B's entries and T's diagonal first
 * (synchronously) and returns FF_EINVAL without writing.  The solve is the
 * block recursive algorithm of Section 4.1 on the unit triangular system
 * D^-1 op(T) X = alpha D^-1 B of Section 4.2 (D the diagonal of op(T));
 * its updates are fgemm calls that follow opts->path, and its leaves (up
 * to 512 rows) are solved on the device with the inverses of the 64 x 64
 * diagonal blocks, exactly for every p.  m == 0 or n == 0 does nothing;
 * alpha == 0 (mod p) gives B <- 0.  Workspace: 4 mp^2 + 256 mp bytes
 * (mp = m rounded up to a multiple of 64) held by the library per stream,
 * besides the fgemm workspace. */
int ff_ftrsm(uint32_t p, int uplo, int transT, int diag, int64_t m, int64_t n,
             uint32_t alpha, const uint32_t *T, int64_t ldt, uint32_t *B, int64_t ldb);

/* Same, with explicit options (NULL opts = automatic). */
int ff_ftrsm_ex(uint32_t p, int uplo, int transT, int diag, int64_t m, int64_t n,
                uint32_t alpha, const uint32_t *T, int64_t ldt, uint32_t *B, int64_t ldb,
                const ff_opts *opts);

/* LQUP factorisation (Section 5.1): A = L Q U P over Z/pZ, p prime, with
 * L m x m unit lower triangular, Q and P permutations and U m x n upper
 * triangular whose first r = rank(A) rows are nonzero.
 *
 * A (device, m x n row-major, lda >= n, entries residues < p) is overwritten
 * by the compressed form: row i keeps its position; with k_i pivots in the
 * rows above it, A[i][j] for j < k_i is row i's multiplier on pivot j (L),
 * and A[i][j] for j >= k_i is U's row (a pivot row, pivot at j = k_i) or 0
 * (a dependent row), columns in the permuted order.  Pivots are chosen row
 * by row, each row on its first nonzero entry among the columns no pivot
 * uses yet (brought into place by exchanging two whole columns), so the
 * result is unique.  On return (host arrays, caller-owned):
 *   *rank       = r;
 *   pivrows[m]  = the pivot rows in order, then the dependent rows in
 *                 increasing order (Q: U's row k sits at row pivrows[k]);
 *   colperm[n]  = colperm[j] is the input column now at position j (P), so
 *                 that A_in[:, colperm] = L (QU).
 * The call is synchronous (each block's pivots decide what follows).  The
 * row recursion's solves and updates are ff_ftrsm and ff_fgemm calls that
 * follow opts->path.  When m <= n the work first runs on the guess that A
 * has full rank (m pivots in their own columns), which fixes every size in
 * advance.  For p above about 2^26.5 part of that work runs on a second
 * stream the library owns (ordered by events after the work already on
 * opts->stream; all of it has finished when the call returns); below, the
 * panel kernels take that part into their own launches.  If the guess
 * fails A is restored from a copy and factored again with the pivot search.  A nonzero pivot is
 * assumed invertible (p prime); validate checks the entries of A first.
 * Workspace: about 4 min(m, n) n bytes and, when m <= n, a copy of A
 * (4 m n bytes) per stream, besides those of fgemm and ftrsm. */
int ff_flqup(uint32_t p, int64_t m, int64_t n, uint32_t *A, int64_t lda, int64_t *rank,
             int64_t *pivrows, int64_t *colperm, const ff_opts *opts);

/* rank(A) over Z/pZ (Section 6: the nonzero rows of U).  A is overwritten
 * by its LQUP factorisation as in ff_flqup. */
int ff_frank(uint32_t p, int64_t m, int64_t n, uint32_t *A, int64_t lda, int64_t *rank,
             const ff_opts *opts);

/* det(A) over Z/pZ for square A (Section 6: the product of U's diagonal,
 * with the sign of the column permutation; 0 below full rank), in *det.
 * n = 0 gives 1.  A is overwritten by its LQUP factorisation. */
int ff_fdet(uint32_t p, int64_t n, uint32_t *A, int64_t lda, uint32_t *det,
            const ff_opts *opts);

/* Inverse over Z/pZ (Section 6, on LQUP), p prime: for square A (device,
 * n x n, lda >= n, residues < p), X <- A^-1 (device, n x n, ldx >= n), and
 * *invertible (host) = 1; for singular A, *invertible = 0 and X is not
 * written.  A is overwritten by its LQUP factorisation (ff_flqup); X may be
 * A itself or overlap it, since X is written last, from a separate buffer.
 * The inverse is P U^-1 L^-1: two ff_ftrsm_ex solves on the identity and a
 * row permutation, on the path opts->path selects; opts->validate checks
 * the entries of A first, as in ff_flqup.  n = 0 gives *invertible = 1; n
 * is at most 65535.  The call is synchronous.  Workspace: that of ff_flqup and ff_ftrsm, plus
 * 4 n^2 + 8 n bytes held by the library per stream. */
int ff_finv(uint32_t p, int64_t n, uint32_t *A, int64_t lda, uint32_t *X, int64_t ldx,
            int *invertible, const ff_opts *opts);

/* Symmetric product (Section 6: the product A x A^T, here with a diagonal D between the factors):
 *
 *     C <- alpha A diag(D) A^T + beta C   (mod p).
 *
 * A is m x k (lda >= k), D a device vector of k residues or NULL (the
 * identity), C m x m (ldc >= m); all device pointers owned by the caller,
 * C not overlapping A or D.  The result is symmetric, so only its lower
 * triangle is computed (about half the work of ff_fgemm_ex on the same
 * shape) and then mirrored: on return C is symmetric, and the result
 * depends only on the lower triangle (i >= j) of C on entry.  Arithmetic
 * path, asynchrony and validate (A, D and C checked) as in ff_fgemm_ex;
 * Winograd levels are not used.  Workspace: the operands' digit planes or
 * packed doubles (once each), plus m k 4 bytes for A diag(D). */
int ff_faat(uint32_t p, int64_t m, int64_t k, uint32_t alpha, const uint32_t *A, int64_t lda,
            const uint32_t *D, uint32_t beta, uint32_t *C, int64_t ldc, const ff_opts *opts);

/* The plan ff_fgemm_ex would follow for these sizes (host-only). */
int ff_plan_query(uint32_t p, int transA, int transB,
                  int64_t m, int64_t n, int64_t k,
                  const ff_opts *opts, ff_plan_info *out);

/* Runs njobs independent fgemms (each with its own p, sizes, pointers) as
 * one persistent launch over a shared tile queue, preceded by one digit
 * slicing launch for the whole batch (INT8 path).  Outputs must not
 * overlap.  This is the multi-modular workload of the Chinese remaindering
 * approach (Sections 1 and 7). */
int ff_fgemm_batched(const ff_job *jobs, int njobs, const ff_opts *opts);

/* Captures the launches of a batch into a HIP graph bound to the given
 * pointers, for repeated replay with one launch call.  *graph receives an
 * opaque handle. */
int ff_batch_graph_create(const ff_job *jobs, int njobs, const ff_opts *opts,
                          void **graph);
int ff_batch_graph_launch(void *graph, void *hip_stream);
int ff_batch_graph_destroy(void *graph);

/* Serving loop.  A server owns a device arena of hbm_budget_bytes for the
 * workspaces of its requests and a thread that admits queued requests while
 * their footprint fits, merges them into persistent batched launches on up
 * to four streams of its own and retires them on completion (continuous
 * batching).  Request matrices stay device-resident and caller-owned until
 * the request is done.  submit returns FF_EBUSY only for a request that can
 * never fit the budget.  Ordering: submit records an event on the
 * submitting thread's stream (opts->stream given at create, else the
 * ff_set_stream stream of the submitting thread) and the request's batch
 * waits for it, so work enqueued on that stream before the submit (the
 * writes of A, B, C) is complete before the request reads them.  The
 * INT8 tile of a batch is the autotuner's choice for its largest product
 * (the default tiling when nothing is tuned). */
int ff_server_create(int64_t hbm_budget_bytes, const ff_opts *opts, void **server);
int ff_server_submit(void *server, const ff_job *job, uint64_t *id);
int ff_server_poll(void *server, uint64_t id, int *done);
int ff_server_wait(void *server, uint64_t id);
/* Latency (submit to completion) percentiles in ms over finished requests,
 * and throughput in Gop/s (sum of 2mnk over the busy interval). */
int ff_server_stats(void *server, double *p50_ms, double *p99_ms, double *gops,
                    int64_t *completed, int64_t *max_inflight);
/* Counters of a server's life so far: requests by state, launches, the
 * most requests merged into one launch and on the device at once, the
 * memory budget and what is admitted against it, the INT8 tile
 * configuration of the last INT8 batch (-1 if none) and the number of
 * stream slots. */
typedef struct ff_server_info {
    int64_t submitted, completed, failed, queued, running;
    int64_t batches;            /* launches (each one persistent batch) */
    int64_t max_batch_requests; /* most requests merged into one launch */
    int64_t max_inflight;       /* most requests on the device at once */
    int64_t hbm_budget, hbm_in_use;
    int last_i8_tile;
    int stream_slots;
} ff_server_info;
int ff_server_query(void *server, ff_server_info *out);
int ff_server_destroy(void *server);

/* Autotuner (the self-adapting thresholds of Section 7 applied to kernel
 * tiling).  Times every compiled INT8 tile configuration for the given
 * number of digit slices on an m x n x k product, using scratch buffers of
 * its own on the ff_set_stream stream, and records the fastest in the tuning
 * cache (file FF_TUNE_CACHE, else $HOME/.cache/ffgemm/tune_gfx950.txt) that
 * later plans of the same slice count and size class use.  Synchronous.
 * *best_tile receives the configuration id, *best_ms its kernel time. */
int ff_autotune(int slices, int64_t m, int64_t n, int64_t k, int *best_tile,
                double *best_ms);

/* Kernel timing for measurement.  ff_profile_enable(mask) clears what was
 * recorded and selects which launches get bracketed by a HIP event pair on
 * the stream they are launched on: FF_PROFILE_GEMM the matrix-core kernels
 * (FP64 and INT8 fgemm, single or batched), FF_PROFILE_PREP the operand
 * passes (digit slicing, FP64 packing); 0 disables.  Each event pair adds a
 * few microseconds between kernels, so a timing run brackets only what it
 * reports.  ff_profile_read synchronises those events and returns the
 * summed durations (ms) and launch counts since the last enable or read,
 * then clears them.  Not thread-safe against concurrent fgemm calls; meant
 * for benchmarks. */
#define FF_PROFILE_GEMM 1
#define FF_PROFILE_PREP 2
int ff_profile_enable(int mask);
int ff_profile_read(double *gemm_ms, int64_t *gemm_launches,
                    double *slice_ms, int64_t *slice_launches);

/* Thread-local text of the last non-OK status. */
const char *ff_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FFGEMM_H */
