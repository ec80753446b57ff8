// Internal declarations of the fgemm library: plans, job descriptors shared
// by host code and kernels, kernel launchers.  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/ffgemm.h"

namespace ff {

// ---------------------------------------------------------------------------
// Error reporting
// ---------------------------------------------------------------------------
void set_error(const std::string &msg);
int fail(int status, const std::string &msg);
#define FF_HIP_CHECK(expr)                                                    \
    do {                                                                      \
        hipError_t e_ = (expr);                                               \
        if (e_ != hipSuccess)                                                 \
            return ::ff::fail(FF_EHIP, std::string(#expr) + ": " +           \
                                           hipGetErrorString(e_));            \
    } while (0)

// ---------------------------------------------------------------------------
// Tile configurations
// ---------------------------------------------------------------------------
// FP64 kernel: operands packed as centered doubles, K step 16, waves of 64
// lanes each owning 64 x 64 outputs, WGM x WGN waves per workgroup, NST
// LDS stages.  Several configurations are compiled; the planner picks one.
constexpr int F64_BK = 16;
struct F64Tile {
    int id;
    int WGM, WGN;
    int NST;    // LDS ring stages
    int WPE;    // waves per SIMD the kernel is built for
    int GM;     // tile rows per group of the tile order
    int bm() const { return 64 * WGM; }
    int bn() const { return 64 * WGN; }
    int threads() const { return 64 * WGM * WGN; }
};
int f64_tile_count();
const F64Tile &f64_tile(int id);
int f64_default_tile();
// The configuration the planner uses for an m x n product (FF_F64_TILE
// overrides; m = n = 0: the batched default).
int choose_f64_tile(int64_t m = 0, int64_t n = 0, int64_t count = 1);
// Number of K splits of a single FP64 launch with `tiles` workgroup tiles
// and nk K stages (1: no split), and the stages per split.
int f64_splits(int64_t tiles, int64_t nk, int *kt_split);

// INT8 kernel: workgroup tile BM x BN, K step 64 bytes, waves of 64 lanes
// each owning (32*TM) x (32*TN) outputs.  Several configurations per slice
// count are compiled; the planner picks one (default table, autotuner cache
// or an explicit id).
struct I8Tile {
    int id;
    int S;      // digits per operand (compile-time in the kernel)
    int TM, TN; // 32x32 MFMA tiles per wave
    int WGM, WGN;
    int KS;     // K bytes per LDS stage (32 or 64)
    int GM;     // tile rows per group of the tile order (L2 reuse)
    int pipe;   // next stage's fragments read while the current one computes
    int occ;    // workgroups per CU (each gets 1/occ of the LDS ring space)
    int bm() const { return WGM * 32 * TM; }
    int bn() const { return WGN * 32 * TN; }
    int threads() const { return 64 * WGM * WGN; }
};
// Registry of compiled configurations (kernels_i8.hip).
int i8_tile_count();
const I8Tile &i8_tile(int id);
int i8_default_tile(int S);
// Tile chosen by the autotuner for this slice count and size, or -1.
int tuned_i8_tile(int S, int64_t m, int64_t n, int64_t k);
constexpr int I8_BK = 64;

// ---------------------------------------------------------------------------
// Plan (the host-side decisions of one call)
// ---------------------------------------------------------------------------
struct Plan {
    int path = FF_PATH_INT8;
    int levels = 0;
    int preadds_reduced = 0; // Winograd pre-additions reduced to centered residues
    int bits = 0;            // INT8 digit width
    int slices = 0;          // INT8 digits per operand
    int64_t lo = 0, hi = 0;  // range of leaf operands
    int64_t max_prod = 0;    // bound on |a*b| of one leaf product term
    int64_t kblock = 0;      // FP64: products between folds; INT8: K per pass
    int tile = 0;
    int pairing = 0;         // INT8: products of digit sums for the cross terms
    int small = 0;           // FP64 without Winograd in one launch (no workspace)
    int64_t ws_bytes = 0;
    // leaf problem shape (after peeling the top level to multiples of 2^L)
    int64_t me = 0, ne = 0, ke = 0;
};

// Fills *pl for the given problem.  Returns FF_OK or an error status (with
// the message set).  Pure host code.
int make_plan(uint32_t p, int64_t m, int64_t n, int64_t k, const ff_opts &o,
              Plan *pl);

// Centered range of residues modulo p: [-(p/2), (p-1)/2].
inline int64_t centered_lo(uint32_t p) { return -(int64_t)(p / 2); }
inline int64_t centered_hi(uint32_t p) { return (int64_t)((p - 1) / 2); }

// ---------------------------------------------------------------------------
// Device job descriptors
// ---------------------------------------------------------------------------
// Operand of the packing kernels: uint32 residues (centered while packing)
// or int32 values already centered (Winograd leaves).
enum { IN_RESIDUE = 0, IN_SIGNED = 1 };

// FP64 GEMM job on packed double operands.  An operand with rows r (m
// index of op(A), n index of op(B)), K index k and row tile RT holds the
// centered value of element (r, k) at double offset
//     (r/RT)*RT*KP + (k/16)*RT*16 + ((r%RT)/16)*256 + ((k%16)/2)*32
//       + (r%16)*2 + k%2,
// zero padded to rows_pad x KP: each K stage of a row tile is one contiguous
// block, and inside it the two consecutive K values that a lane feeds to two
// matrix-core steps are one 16-byte word.
struct F64Job {
    const double *Ad;   // op(A) packed with row tile bm
    const double *Bd;   // op(B)^T packed with row tile bn
    uint32_t *C;
    int64_t ldc;
    int m, n, KP;       // KP: K padded to a multiple of F64_BK
    uint32_t p, alpha, beta;
    double pd, pinv;
    int fold_stages;    // K stages between reductions; 0: after every 4-product step
    int gm;             // tile-order group height
    int tiles_m, tiles_n;
    int tile_start;     // first global tile index of this job (batched launches)
    // Split K (single launches only): with kt_split > 0 the grid holds
    // tiles_m * tiles_n workgroups per split of kt_split K stages; each
    // writes its partial product, reduced to [0, p), to part[split][m][n]
    // and a reduction pass forms C.
    int kt_split;
    uint32_t *part;
};

// Small FP64 product in one launch (kernels_small.hip): C <- alpha op(A)
// op(B) + beta C (mod p) read straight from the residues, reduced every
// fold_steps 4-product steps.
struct F64Small {
    const uint32_t *A, *B;
    int64_t lda, ldb;
    int ta, tb;
    uint32_t *C;
    int64_t ldc;
    int m, n, k;
    uint32_t p, alpha, beta;
    double pd, pinv;
    int fold_steps;
};
hipError_t launch_f64_small(const F64Small &J, hipStream_t st);
// Whether an FP64 product without Winograd takes the one-launch kernel
// (FF_F64_SMALL=0 never, =1 always, else by size).
bool f64_small(int64_t m, int64_t n, int64_t k);

// Slicing task: one operand of one job into packed digit planes.
struct SliceJob {
    const void *X;      // uint32 residues or int32 signed values
    int64_t ldx;
    int rows, K;        // logical operand: rows x K (A: m x k, B^T: n x k)
    int trans;          // element (r, c) at X[c*ldx + r] instead of X[r*ldx + c]
    int in_mode;        // IN_RESIDUE (center with p) or IN_SIGNED
    uint32_t p;
    int S, bits;        // S == 0: one plane of doubles for the FP64 kernel
    int pairs;          // after the S digit planes, the S(S-1)/2 planes of
                        // digit sums d_i + d_j (i < j, lexicographic order)
    int8_t *D;          // packed planes
    int RT;             // row tile of the packing
    int rows_pad, KP;   // padded sizes
    int64_t plane;      // bytes per digit plane = rows_pad * KP (x 8 for doubles)
    int block_start;    // first global block of this task
};

// INT8 GEMM job on packed digit planes.
struct I8Job {
    const int8_t *Ad;
    const int8_t *Bd;
    int64_t a_plane, b_plane;
    uint32_t *C;
    int64_t ldc;
    int m, n, KP;
    int s;              // digits of this job (<= kernel's S)
    uint32_t p, beta;
    double pd, pinv;
    uint32_t w[12];     // weight of each accumulator set: alpha * R^t mod p for
                        // E_t, t = 0 .. 2s-2 (digit pairing: the 3s-3 sets of
                        // the pairing kernel, see i8_weights)
    double wc[12];      // the same weights centered, as doubles
    int fp_epi;         // recombine in binary64: (2s-1)(p/2)(p/2+1) + p <= 2^53
    int epi_direct;     // sum wc_t E_t exactly in binary64 without reducing each E_t:
                        // (2s-1) max|wc_t| max|E_t| + p <= 2^53 for this job's K
    int gm;             // tile-order group height
    int tiles_m, tiles_n;
    int tile_start;
};

// Fills w, wc and fp_epi of an INT8 job for digit width bits; with
// pairing, the weights of the pairing kernel's accumulator sets.
void i8_weights(I8Job &J, uint32_t alpha, int bits, int pairing = 0);

// Digit pairing (kernels_i8p.hip): workgroup tile i8p_bm(S) x i8p_bn(S)
// for S in 2..5; the digit planes and digit-sum planes are packed with row
// tiles of these heights.
inline int i8p_bm(int S) { return S >= 5 ? 64 : 128; }
inline int i8p_bn(int) { return 64; }
// Largest number of pairs i < j < S with the same i + j.
inline int pairing_max_pairs(int S)
{
    int best = 0;
    for (int t = 1; t <= 2 * S - 3; ++t) {
        int c = 0;
        for (int i = 0; i < S; ++i)
            for (int j = i + 1; j < S; ++j) c += i + j == t;
        best = c > best ? c : best;
    }
    return best;
}
hipError_t launch_i8_pair(const I8Job &J, hipStream_t st);

// ---------------------------------------------------------------------------
// Kernel launchers (defined in the .hip files)
// ---------------------------------------------------------------------------
// FP64 GEMM on packed operands with tile configuration `tile`: one job
// passed by value, or a device job table; grid = total tiles (persistent ==
// 0) or a persistent grid draining a tile counter (ctr: 2 words, zero on
// entry, left at zero on exit).  In a table either every job has
// fold_stages == 0 (fine != 0) or none has.
hipError_t launch_f64(int tile, const F64Job &job, hipStream_t st);
hipError_t launch_f64_batched(int tile, const F64Job *dev_jobs, int njobs, int total_tiles,
                              int persistent, unsigned *ctr, int fine, hipStream_t st);
// Operands -> packed centered doubles (SliceJobs with S == 0), both
// operands of one product in one launch.
hipError_t launch_pack_f64_2(const SliceJob &a, const SliceJob &b, hipStream_t st);
hipError_t launch_pack_f64_batched(const SliceJob *dev_jobs, int njobs, int total_blocks,
                                   hipStream_t st);

// Digit slicing of both operands of one product in one launch.
hipError_t launch_slice2(const SliceJob &a, const SliceJob &b, hipStream_t st);
hipError_t launch_slice_batched(const SliceJob *dev_jobs, int njobs,
                                int total_blocks, hipStream_t st);

hipError_t launch_i8(int tile, const I8Job &job, hipStream_t st);
// A device job table whose jobs all have the tile's digit count: one
// workgroup per tile, no persistent queue.
hipError_t launch_i8_jobs(int tile, const I8Job *dev_jobs, int njobs, int total_tiles,
                          hipStream_t st);
// uniform_s: every job has the tile's digit count, so the tile loop is
// compiled for that count alone (no dispatch over digit counts).
hipError_t launch_i8_batched(int tile, const I8Job *dev_jobs, int njobs,
                             int total_tiles, int persistent, unsigned *ctr,
                             hipStream_t st, bool uniform_s = false);

// Triangular solve (kernels_trsm.hip): the block recursion stops at leaves
// of at most TRSM_LEAF_MAX rows (a multiple of 64), solved by one kernel.
constexpr int TRSM_LEAF_MAX = 512;
// dinv_i = op(T)_ii^-1 mod p (1 when unit); bad (may be null) counts
// diagonal entries with no inverse.
hipError_t launch_trsm_dinv(const uint32_t *T, int64_t ldt, int64_t m, uint32_t p, int unit,
                            uint32_t *dinv, unsigned *bad, hipStream_t st);
// Tn = D^-1 op(T) (dinv null: D = I) restricted to its triangle (lower: op(T) lower), unit
// diagonal, zero elsewhere; ldn x ldn row-major (ldn = m rounded up to a
// multiple of 64, padding = identity).
hipError_t launch_trsm_prep(const uint32_t *T, int64_t ldt, int trans, int lower, int64_t m,
                            int64_t ldn, uint32_t p, const uint32_t *dinv, uint32_t *Tn,
                            hipStream_t st);
// B(i, :) <- alpha dinv_i B(i, :) mod p (dinv null: all ones).
hipError_t launch_trsm_scale(uint32_t *B, int64_t ldb, int64_t m, int64_t n, uint32_t p,
                             uint32_t alpha, const uint32_t *dinv, hipStream_t st);
// Tinv[g] = inverse of the 64 x 64 diagonal block g of Tn, g < ldn / 64
// (64 x 64 row-major each); split as for the leaf.
hipError_t launch_trsm_inv(const uint32_t *Tn, int64_t ldn, int lower, uint32_t p, int split,
                           uint32_t *Tinv, hipStream_t st);
// The same for a system of m <= 64 rows, read straight from op(T) (trans:
// op(T) = T^T) and scaled by dinv (null: unit), with no Tn: its single
// leaf needs only the inverse.
hipError_t launch_trsm_inv_direct(const uint32_t *T, int64_t ldt, int trans, int lower,
                                  int64_t m, uint32_t p, int split, const uint32_t *dinv,
                                  uint32_t *Tinv, hipStream_t st);
// B(i, :) <- alpha inv(T(i, i)) B(i, :) mod p with the inverses taken in the
// same launch (unit: alpha only), written to dinv_out unless null, or read
// from dinv_in when it is given (then more workgroups); bt: the
// m x n matrix B is stored transposed (entry (i, j) at B[j ldb + i]).  Replaces launch_trsm_dinv + launch_trsm_scale where no
// count of non-invertible diagonal entries is wanted.
hipError_t launch_trsm_dscale(const uint32_t *T, int64_t ldt, int unit, uint32_t *B,
                              int64_t ldb, int bt, int64_t m, int64_t n, uint32_t p,
                              uint32_t alpha, uint32_t *dinv_out, hipStream_t st,
                              const uint32_t *dinv_in = nullptr);
// Solves rows [r0, r0 + rows) of Tn X = B in place, every other row's
// contribution already subtracted; r0 a multiple of 64, rows <=
// TRSM_LEAF_MAX.  split: operands cut in two (needed once
// 64 (p/2)(p/2 + 2) + p/2 + 2 > 2^53).  bt: B (m x n) stored transposed.
hipError_t launch_trsm_leaf(const uint32_t *Tn, int64_t ldn, const uint32_t *Tinv, int lower,
                            int64_t r0, int rows, uint32_t *B, int64_t ldb, int bt, int64_t m,
                            int64_t n, uint32_t p, int split, hipStream_t st);

// LQUP (kernels_lqup.hip): rows and window columns of one pivot panel.
constexpr int LQUP_PANEL = 64;
constexpr int LQUP_WINDOW = 64;
// Factors rows [i0, i0 + nr) over columns [k, k + W) (every entry already
// reduced by the pivots above); out as described in kernels_lqup.hip
// (3 + 2 LQUP_PANEL int32).  whole: the window reaches the last column.
// fail (may be null): set to 1 when the panel does not find nr pivots in
// their own columns (a dependent row, a stop, or a column exchange).
hipError_t launch_lqup_panel(uint32_t *A, int64_t lda, int64_t i0, int nr, int64_t k, int W,
                             int whole, uint32_t p, int32_t *out, hipStream_t st,
                             int32_t *fail = nullptr);
// Panel of the full-rank guess: rows [i0, i0 + nr) pivot in columns k, k + 1,
// ... in order, or *fail becomes nonzero (1: a zero pivot or nr > W; 2: the
// kernel's internal wait gave up, an error).  The nc columns past the window
// [k, k + W) leave as the pivot rows' U entries (the unit lower triangular
// solve fused).  m2 > 0 (needs nr == W): rows [g0, g0 + m2) of the window
// are overwritten by G with G T = X, T the panel's U in the window (the
// right-hand solve for the rows below, fused).  ctr: the stream's zeroed
// counter block (word 2, left zero).  Only for p with lqup_panel_fast_ok(p)
// (centered products exact in binary64).
// so.ad set (needs m2 > 0, nc > 0, nr == 64): G and the nc carried columns
// are also written as the INT8 digit planes of the product G times those
// columns (K = 64; A operand rows m2 with row tile rta, transposed B operand
// rows nc with row tile rtb; S digits of `bits` bits, planes plane_a and
// plane_b bytes apart; the digit slicer's layout with KP = 64).
struct LqupDigits {
    int8_t *ad = nullptr, *bd = nullptr;
    int64_t plane_a = 0, plane_b = 0;
    int rta = 0, rtb = 0, S = 0, bits = 0;
};
bool lqup_panel_fast_ok(uint32_t p);
hipError_t launch_lqup_panel_fast(uint32_t *A, int64_t lda, int64_t i0, int nr, int64_t k, int W,
                                  int64_t nc, int64_t g0, int m2, uint32_t p, int32_t *fail,
                                  unsigned *ctr, hipStream_t st,
                                  const LqupDigits &so = LqupDigits{});
// Column exchanges pairs[2j] <-> pairs[2j + 1] in order, rows outside
// [skip_lo, skip_hi).
hipError_t launch_lqup_swap(uint32_t *A, int64_t lda, int64_t m, int64_t skip_lo, int64_t skip_hi,
                            const int64_t *pairs, int npairs, hipStream_t st);
// Z = I (n x n, row stride n).
hipError_t launch_lqup_identity(uint32_t *Z, int64_t n, hipStream_t st);
// U[j][c] = A[rows[j]][c0 + c].
hipError_t launch_lqup_gather(const uint32_t *A, int64_t lda, const int64_t *rows, int64_t r,
                              int64_t c0, int64_t ncols, uint32_t *U, int64_t ldu, hipStream_t st);
// out[r] = first c in [c0, n) with A[i0 + r][c] != 0, or -1, for r < nr.
hipError_t launch_lqup_first_nonzero(const uint32_t *A, int64_t lda, int64_t i0, int64_t nr,
                                     int64_t c0, int64_t n, int64_t *out, hipStream_t st);

// Symmetric product (kernels_aat.hip): AD = A diag(d) mod p (m x k), and the
// mirror C[r][c] = C[c][r] for r < c < m.
hipError_t launch_aat_scale_cols(const uint32_t *A, int64_t lda, const uint32_t *d, int64_t m,
                                 int64_t k, uint32_t p, uint32_t *AD, int64_t ldd, hipStream_t st);
hipError_t launch_aat_mirror(uint32_t *C, int64_t ldc, int64_t m, hipStream_t st);

// C <- (alpha * sum_s part[s] + beta*C) mod p over nsplit partial products
// part[s][m][n] in [0, p).
hipError_t launch_split_reduce(const uint32_t *part, int nsplit, int64_t m, int64_t n,
                               uint32_t *C, int64_t ldc, uint32_t p, uint32_t alpha,
                               uint32_t beta, hipStream_t st);

// C <- beta*C mod p (beta == 0: C <- 0), m x n, ldc.
hipError_t launch_scale(uint32_t *C, int64_t ldc, int64_t m, int64_t n,
                        uint32_t p, uint32_t beta, hipStream_t st);

// Counts entries >= p of an m x n (ld) uint32 matrix into *bad (device).
hipError_t launch_validate(const uint32_t *X, int64_t ld, int64_t rows,
                           int64_t cols, uint32_t p, unsigned *bad,
                           hipStream_t st);

// One level of Winograd pre-additions for one operand side: each of the
// count_in input operands (2*rows x 2*cols) gives seven operands (rows x
// cols) in product order P1..P7 (A side: A11, A12, S4, A22, S1, S2, S3; B
// side: B11, B21, B22, T4, T1, T2, T3; Appendix A).  Input: the caller's
// residues (level 1, centered on load, op() applied) or int32 operands of
// the previous level; output: int32, optionally reduced to centered
// residues.
struct PreLevel {
    const void *X;
    int64_t ldx;
    int trans;          // level 1 only: element (r, c) at X[c*ldx + r]
    int in_residue;     // 1: X holds uint32 residues (level 1)
    int count_in;
    int rows, cols;     // output operand size
    int side;           // 0: A side, 1: B side
    int reduce;
    uint32_t p;
    int32_t *Y;         // [count_in*7][rows][cols]
};
hipError_t launch_preadd(const PreLevel &job, hipStream_t st);

// One level of post-additions: count_out groups of seven products P1..P7
// (canonical residues, rows x cols each) give the four quadrants of a
// (2*rows) x (2*cols) block: U1, U5, U6, U7 (mod p).  At the top level the
// result is combined with C: C <- alpha*U + beta*C (mod p).
struct PostLevel {
    const uint32_t *P;  // [count_out*7][rows][cols]
    int count_out;
    int rows, cols;
    uint32_t *Y;        // output blocks
    int64_t ldy;        // row pitch of an output block
    int64_t block_stride; // elements between consecutive output blocks
    int final_level;
    uint32_t p, alpha, beta;
    double pinv;
};
hipError_t launch_postadd(const PostLevel &job, hipStream_t st);

// Last level of pre-additions fused with the digit slicing (INT8 leaves) or
// the binary64 packing (FP64 leaves) of the leaves' operands: for each of
// `count` input blocks, the seven combinations of its four quadrants are
// formed in registers and written straight into the packed operands of
// leaves 7*o .. 7*o + 6 (the values, hence the digits or doubles, are those
// of launch_preadd followed by the slicer or packer).
struct WinoSlice {
    SliceJob J;           // reads of quadrant 11 of block 0, packing layout (J.D unused)
    int64_t qoff[4];      // element offset of quadrant 11, 12, 21, 22 from a block's base
    int64_t block_stride; // elements between input blocks
    int count;            // input blocks
    int side;             // 0: A coefficients, 1: B coefficients
    int reduce;           // reduce each combination to a centered residue
    int8_t *D;            // digit planes (or packed doubles) of leaf 0
    int64_t leaf_stride;  // bytes between the operands of consecutive leaves
    int f64;              // packed binary64 (FP64 leaves) instead of digit planes
};
int wino_slice_blocks(const WinoSlice &w);
// Fused last level on (FF_WINO_FUSED=0 turns it off).
bool wino_fused_enabled();
hipError_t launch_wino_slice(const WinoSlice &a, const WinoSlice &b, hipStream_t st);

} // namespace ff
