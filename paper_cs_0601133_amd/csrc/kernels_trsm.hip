// Kernels of the triangular solve op(T) X = alpha B (mod p), Section 4.
//
// The solve runs on a normalised copy T' = D^-1 op(T) with unit diagonal (D
// the diagonal of op(T)): the system T' X = alpha D^-1 B involves ring
// operations only (Section 4.2).  Element-wise passes prepare it (diagonal
// inverses, T', the scaled right-hand side), one kernel inverts every 64 x 64
// diagonal block of T', and one kernel solves a leaf of the block recursion
// (at most TRSM_LEAF_MAX rows) for a strip of 16 columns of B; the updates
// between leaves are fgemm calls (trsm.cpp).
#include <algorithm>
#include <utility>

#include "ff_device.h"
#include "ff_internal.h"

namespace ff {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int TT = 256;

// op(T)(i, j) for T stored row-major with leading dimension ldt.
__device__ __forceinline__ uint32_t op_t(const uint32_t *T, int64_t ldt, int trans, int64_t i,
                                         int64_t j)
{
    return trans ? T[j * ldt + i] : T[i * ldt + j];
}

// Inverse of a modulo p by the extended Euclidean algorithm, 0 when a is
// not a unit (gcd(a, p) != 1).  Remainders stay below p < 2^31, so each
// division step is a 32-bit one; the Bezout coefficients need 64 bits.
__device__ __forceinline__ uint32_t inv_mod32(uint32_t a, uint32_t p)
{
    uint32_t r0 = p, r1 = a % p;
    int64_t s0 = 0, s1 = 1;
    while (r1 != 0) {
        const uint32_t q = r0 / r1, r2 = r0 - q * r1;
        const int64_t s2 = s0 - (int64_t)q * s1;
        r0 = r1; r1 = r2; s0 = s1; s1 = s2;
    }
    if (r0 != 1) return 0;
    return (uint32_t)(s0 < 0 ? s0 + (int64_t)p : s0);
}

__global__ __launch_bounds__(TT) void k_trsm_dinv(const uint32_t *T, int64_t ldt, int64_t m,
                                                  uint32_t p, int unit, uint32_t *dinv,
                                                  unsigned *bad)
{
    const int64_t i = (int64_t)blockIdx.x * TT + threadIdx.x;
    if (i >= m) return;
    uint32_t d = 1;
    if (!unit) {
        d = inv_mod32(T[i * ldt + i], p);
        if (d == 0 && bad) atomicAdd(bad, 1u);
    }
    dinv[i] = d;
}

// T'(i, j) = dinv_i op(T)(i, j) (dinv null: unit diagonal, all ones) inside
// the triangle (i, j < m), 1 on the whole diagonal, 0 elsewhere; ldn x ldn
// row-major, ldn = m rounded up to a multiple of 64, so that every 64-row
// block is whole and its padding rows and columns are those of the
// identity.  One workgroup per 64 x 64 tile of the triangle (diagonal tiles
// included); the tiles beyond it are not written, since no kernel reads them
// (the inverses read diagonal tiles, the leaves and the updates tiles inside
// the triangle).  op(T) = T^T goes through LDS so that both the reads and
// the writes run along rows.
__global__ __launch_bounds__(TT) void k_trsm_prep(const uint32_t *T, int64_t ldt, int trans,
                                                  int lower, int64_t m, int64_t ldn, uint32_t p,
                                                  double pinv, const uint32_t *dinv,
                                                  uint32_t *Tn)
{
    __shared__ uint32_t tile[64][65];
    // workgroup b takes the b-th tile of the triangle, numbered row by row
    // in the lower-triangle order (a, c), c <= a, and mirrored for upper
    const int64_t b = blockIdx.x;
    int64_t a = (int64_t)((__builtin_sqrt(8.0 * (double)b + 1.0) - 1.0) * 0.5);
    while (a * (a + 1) / 2 > b) --a;
    while ((a + 1) * (a + 2) / 2 <= b) ++a;
    const int64_t cb = b - a * (a + 1) / 2;
    const int64_t ti = lower ? a : cb, tj = lower ? cb : a;
    const int c = threadIdx.x & 63, r4 = threadIdx.x >> 6;
    const int64_t i0 = 64 * ti, j0 = 64 * tj;
    uint32_t *dst = Tn + i0 * ldn + j0;
    // op(T)(i0 + r, j0 + c) into tile[r][c]
    for (int r = r4; r < 64; r += 4) {
        uint32_t v = 0;
        if (trans) {
            // read T(j0 + r, i0 + c) along the row, store transposed
            if (j0 + r < m && i0 + c < m) v = T[(j0 + r) * ldt + i0 + c];
            tile[c][r] = v;
        } else {
            if (i0 + r < m && j0 + c < m) v = T[(i0 + r) * ldt + j0 + c];
            tile[r][c] = v;
        }
    }
    __syncthreads();
    for (int r = r4; r < 64; r += 4) {
        const int64_t i = i0 + r, j = j0 + c;
        uint32_t v = 0;
        if (i == j) v = 1;
        else if (i < m && j < m && (lower ? j < i : j > i))
            v = dinv ? mulmod(dinv[i], tile[r][c], p, pinv) : tile[r][c];
        dst[(int64_t)r * ldn + c] = v;
    }
}

// B(i, j) <- alpha dinv_i B(i, j) mod p (dinv null: all ones): workgroup (x, y) scales 1024
// columns of rows y, y + gridDim.y, ...
__global__ __launch_bounds__(TT) void k_trsm_scale(uint32_t *B, int64_t ldb, int64_t m,
                                                   int64_t n, uint32_t p, double pinv,
                                                   uint32_t alpha, const uint32_t *dinv)
{
    const int64_t j0 = (int64_t)blockIdx.x * 4 * TT + threadIdx.x;
    for (int64_t i = blockIdx.y; i < m; i += gridDim.y) {
        const uint32_t f = dinv ? mulmod(alpha, dinv[i], p, pinv) : alpha;
        uint32_t *row = B + i * ldb;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t j = j0 + u * TT;
            if (j < n) row[j] = mulmod(f, row[j], p, pinv);
        }
    }
}

// B(i, j) <- alpha dinv_i B(i, j) with dinv_i the inverse of T(i, i) taken
// here (unit: none), in one pass: every workgroup inverts the diagonal
// entries of the rows it scales, and one column of workgroups also writes
// them to dinv_out (null: not wanted) for the kernels that normalise T.
// BT: B stored transposed (entry (i, j) at B[j ldb + i]).  Workgroup (x, y):
// BT: rows i in [1024 x, 1024 x + 1024), storage rows j = y, y + gridDim.y, ..;
// else: columns [1024 x, 1024 x + 1024), rows i = y, y + gridDim.y, ...
// gridDim.y is kept small (64): it is the number of times each inverse is
// taken.
template <bool BT>
__global__ __launch_bounds__(TT) void k_trsm_dscale(const uint32_t *T, int64_t ldt, int unit,
                                                    uint32_t *B, int64_t ldb, int64_t m,
                                                    int64_t n, uint32_t p, double pinv,
                                                    uint32_t alpha, uint32_t *dinv_out,
                                                    const uint32_t *dinv_in)
{
    auto factor = [&](int64_t i, bool write) {
        if (unit) return alpha;
        if (dinv_in) return mulmod(alpha, dinv_in[i], p, pinv);
        const uint32_t d = inv_mod32(T[i * ldt + i], p);
        if (write && dinv_out) dinv_out[i] = d;
        return mulmod(alpha, d, p, pinv);
    };
    if (BT) {
        const int64_t i0 = (int64_t)blockIdx.x * 4 * TT + threadIdx.x;
        uint32_t f[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t i = i0 + u * TT;
            f[u] = i < m ? factor(i, blockIdx.y == 0) : 0u;
        }
        // four storage rows at a time, all loads before the stores (a load
        // after a store to B would wait for it: the addresses may alias)
        const int64_t G = gridDim.y;
        for (int64_t j = blockIdx.y; j < n; j += 4 * G) {
            uint32_t v[4][4];
#pragma unroll
            for (int b = 0; b < 4; ++b)
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int64_t i = i0 + u * TT, jj = j + b * G;
                    v[b][u] = i < m && jj < n ? B[jj * ldb + i] : 0u;
                }
#pragma unroll
            for (int b = 0; b < 4; ++b)
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int64_t i = i0 + u * TT, jj = j + b * G;
                    if (i < m && jj < n) B[jj * ldb + i] = mulmod(f[u], v[b][u], p, pinv);
                }
        }
    } else {
        // the workgroup's rows i = y + k gridDim.y, their factors taken TT
        // at a time (one inversion per thread) and shared through LDS
        __shared__ uint32_t sf[TT];
        const int64_t j0 = (int64_t)blockIdx.x * 4 * TT + threadIdx.x;
        const int64_t nk = (m - blockIdx.y + gridDim.y - 1) / gridDim.y;
        for (int64_t k0 = 0; k0 < nk; k0 += TT) {
            const int64_t kk = k0 + threadIdx.x;
            if (kk < nk) sf[threadIdx.x] = factor(blockIdx.y + kk * gridDim.y, blockIdx.x == 0);
            __syncthreads();
            const int64_t kend = nk - k0 < TT ? nk - k0 : TT;
            for (int64_t q = 0; q < kend; ++q) {
                const uint32_t f = sf[q];
                uint32_t *row = B + (blockIdx.y + (k0 + q) * gridDim.y) * ldb;
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int64_t j = j0 + u * TT;
                    if (j < n) row[j] = mulmod(f, row[j], p, pinv);
                }
            }
            __syncthreads();
        }
    }
}

// x - p rint(x / p) for an integer-valued x, |x| <= 2^53: |result| <= p/2 + 2.
__device__ __forceinline__ double reduce_c(double x, double pd, double pinv)
{
    return __builtin_fma(-__builtin_rint(x * pinv), pd, x);
}

// Inverse Y of the unit triangular diagonal block g of T' (rows and columns
// [64g, 64g + 64)), written to Tinv + 4096 g (64 x 64 row-major).  Column j
// of Y solves T' y = e_j; in the triangle's order (lower: l = 0, 1, ..;
// upper: l = 63, 62, ..) y_l is final once the rows before it have been
// subtracted, and is then subtracted, times T'(i, l), from every other row
// (T' is read with its diagonal set to 0, and it is 0 on the far side of the
// triangle, so no row needs a test).  One wave takes 4 columns of one
// block (16 workgroups per block); lane 16 jl + rl keeps rows rl + 16q,
// q < 4, of column 4 jq + jl in registers, unreduced: each is a sum of at
// most 63 products of centered values, exact in binary64 under the bound of
// the leaf solve (SPLIT: the entries of T' cut in two as there).  Row l,
// reduced, reaches the 16 lanes of its column by a DPP row broadcast (a
// register move, no LDS round trip): no barrier and no global memory access
// on the 64-step chain, and 4 products per lane and step (with 4 lanes per
// column and 16 products per step the chain took 14.6 us per block).  With
// one wave per workgroup nothing hides LDS latency, so each step's
// coefficients are requested during the step before, and the product that
// completes the next step's row is issued first.
//
// DIRECT (systems of at most 64 rows, whose one leaf reads no T'): the
// entries come straight from op(T) (InvDirect), restricted to the triangle
// and scaled by the diagonal inverses here, so T' is never formed.
struct InvDirect {
    const uint32_t *T;
    int64_t ldt;
    int trans;
    int m;
    const uint32_t *dinv; // null: unit diagonal
};

// Lanes per column of the inverse: lane LPC jl + rl keeps rows rl + LPC q
// (q < NQ) of one column, so each of the 64 steps costs NQ products per lane.
constexpr int LPC = 16;
constexpr int NQ = 64 / LPC;
constexpr int WPB = LPC; // workgroups (one wave, 64 / LPC columns each) per block

// v of lane LPC (lane / LPC) + R, to every lane of its group of LPC (a DPP
// row broadcast: the groups are the 16-lane rows).
template <int R>
__device__ __forceinline__ double group_bcast(double v)
{
    static_assert(LPC == 16, "one DPP row per column");
    constexpr int ctrl = 0x150 | R; // row_newbcast:R
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), ctrl, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), ctrl, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

template <int... R>
__device__ __forceinline__ double group_bcast_rt(double v, int r, std::integer_sequence<int, R...>)
{
    double out = 0.0;
    ((r == R ? (void)(out = group_bcast<R>(v)) : (void)0), ...);
    return out;
}

template <bool SPLIT, bool LOWER, bool DIRECT>
__global__ __launch_bounds__(64) void k_trsm_inv(const uint32_t *Tn, int64_t ldn, uint32_t p,
                                                 double pinv, uint32_t *Tinv, InvDirect d)
{
    // sT[.][l][i] = T'(i, l), diagonal 0; rows padded to 65 so that the
    // transposing stores (one l per lane) spread over the banks
    __shared__ double sT[SPLIT ? 2 : 1][64][65];
    const int g = blockIdx.x / WPB, jq = blockIdx.x % WPB;
    const int lane = threadIdx.x, jl = lane / LPC, rl = lane % LPC;
    const int j = (64 / LPC) * jq + jl;
    const uint32_t half = (p - 1) / 2;
    const double pd = (double)p;
    uint32_t raw[64]; // row i, column l = lane: all loads in flight at once
    if constexpr (DIRECT) {
        // T(i, lane) from addresses clamped into the m x m matrix (the loads
        // carry no condition and run along rows of T; entries outside are
        // zeroed below).  It is op(T)(i, lane), or op(T)(lane, i) if trans.
        const int lc = min(lane, d.m - 1);
#pragma unroll
        for (int i = 0; i < 64; ++i) raw[i] = d.T[(int64_t)min(i, d.m - 1) * d.ldt + lc];
    } else {
        const uint32_t *src = Tn + (int64_t)64 * g * ldn + 64 * g;
#pragma unroll
        for (int i = 0; i < 64; ++i) raw[i] = src[(int64_t)i * ldn + lane];
    }
#pragma unroll
    for (int i = 0; i < 64; ++i) {
        double t;
        int row = i, col = lane; // of T', where t goes
        if constexpr (DIRECT) {
            if (d.trans) { row = lane; col = i; }
            const bool in = row < d.m && col < d.m && (LOWER ? col < row : col > row);
            uint32_t u = in ? raw[i] : 0u;
            if (d.dinv) u = mulmod(d.dinv[min(row, d.m - 1)], u, p, pinv);
            t = (double)center(u, p, half);
        } else {
            t = i == lane ? 0.0 : (double)center(raw[i], p, half);
        }
        if (SPLIT) {
            const double th = __builtin_rint(t * (1.0 / 32768.0));
            sT[0][col][row] = th;
            sT[SPLIT ? 1 : 0][col][row] = __builtin_fma(-th, 32768.0, t);
        } else {
            sT[0][col][row] = t;
        }
    }
    double y[NQ], yh[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        y[q] = rl + LPC * q == j ? 1.0 : 0.0;
        yh[q] = 0.0;
    }
    __syncthreads();
    // coefficients of a step, requested one step ahead (double-buffered)
    double cf[2][NQ], cfh[2][NQ];
    auto fetch = [&](int s, double (&c)[NQ], double (&ch)[NQ]) {
        const int l = LOWER ? s : 63 - s;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            c[q] = sT[SPLIT ? 1 : 0][l][rl + LPC * q];
            if (SPLIT) ch[q] = sT[0][l][rl + LPC * q];
        }
    };
    fetch(0, cf[0], cfh[0]);
#pragma unroll
    for (int s = 0; s < 64; ++s) {
        const int l = LOWER ? s : 63 - s;
        const int qo = l / LPC, ro = l % LPC;
        if (s + 1 < 64) fetch(s + 1, cf[(s + 1) & 1], cfh[(s + 1) & 1]);
        // every lane reduces its entry q = qo (a value-preserving step); the
        // lane with rl == ro holds row l, now final
        double v = y[qo];
        if (SPLIT) v = __builtin_fma(reduce_c(yh[qo], pd, pinv), 32768.0, v);
        v = reduce_c(v, pd, pinv);
        y[qo] = v;
        yh[qo] = 0.0;
        // ro is a constant once the loop is unrolled
        const double yl = group_bcast_rt(v, ro, std::make_integer_sequence<int, LPC>{});
        // the row the next step reduces first
        const int qn = ((LOWER ? (l + 1) : (l - 1 + 64)) % 64) / LPC;
#pragma unroll
        for (int qq = 0; qq < NQ; ++qq) {
            const int q = (qn + qq) % NQ;
            if (SPLIT) {
                yh[q] = __builtin_fma(-cfh[s & 1][q], yl, yh[q]);
                y[q] = __builtin_fma(-cf[s & 1][q], yl, y[q]);
            } else {
                y[q] = __builtin_fma(-cf[s & 1][q], yl, y[q]);
            }
        }
    }
    // every row was reduced when it became final (its later updates add
    // T'(i, l) = 0 terms only)
    uint32_t *dst = Tinv + (int64_t)4096 * g;
#pragma unroll
    for (int q = 0; q < NQ; ++q) dst[(rl + LPC * q) * 64 + j] = canon_f64(y[q], pd, pinv, p);
}

// ---------------------------------------------------------------------------
// Leaf solve on the FP64 matrix cores.
//
// A workgroup owns 16 columns of B and walks the leaf's 64-row sub-blocks in
// the triangle's order (lower: top down, upper: bottom up).  For sub-block b
// it forms the residual
//     R_b = B_b - sum_{q solved} T'_{bq} X_q           (reduced after every q)
// with v_mfma_f64_16x16x4, then X_b = inv(T'_bb) R_b, one more 64-deep
// product through LDS.  Values are centered residues in binary64: a sum of
// at most 64 products stays an exact integer while
// 64 (p/2)(p/2 + 2) + p/2 + 2 <= 2^53 (the delayed reduction of Section
// 2.1.2); beyond that (SPLIT) each T' entry t is cut into t_hi 2^15 + t_lo
// (|t_lo| <= 2^14) and the two sums, each below 2^51, are reduced
// separately.
//
// Eight waves: wave (g, h) = (w % 4, w / 4) owns rows 16g .. 16g + 15 of the
// sub-block and half h of every product's 64-deep sum, so two waves share a
// SIMD and one's conversions overlap the other's matrix-core steps (with one
// wave per SIMD they serialise).  Each wave reduces its own partial sum
// after every product (reduction is a ring map, so the halves add up to the
// residual modulo p); the halves meet in LDS before and after the inverse
// step.
//
// Operand layout: at MFMA step s lane l supplies A(l % 16, k) and
// B(k, l % 16) with k = 16 (l / 16) + 8h + s, s < 8, so each lane reads 8
// consecutive entries of its row of T' (two 16-byte loads straight from
// global memory) and the X blocks in LDS are read along k; the result
// D(i, j) sits in lane j + 16 (i % 4), register i / 4.  LDS blocks are
// 64 x 16 doubles with a spare row after every 16 so that the k-rows read
// together (k and k + 16) fall in opposite halves of the banks.
constexpr int LT = 512;                // threads per leaf workgroup
constexpr int LW = 16;                 // columns per workgroup
constexpr int KROWS = 68;              // 64 rows + one spare per 16
constexpr int OPB = KROWS * LW;        // doubles per LDS operand block
constexpr int NSB = TRSM_LEAF_MAX / 64;

__device__ __forceinline__ int krow(int k) { return k + (k >> 4); }

__device__ __forceinline__ void load_row8(const uint32_t *src, uint4 (&v)[2])
{
    const uint4 *s = (const uint4 *)src;
    v[0] = s[0];
    v[1] = s[1];
}

__device__ __forceinline__ uint32_t word(const uint4 (&v)[2], int s)
{
    const uint4 &q = v[s >> 2];
    switch (s & 3) {
    case 0: return q.x;
    case 1: return q.y;
    case 2: return q.z;
    default: return q.w;
    }
}

// This lane's 8 B-operand entries of the LDS block `xb` (k = k0 + s).
__device__ __forceinline__ void read_x(const double *xb, int k0, int col, double (&xv)[8])
{
#pragma unroll
    for (int s = 0; s < 8; ++s) xv[s] = xb[krow(k0 + s) * LW + col];
}

// acc (+)= sign * A X over this wave's half of a 64-deep product: A's row
// for this lane in `row` (8 residues), X's entries in `xv`.
template <bool SPLIT>
__device__ __forceinline__ void product(const uint4 (&row)[2], const double (&xv)[8],
                                        double sign, uint32_t p, uint32_t half, v4d &acc,
                                        v4d &acc_hi)
{
#pragma unroll
    for (int s = 0; s < 8; ++s) {
        const double t = sign * (double)center(word(row, s), p, half);
        const double x = xv[s];
        if (SPLIT) {
            const double th = __builtin_rint(t * (1.0 / 32768.0));
            const double tl = __builtin_fma(-th, 32768.0, t);
            acc_hi = __builtin_amdgcn_mfma_f64_16x16x4f64(th, x, acc_hi, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(tl, x, acc, 0, 0, 0);
        } else {
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(t, x, acc, 0, 0, 0);
        }
    }
}

template <bool SPLIT>
__device__ __forceinline__ void settle(v4d &acc, v4d &acc_hi, double pd, double pinv)
{
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        double v = acc[r];
        if (SPLIT) v = __builtin_fma(reduce_c(acc_hi[r], pd, pinv), 32768.0, v);
        acc[r] = reduce_c(v, pd, pinv);
    }
}

// NS = number of 64-row sub-blocks in the leaf; the whole walk unrolls.
// Global loads take microseconds, so each row's operands are requested a row
// ahead: when row t starts, the entries of B, the inverse block and the
// first T' block of row t + 1 are requested (double-buffered by parity); its
// remaining T' blocks follow once row t's products have freed their
// registers.  The X entries of the next product are read from LDS before the
// current product's matrix-core steps (scheduling barriers keep the
// compiler from sinking the reads).
template <bool SPLIT, int NS>
__global__ __launch_bounds__(LT) void k_trsm_leaf(const uint32_t *Tn, int64_t ldn,
                                                  const uint32_t *Tinv, int lower, int64_t r0,
                                                  uint32_t *B, int64_t ldb, int bt, int64_t m,
                                                  int64_t n, uint32_t p, double pinv)
{
    __shared__ __attribute__((aligned(16))) double sC[2][OPB]; // residual halves
    __shared__ __attribute__((aligned(16))) double sP[2][OPB]; // halves of X_b
    __shared__ __attribute__((aligned(16))) double sX[NS * OPB];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int g = w & 3, h = w >> 2;
    const int col = lane & 15, kg = lane >> 4;
    const int k0 = 16 * kg + 8 * h; // this lane's first k of a product
    const int64_t gcol = (int64_t)blockIdx.x * LW + col;
    const bool colok = gcol < n;
    const uint32_t half = (p - 1) / 2;
    const double pd = (double)p;
    // this lane's row of a 64 x 64 block: 16g + col, entries k0 .. k0 + 7
    const int arow = 16 * g + col;

    uint4 s0[2][2];                   // first T' block of a row (by parity)
    uint4 sl[NS > 2 ? NS - 1 : 2][2]; // T' blocks 1.. of the current row
    uint4 si[2][2];                   // inverse block of a row (by parity)
    uint32_t braw[2][4];              // a row's entries of B (by parity; h = 0)
    // entry (row, this lane's column) of B; bt: B stored transposed
    auto bidx = [&](int64_t row) { return bt ? gcol * ldb + row : row * ldb + gcol; };
    auto sub = [&](int t) { return lower ? t : NS - 1 - t; };
    auto trow = [&](int t) { return Tn + (r0 + 64 * sub(t) + arow) * ldn + r0 + k0; };
    auto early = [&](int t) {
        const int64_t rb = r0 + 64 * sub(t);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t gr = rb + 16 * g + kg + 4 * r;
            braw[t & 1][r] = h == 0 && gr < m && colok ? B[bidx(gr)] : 0u;
        }
        load_row8(Tinv + (int64_t)4096 * (rb >> 6) + arow * 64 + k0, si[t & 1]);
        if (t > 0) load_row8(trow(t) + 64 * sub(0), s0[t & 1]);
    };
    auto late = [&](int t) {
#pragma unroll
        for (int u = 1; u < t; ++u) load_row8(trow(t) + 64 * sub(u), sl[u]);
    };
    early(0);
#pragma unroll
    for (int t = 0; t < NS; ++t) {
        const int b = sub(t);
        const int64_t rb = r0 + 64 * b;
        if (t + 1 < NS) early(t + 1);
        v4d acc, acc_hi = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[r] = (double)center(braw[t & 1][r], p, half);
        double xv[2][8];
        if (t > 0) read_x(sX + sub(0) * OPB, k0, col, xv[0]);
#pragma unroll
        for (int u = 0; u < t; ++u) {
            if (u + 1 < t) read_x(sX + sub(u + 1) * OPB, k0, col, xv[(u + 1) & 1]);
            __builtin_amdgcn_sched_barrier(0);
            if (SPLIT) acc_hi = v4d{0.0, 0.0, 0.0, 0.0};
            product<SPLIT>(u == 0 ? s0[t & 1] : sl[u], xv[u & 1], -1.0, p, half, acc, acc_hi);
            settle<SPLIT>(acc, acc_hi, pd, pinv);
            __builtin_amdgcn_sched_barrier(0);
        }
        if (t + 1 < NS) late(t + 1);
        // X_b = inv(T'_bb) R_b with R_b = the two halves' sum, read along k
#pragma unroll
        for (int r = 0; r < 4; ++r) sC[h][krow(16 * g + kg + 4 * r) * LW + col] = acc[r];
        __syncthreads();
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            const int e = krow(k0 + s) * LW + col;
            xv[0][s] = reduce_c(sC[0][e] + sC[1][e], pd, pinv);
        }
        v4d x = {0.0, 0.0, 0.0, 0.0}, x_hi = {0.0, 0.0, 0.0, 0.0};
        product<SPLIT>(si[t & 1], xv[0], 1.0, p, half, x, x_hi);
        settle<SPLIT>(x, x_hi, pd, pinv);
#pragma unroll
        for (int r = 0; r < 4; ++r) sP[h][krow(16 * g + kg + 4 * r) * LW + col] = x[r];
        __syncthreads();
        // wave (g, h) finishes rows kg + 4r, r in {2h, 2h + 1}, of its block
#pragma unroll
        for (int rr = 0; rr < 2; ++rr) {
            const int i = 16 * g + kg + 4 * (2 * h + rr);
            const int e = krow(i) * LW + col;
            const double v = reduce_c(sP[0][e] + sP[1][e], pd, pinv);
            sX[b * OPB + e] = v;
            const int64_t gr = rb + i;
            if (gr < m && colok) B[bidx(gr)] = canon_f64(v, pd, pinv, p);
        }
        __syncthreads();
    }
}

template <bool SPLIT, int NS>
void launch_leaf_ns(dim3 grid, hipStream_t st, const uint32_t *Tn, int64_t ldn,
                    const uint32_t *Tinv, int lower, int64_t r0, uint32_t *B, int64_t ldb, int bt,
                    int64_t m, int64_t n, uint32_t p)
{
    hipLaunchKernelGGL((k_trsm_leaf<SPLIT, NS>), grid, dim3(LT), 0, st, Tn, ldn, Tinv, lower, r0,
                       B, ldb, bt, m, n, p, 1.0 / (double)p);
}

template <bool SPLIT>
void launch_leaf(int ns, dim3 grid, hipStream_t st, const uint32_t *Tn, int64_t ldn,
                 const uint32_t *Tinv, int lower, int64_t r0, uint32_t *B, int64_t ldb, int bt,
                 int64_t m, int64_t n, uint32_t p)
{
    static_assert(NSB == 8, "one instantiation per sub-block count");
    switch (ns) {
#define FF_LEAF_CASE(k)                                                                        \
    case k: launch_leaf_ns<SPLIT, k>(grid, st, Tn, ldn, Tinv, lower, r0, B, ldb, bt, m, n, p); break;
        FF_LEAF_CASE(1) FF_LEAF_CASE(2) FF_LEAF_CASE(3) FF_LEAF_CASE(4)
        FF_LEAF_CASE(5) FF_LEAF_CASE(6) FF_LEAF_CASE(7) FF_LEAF_CASE(8)
#undef FF_LEAF_CASE
    default: break;
    }
}


} // namespace

hipError_t launch_trsm_dinv(const uint32_t *T, int64_t ldt, int64_t m, uint32_t p, int unit,
                            uint32_t *dinv, unsigned *bad, hipStream_t st)
{
    hipLaunchKernelGGL(k_trsm_dinv, dim3((unsigned)((m + TT - 1) / TT)), dim3(TT), 0, st, T,
                       ldt, m, p, unit, dinv, bad);
    return hipGetLastError();
}

hipError_t launch_trsm_prep(const uint32_t *T, int64_t ldt, int trans, int lower, int64_t m,
                            int64_t ldn, uint32_t p, const uint32_t *dinv, uint32_t *Tn,
                            hipStream_t st)
{
    const int64_t nt = ldn / 64, tiles = nt * (nt + 1) / 2; // the triangle's tiles
    if (tiles > 0x7FFFFFFF) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_trsm_prep, dim3((unsigned)tiles), dim3(TT), 0, st, T, ldt, trans, lower,
                       m, ldn, p, 1.0 / (double)p, dinv, Tn);
    return hipGetLastError();
}

hipError_t launch_trsm_scale(uint32_t *B, int64_t ldb, int64_t m, int64_t n, uint32_t p,
                             uint32_t alpha, const uint32_t *dinv, hipStream_t st)
{
    const dim3 grid((unsigned)((n + 4 * TT - 1) / (4 * TT)), (unsigned)std::min<int64_t>(m, 4096));
    hipLaunchKernelGGL(k_trsm_scale, grid, dim3(TT), 0, st, B, ldb, m, n, p, 1.0 / (double)p,
                       alpha, dinv);
    return hipGetLastError();
}

namespace {

template <bool DIRECT>
void launch_inv(dim3 grid, hipStream_t st, const uint32_t *Tn, int64_t ldn, int lower,
                uint32_t p, int split, uint32_t *Tinv, const InvDirect &d)
{
    const double pinv = 1.0 / (double)p;
    if (split && lower)
        hipLaunchKernelGGL((k_trsm_inv<true, true, DIRECT>), grid, dim3(64), 0, st, Tn, ldn, p,
                           pinv, Tinv, d);
    else if (split)
        hipLaunchKernelGGL((k_trsm_inv<true, false, DIRECT>), grid, dim3(64), 0, st, Tn, ldn, p,
                           pinv, Tinv, d);
    else if (lower)
        hipLaunchKernelGGL((k_trsm_inv<false, true, DIRECT>), grid, dim3(64), 0, st, Tn, ldn, p,
                           pinv, Tinv, d);
    else
        hipLaunchKernelGGL((k_trsm_inv<false, false, DIRECT>), grid, dim3(64), 0, st, Tn, ldn, p,
                           pinv, Tinv, d);
}

} // namespace

hipError_t launch_trsm_inv(const uint32_t *Tn, int64_t ldn, int lower, uint32_t p, int split,
                           uint32_t *Tinv, hipStream_t st)
{
    launch_inv<false>(dim3((unsigned)(ldn / 64 * WPB)), st, Tn, ldn, lower, p, split, Tinv,
                      InvDirect{nullptr, 0, 0, 0, nullptr});
    return hipGetLastError();
}

hipError_t launch_trsm_inv_direct(const uint32_t *T, int64_t ldt, int trans, int lower,
                                  int64_t m, uint32_t p, int split, const uint32_t *dinv,
                                  uint32_t *Tinv, hipStream_t st)
{
    if (m < 1 || m > 64) return hipErrorInvalidValue;
    launch_inv<true>(dim3(WPB), st, nullptr, 0, lower, p, split, Tinv,
                     InvDirect{T, ldt, trans, (int)m, dinv});
    return hipGetLastError();
}

hipError_t launch_trsm_dscale(const uint32_t *T, int64_t ldt, int unit, uint32_t *B,
                              int64_t ldb, int bt, int64_t m, int64_t n, uint32_t p,
                              uint32_t alpha, uint32_t *dinv_out, hipStream_t st,
                              const uint32_t *dinv_in)
{
    const double pinv = 1.0 / (double)p;
    if (bt) {
        // inverting in the pass: few workgroup rows, each one inverts its
        // 1024 diagonal entries; with the inverses given, enough workgroups
        // to keep the loads of a large B in flight (four storage rows each)
        const int64_t gy = dinv_in || unit ? std::max<int64_t>(64, (n + 3) / 4) : 64;
        const dim3 grid((unsigned)((m + 4 * TT - 1) / (4 * TT)),
                        (unsigned)std::min<int64_t>(n, std::min<int64_t>(gy, 1024)));
        hipLaunchKernelGGL(k_trsm_dscale<true>, grid, dim3(TT), 0, st, T, ldt, unit, B, ldb, m,
                           n, p, pinv, alpha, dinv_out, dinv_in);
    } else {
        const dim3 grid((unsigned)((n + 4 * TT - 1) / (4 * TT)), (unsigned)std::min<int64_t>(m, 64));
        hipLaunchKernelGGL(k_trsm_dscale<false>, grid, dim3(TT), 0, st, T, ldt, unit, B, ldb, m,
                           n, p, pinv, alpha, dinv_out, dinv_in);
    }
    return hipGetLastError();
}

hipError_t launch_trsm_leaf(const uint32_t *Tn, int64_t ldn, const uint32_t *Tinv, int lower,
                            int64_t r0, int rows, uint32_t *B, int64_t ldb, int bt, int64_t m,
                            int64_t n, uint32_t p, int split, hipStream_t st)
{
    const int ns = (rows + 63) / 64;
    if (rows < 1 || ns > NSB || r0 % 64) return hipErrorInvalidValue;
    const dim3 grid((unsigned)((n + LW - 1) / LW));
    if (split) launch_leaf<true>(ns, grid, st, Tn, ldn, Tinv, lower, r0, B, ldb, bt, m, n, p);
    else launch_leaf<false>(ns, grid, st, Tn, ldn, Tinv, lower, r0, B, ldb, bt, m, n, p);
    return hipGetLastError();
}

} // namespace ff
