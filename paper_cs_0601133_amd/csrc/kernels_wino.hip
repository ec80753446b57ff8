// Winograd pre- and post-additions (Section 3.2, Appendix A), one level per
// launch.  All are streaming kernels bound by HBM bandwidth: each thread
// reads the four quadrant values of one position and writes the seven
// combinations (pre) or reads seven products and writes four quadrants
// (post).  The last level of pre-additions is fused with the digit slicing
// (INT8 leaves) or the packing into binary64 (FP64 leaves) of the leaves'
// operands (k_wino_slice), so its seven int32 combinations never reach
// memory.
#include <algorithm>

#include "ff_device.h"
#include "ff_internal.h"
#include "ff_operand.h"

namespace ff {

namespace {

constexpr int WT = 256;

// Coefficients of the seven combinations, quadrant order 11, 12, 21, 22,
// products P1..P7 (Appendix A), by side, as compile-time constants so that
// a combination is a few adds.
template <int SIDE>
__device__ __forceinline__ constexpr int pre_coef(int t, int q)
{
    constexpr int a[7][4] = {{1, 0, 0, 0}, {0, 1, 0, 0}, {1, 1, -1, -1}, {0, 0, 0, 1},
                             {0, 0, 1, 1}, {-1, 0, 1, 1}, {1, 0, -1, 0}};
    constexpr int b[7][4] = {{1, 0, 0, 0}, {0, 0, 1, 0}, {0, 0, 0, 1}, {1, -1, -1, 1},
                             {-1, 1, 0, 0}, {1, -1, 0, 1}, {0, -1, 0, 1}};
    return SIDE ? b[t][q] : a[t][q];
}

__device__ __forceinline__ int64_t center_mod(int64_t x, uint32_t p, double pd, double pinv)
{
    const double xd = (double)x;
    int64_t r = (int64_t)__builtin_fma(-__builtin_rint(xd * pinv), pd, xd);
    const int64_t hi = (int64_t)((p - 1) / 2), lo = -(int64_t)(p / 2);
    r -= r > hi ? (int64_t)p : 0;
    r += r < lo ? (int64_t)p : 0;
    return r;
}

// Grid: x covers the columns of one row of quadrant positions, y the rows
// from i0 on, z the block o of the previous level, so no thread divides.
template <int SIDE>
__global__ __launch_bounds__(WT) void k_preadd(PreLevel J, int i0)
{
    const int j = blockIdx.x * WT + threadIdx.x;
    if (j >= J.cols) return;
    const int i = i0 + (int)blockIdx.y, o = blockIdx.z;
    const int64_t per = (int64_t)J.rows * J.cols;
    int64_t v[4];
    const uint32_t half = (J.p - 1) / 2;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int r = (q >> 1) * J.rows + i, c = (q & 1) * J.cols + j;
        if (J.in_residue) {
            const uint32_t *X = (const uint32_t *)J.X;
            const uint32_t u = J.trans ? X[(int64_t)c * J.ldx + r] : X[(int64_t)r * J.ldx + c];
            v[q] = center(u, J.p, half);
        } else {
            const int32_t *X = (const int32_t *)J.X + (int64_t)o * (4 * per);
            v[q] = X[(int64_t)r * (2 * J.cols) + c];
        }
    }
    const double pd = (double)J.p, pinv = 1.0 / pd;
    int32_t *Y = J.Y + (int64_t)(o * 7) * per + (int64_t)i * J.cols + j;
#pragma unroll
    for (int t = 0; t < 7; ++t) {
        int64_t x = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int cf = pre_coef<SIDE>(t, q);
            if (cf > 0) x += v[q];
            if (cf < 0) x -= v[q];
        }
        if (J.reduce) x = center_mod(x, J.p, pd, pinv);
        Y[(int64_t)t * per] = (int32_t)x;
    }
}

// Same grid as k_preadd.
__global__ __launch_bounds__(WT) void k_postadd(PostLevel J, int i0)
{
    const int j = blockIdx.x * WT + threadIdx.x;
    if (j >= J.cols) return;
    const int i = i0 + (int)blockIdx.y, o = blockIdx.z;
    const int64_t per = (int64_t)J.rows * J.cols;
    const int64_t rem = (int64_t)i * J.cols + j;
    const uint32_t *P = J.P + (int64_t)(o * 7) * per + rem;
    uint64_t x[7];
#pragma unroll
    for (int t = 0; t < 7; ++t) x[t] = P[(int64_t)t * per];
    const uint64_t p = J.p;
    // U1 = P1 + P2; U5 = P1 + P6 + P5 + P3; U6 = P1 + P6 + P7 - P4;
    // U7 = P1 + P6 + P7 + P5 (all below 5p < 2^34)
    const uint64_t u2 = x[0] + x[5];
    uint64_t q[4] = {x[0] + x[1], u2 + x[4] + x[2], u2 + x[6] + p - x[3], u2 + x[6] + x[4]};
    uint32_t *Y = J.Y + (int64_t)o * J.block_stride;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const double qd = (double)q[t]; // < 2^34: exact
        int64_t rr = (int64_t)__builtin_fma(-__builtin_rint(qd * J.pinv), (double)J.p, qd);
        rr += rr < 0 ? (int64_t)p : 0;
        uint32_t r = (uint32_t)rr;
        const int row = (t >> 1) * J.rows + i, col = (t & 1) * J.cols + j;
        uint32_t *yp = Y + (int64_t)row * J.ldy + col;
        if (J.final_level) {
            r = mulmod(J.alpha, r, J.p, J.pinv);
            if (J.beta) r = addmod(r, mulmod(J.beta, *yp, J.p, J.pinv), J.p);
        }
        *yp = r;
    }
}

// x mod p, centered, for |x| < 2^31 (binary64 quotient estimate; the
// remainder is exact and at most one step from the range).
__device__ __forceinline__ int32_t center_mod32(int32_t x, int32_t p, double pd, double pinv)
{
    const double xd = (double)x;
    int32_t r = (int32_t)__builtin_fma(-__builtin_rint(xd * pinv), pd, xd);
    const int32_t hi = (p - 1) / 2, lo = -(p / 2);
    r -= r > hi ? p : 0;
    r += r < lo ? p : 0;
    return r;
}

// One unit position of one input block: the four quadrant units are read
// (all loads issued before the LDS transposes when K-contiguous), the seven
// combinations formed and written to the block's seven leaves: as digit
// planes (INT8 leaves) or as packed binary64 (F64).  NARROW: |values| <
// 2^29, so four-term sums fit int32.
template <int SIDE, bool NARROW, bool F64>
__device__ __forceinline__ void wino_slice_block(const WinoSlice &W, int b, UnitTile &tile)
{
    const int ub = unit_blocks(W.J);
    const int o = b / ub;
    b -= o * ub;
    uint32_t u[4][16];
    int r = 0, kc = 0;
    bool ok = false;
    const uint32_t *base = (const uint32_t *)W.J.X + (int64_t)o * W.block_stride;
    if (W.J.trans) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            SliceJob J = W.J;
            J.X = base + W.qoff[q];
            ok = load_unit(J, b, tile, u[q], r, kc);
        }
    } else {
        uint32_t w[4][4][4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            SliceJob J = W.J;
            J.X = base + W.qoff[q];
            load_raw(J, b, w[q]);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (q) __syncthreads(); // every read of the tile by the previous quadrant is done
            ok = unit_from_raw(W.J, b, tile, w[q], u[q], r, kc);
        }
    }
    if (!ok) return;
    int32_t c[4][16]; // centered residues or int32 inputs
    const uint32_t half = (W.J.p - 1) / 2;
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int e = 0; e < 16; ++e)
            c[q][e] = W.J.in_mode == IN_SIGNED ? (int32_t)u[q][e] : center(u[q][e], W.J.p, half);
    const double pd = (double)W.J.p, pinv = 1.0 / pd;
    int8_t *D = W.D + (int64_t)o * 7 * W.leaf_stride;
#pragma unroll
    for (int t = 0; t < 7; ++t) {
        int32_t v[16];
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            if constexpr (NARROW) {
                int32_t x = 0;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int cf = pre_coef<SIDE>(t, q);
                    if (cf > 0) x += c[q][e];
                    if (cf < 0) x -= c[q][e];
                }
                v[e] = W.reduce ? center_mod32(x, (int32_t)W.J.p, pd, pinv) : x;
            } else {
                int64_t x = 0;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int cf = pre_coef<SIDE>(t, q);
                    if (cf > 0) x += c[q][e];
                    if (cf < 0) x -= c[q][e];
                }
                v[e] = (int32_t)(W.reduce ? center_mod(x, W.J.p, pd, pinv) : x);
            }
        }
        if constexpr (F64) {
            double d[16];
#pragma unroll
            for (int e = 0; e < 16; ++e) d[e] = (double)v[e];
            write_f64(W.J, (double *)(D + (int64_t)t * W.leaf_stride), d, r, kc);
        } else {
            write_digits(W.J, D + (int64_t)t * W.leaf_stride, v, r, kc);
        }
    }
}

// Both sides in one launch: blocks [0, blocks_a) take a, the rest b.
template <bool NARROW, bool F64>
__global__ __launch_bounds__(UNIT_THREADS) void k_wino_slice(WinoSlice a, WinoSlice b,
                                                             int blocks_a)
{
    __shared__ UnitTile tile;
    const int blk = blockIdx.x;
    if (blk < blocks_a)
        wino_slice_block<0, NARROW, F64>(a, blk, tile);
    else
        wino_slice_block<1, NARROW, F64>(b, blk - blocks_a, tile);
}

// Rows per launch: the y extent of a grid stays within 65535.
constexpr int ROW_CHUNK = 32768;

dim3 grid_of(int rows, int cols, int count)
{
    return dim3((unsigned)((cols + WT - 1) / WT), (unsigned)rows, (unsigned)count);
}

} // namespace

hipError_t launch_preadd(const PreLevel &J, hipStream_t st)
{
    if ((int64_t)J.rows * J.cols * J.count_in == 0) return hipSuccess;
    if (J.count_in > 65535) return hipErrorInvalidValue;
    for (int i0 = 0; i0 < J.rows; i0 += ROW_CHUNK) {
        const int h = std::min(ROW_CHUNK, J.rows - i0);
        if (J.side)
            hipLaunchKernelGGL(k_preadd<1>, grid_of(h, J.cols, J.count_in), dim3(WT), 0, st, J, i0);
        else
            hipLaunchKernelGGL(k_preadd<0>, grid_of(h, J.cols, J.count_in), dim3(WT), 0, st, J, i0);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

int wino_slice_blocks(const WinoSlice &w) { return w.count * unit_blocks(w.J); }

hipError_t launch_wino_slice(const WinoSlice &a, const WinoSlice &b, hipStream_t st)
{
    const int64_t na = (int64_t)a.count * unit_blocks(a.J), nb = (int64_t)b.count * unit_blocks(b.J);
    if (na + nb == 0) return hipSuccess;
    if (na + nb > 0x7FFFFFFF) return hipErrorInvalidValue;
    // inputs below 2^29 in magnitude (centered residues of p < 2^30, or the
    // int32 blocks of a reduced previous level) keep four-term sums in int32
    const bool narrow = a.J.p < (1u << 30) && (a.J.in_mode == IN_RESIDUE || a.reduce);
    const dim3 grid((unsigned)(na + nb));
    if (a.f64) {
        if (narrow)
            hipLaunchKernelGGL((k_wino_slice<true, true>), grid, dim3(UNIT_THREADS), 0, st, a, b,
                               (int)na);
        else
            hipLaunchKernelGGL((k_wino_slice<false, true>), grid, dim3(UNIT_THREADS), 0, st, a,
                               b, (int)na);
    } else {
        if (narrow)
            hipLaunchKernelGGL((k_wino_slice<true, false>), grid, dim3(UNIT_THREADS), 0, st, a,
                               b, (int)na);
        else
            hipLaunchKernelGGL((k_wino_slice<false, false>), grid, dim3(UNIT_THREADS), 0, st, a,
                               b, (int)na);
    }
    return hipGetLastError();
}

hipError_t launch_postadd(const PostLevel &J, hipStream_t st)
{
    if ((int64_t)J.rows * J.cols * J.count_out == 0) return hipSuccess;
    if (J.count_out > 65535) return hipErrorInvalidValue;
    for (int i0 = 0; i0 < J.rows; i0 += ROW_CHUNK) {
        const int h = std::min(ROW_CHUNK, J.rows - i0);
        hipLaunchKernelGGL(k_postadd, grid_of(h, J.cols, J.count_out), dim3(WT), 0, st, J, i0);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

} // namespace ff
