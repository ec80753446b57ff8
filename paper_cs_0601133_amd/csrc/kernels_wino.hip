// Winograd pre- and post-additions (Section 3.2, Appendix A), one level per
// launch.  Both are streaming kernels bound by HBM bandwidth: each thread
// reads the four quadrant values of one position and writes the seven
// combinations (pre) or reads seven products and writes four quadrants
// (post).
#include "ff_device.h"
#include "ff_internal.h"

namespace ff {

namespace {

constexpr int WT = 256;

// Quadrant order 11, 12, 21, 22; products P1..P7.
__constant__ int PRE_A[7][4] = {
    {1, 0, 0, 0}, {0, 1, 0, 0}, {1, 1, -1, -1}, {0, 0, 0, 1},
    {0, 0, 1, 1}, {-1, 0, 1, 1}, {1, 0, -1, 0}};
__constant__ int PRE_B[7][4] = {
    {1, 0, 0, 0}, {0, 0, 1, 0}, {0, 0, 0, 1}, {1, -1, -1, 1},
    {-1, 1, 0, 0}, {1, -1, 0, 1}, {0, -1, 0, 1}};

__device__ __forceinline__ int64_t center_mod(int64_t x, uint32_t p, double pd, double pinv)
{
    const double xd = (double)x;
    int64_t r = (int64_t)__builtin_fma(-__builtin_rint(xd * pinv), pd, xd);
    const int64_t hi = (int64_t)((p - 1) / 2), lo = -(int64_t)(p / 2);
    r -= r > hi ? (int64_t)p : 0;
    r += r < lo ? (int64_t)p : 0;
    return r;
}

__global__ __launch_bounds__(WT) void k_preadd(PreLevel J)
{
    const int64_t per = (int64_t)J.rows * J.cols;
    const int64_t e = (int64_t)blockIdx.x * WT + threadIdx.x;
    if (e >= per * J.count_in) return;
    const int o = (int)(e / per);
    const int64_t rem = e - (int64_t)o * per;
    const int i = (int)(rem / J.cols), j = (int)(rem - (int64_t)i * J.cols);
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
        const int *cf = J.side ? PRE_B[t] : PRE_A[t];
        int64_t x = cf[0] * v[0] + cf[1] * v[1] + cf[2] * v[2] + cf[3] * v[3];
        if (J.reduce) x = center_mod(x, J.p, pd, pinv);
        Y[(int64_t)t * per] = (int32_t)x;
    }
}

__global__ __launch_bounds__(WT) void k_postadd(PostLevel J)
{
    const int64_t per = (int64_t)J.rows * J.cols;
    const int64_t e = (int64_t)blockIdx.x * WT + threadIdx.x;
    if (e >= per * J.count_out) return;
    const int o = (int)(e / per);
    const int64_t rem = e - (int64_t)o * per;
    const int i = (int)(rem / J.cols), j = (int)(rem - (int64_t)i * J.cols);
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
        uint32_t r = (uint32_t)(q[t] % p);
        const int row = (t >> 1) * J.rows + i, col = (t & 1) * J.cols + j;
        uint32_t *yp = Y + (int64_t)row * J.ldy + col;
        if (J.final_level) {
            r = mulmod(J.alpha, r, J.p, J.pinv);
            if (J.beta) r = addmod(r, mulmod(J.beta, *yp, J.p, J.pinv), J.p);
        }
        *yp = r;
    }
}

unsigned grid_of(int64_t n) { return (unsigned)((n + WT - 1) / WT); }

} // namespace

hipError_t launch_preadd(const PreLevel &J, hipStream_t st)
{
    const int64_t n = (int64_t)J.rows * J.cols * J.count_in;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_preadd, dim3(grid_of(n)), dim3(WT), 0, st, J);
    return hipGetLastError();
}

hipError_t launch_postadd(const PostLevel &J, hipStream_t st)
{
    const int64_t n = (int64_t)J.rows * J.cols * J.count_out;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_postadd, dim3(grid_of(n)), dim3(WT), 0, st, J);
    return hipGetLastError();
}

} // namespace ff
