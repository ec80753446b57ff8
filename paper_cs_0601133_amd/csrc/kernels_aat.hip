// Element-wise kernels of the symmetric product C <- alpha A D A^T + beta C
// (Section 6's A x A^T with a diagonal D between the factors): the column
// scaling A D and the mirror that copies the computed lower triangle of C
// into the upper one.
#include <algorithm>

#include "ff_device.h"
#include "ff_internal.h"

namespace ff {

namespace {

// AD[i][j] = A[i][j] d_j mod p; one workgroup row-chunk per (x, y).
__global__ __launch_bounds__(256) void k_aat_scale_cols(const uint32_t *A, int64_t lda,
                                                        const uint32_t *d, int64_t m, int64_t k,
                                                        uint32_t p, double pinv, uint32_t *AD,
                                                        int64_t ldd)
{
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= k) return;
    const uint32_t dj = d[j];
    for (int64_t i = blockIdx.y; i < m; i += gridDim.y)
        AD[i * ldd + j] = mulmod(A[i * lda + j], dj, p, pinv);
}

// C[r][c] = C[c][r] for r < c < m: 64 x 64 tiles below the diagonal are
// read through LDS and written transposed above it.
__global__ __launch_bounds__(256) void k_aat_mirror(uint32_t *C, int64_t ldc, int64_t m)
{
    __shared__ uint32_t tile[64][65];
    // blockIdx.x enumerates tiles (bi, bj) with bj <= bi
    const int64_t b = blockIdx.x;
    int64_t bi = (int64_t)((__builtin_sqrt(8.0 * (double)b + 1.0) - 1.0) * 0.5);
    while (bi * (bi + 1) / 2 > b) --bi;
    while ((bi + 1) * (bi + 2) / 2 <= b) ++bi;
    const int64_t bj = b - bi * (bi + 1) / 2;
    const int64_t r0 = 64 * bi, c0 = 64 * bj;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int rr = ty; rr < 64; rr += 4)
        if (r0 + rr < m && c0 + tx < m) tile[rr][tx] = C[(r0 + rr) * ldc + c0 + tx];
    __syncthreads();
    // write (c0 + cc, r0 + tx) <- (r0 + tx, c0 + cc) where c0 + cc < r0 + tx
    for (int cc = ty; cc < 64; cc += 4) {
        const int64_t r = c0 + cc, c = r0 + tx;
        if (r < m && c < m && r < c) C[r * ldc + c] = tile[tx][cc];
    }
}

} // namespace

hipError_t launch_aat_scale_cols(const uint32_t *A, int64_t lda, const uint32_t *d, int64_t m,
                                 int64_t k, uint32_t p, uint32_t *AD, int64_t ldd, hipStream_t st)
{
    if (m <= 0 || k <= 0) return hipSuccess;
    const dim3 grid((unsigned)((k + 255) / 256), (unsigned)std::min<int64_t>(m, 1024));
    hipLaunchKernelGGL(k_aat_scale_cols, grid, dim3(256), 0, st, A, lda, d, m, k, p,
                       1.0 / (double)p, AD, ldd);
    return hipGetLastError();
}

hipError_t launch_aat_mirror(uint32_t *C, int64_t ldc, int64_t m, hipStream_t st)
{
    if (m <= 1) return hipSuccess;
    const int64_t nb = (m + 63) / 64, tiles = nb * (nb + 1) / 2;
    if (tiles > 0x7FFFFFFF) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_aat_mirror, dim3((unsigned)tiles), dim3(256), 0, st, C, ldc, m);
    return hipGetLastError();
}

} // namespace ff
