// Element-wise kernels: C <- beta*C mod p (the k == 0 / alpha == 0 case of
// the operation), the sum of split-K partial products with the epilogue, and
// the optional input-range check.
#include "ff_device.h"
#include "ff_internal.h"

namespace ff {

namespace {

constexpr int AUX_THREADS = 256;

__global__ __launch_bounds__(AUX_THREADS) void k_scale(uint32_t *C, int64_t ldc,
                                                       int64_t m, int64_t n,
                                                       uint32_t p, uint32_t beta,
                                                       double pinv)
{
    const int64_t total = m * n;
    for (int64_t e = (int64_t)blockIdx.x * AUX_THREADS + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * AUX_THREADS) {
        const int64_t i = e / n, j = e - i * n;
        uint32_t *cp = C + i * ldc + j;
        *cp = beta ? mulmod(beta, *cp, p, pinv) : 0u;
    }
}

__global__ __launch_bounds__(AUX_THREADS) void k_validate(const uint32_t *X, int64_t ld,
                                                          int64_t rows, int64_t cols,
                                                          uint32_t p, unsigned *bad)
{
    const int64_t total = rows * cols;
    unsigned cnt = 0;
    for (int64_t e = (int64_t)blockIdx.x * AUX_THREADS + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * AUX_THREADS) {
        const int64_t i = e / cols, j = e - i * cols;
        cnt += X[i * ld + j] >= p ? 1u : 0u;
    }
    if (cnt) atomicAdd(bad, cnt);
}

__global__ __launch_bounds__(AUX_THREADS) void k_split_reduce(
    const uint32_t *part, int nsplit, int64_t m, int64_t n, uint32_t *C, int64_t ldc,
    uint32_t p, uint32_t alpha, uint32_t beta, double pinv)
{
    const int64_t total = m * n;
    for (int64_t e = (int64_t)blockIdx.x * AUX_THREADS + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * AUX_THREADS) {
        uint64_t s = 0; // nsplit residues < p < 2^31: no overflow
        for (int q = 0; q < nsplit; ++q) s += part[(int64_t)q * total + e];
        const uint32_t r = (uint32_t)(s % p);
        const int64_t i = e / n, j = e - i * n;
        uint32_t *cp = C + i * ldc + j;
        uint32_t out = mulmod(alpha, r, p, pinv);
        if (beta) out = addmod(out, mulmod(beta, *cp, p, pinv), p);
        *cp = out;
    }
}

int grid_for(int64_t total)
{
    int64_t g = (total + AUX_THREADS - 1) / AUX_THREADS;
    if (g > 65536) g = 65536;
    return g < 1 ? 1 : (int)g;
}

} // namespace

hipError_t launch_scale(uint32_t *C, int64_t ldc, int64_t m, int64_t n,
                        uint32_t p, uint32_t beta, hipStream_t st)
{
    hipLaunchKernelGGL(k_scale, dim3(grid_for(m * n)), dim3(AUX_THREADS), 0, st, C, ldc,
                       m, n, p, beta, 1.0 / (double)p);
    return hipGetLastError();
}

hipError_t launch_split_reduce(const uint32_t *part, int nsplit, int64_t m, int64_t n,
                               uint32_t *C, int64_t ldc, uint32_t p, uint32_t alpha,
                               uint32_t beta, hipStream_t st)
{
    hipLaunchKernelGGL(k_split_reduce, dim3(grid_for(m * n)), dim3(AUX_THREADS), 0, st, part,
                       nsplit, m, n, C, ldc, p, alpha, beta, 1.0 / (double)p);
    return hipGetLastError();
}

hipError_t launch_validate(const uint32_t *X, int64_t ld, int64_t rows,
                           int64_t cols, uint32_t p, unsigned *bad,
                           hipStream_t st)
{
    hipLaunchKernelGGL(k_validate, dim3(grid_for(rows * cols)), dim3(AUX_THREADS), 0, st,
                       X, ld, rows, cols, p, bad);
    return hipGetLastError();
}

} // namespace ff
