// Kernels of the triangular solve op(T) X = alpha B (mod p), Section 4.
//
// The solve runs on a normalised copy T' = D^-1 op(T) with unit diagonal (D
// the diagonal of op(T)): the system T' X = alpha D^-1 B involves ring
// operations only (Section 4.2), so the products can be summed over Z with
// reductions delayed.  Three element-wise passes prepare it (diagonal
// inverses, T', the scaled right-hand side) and one kernel solves a
// diagonal block of at most 64 rows for all columns of B; the updates
// between diagonal blocks are fgemm calls (trsm.cpp).
#include "ff_device.h"
#include "ff_internal.h"

namespace ff {

namespace {

constexpr int TT = 256;

// op(T)(i, j) for T stored row-major with leading dimension ldt.
__device__ __forceinline__ uint32_t op_t(const uint32_t *T, int64_t ldt, int trans, int64_t i,
                                         int64_t j)
{
    return trans ? T[j * ldt + i] : T[i * ldt + j];
}

// Inverse of a modulo p by the extended Euclidean algorithm; 0 when a is
// not a unit (gcd(a, p) != 1).
__device__ __forceinline__ uint32_t inv_mod(uint32_t a, uint32_t p)
{
    int64_t r0 = p, r1 = a % p, s0 = 0, s1 = 1;
    while (r1 != 0) {
        const int64_t q = r0 / r1, r2 = r0 - q * r1, s2 = s0 - q * s1;
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
        d = inv_mod(T[i * ldt + i], p);
        if (d == 0) atomicAdd(bad, 1u);
    }
    dinv[i] = d;
}

// T'(i, j) = dinv_i op(T)(i, j) inside the triangle, 1 on the diagonal, 0
// elsewhere; row-major with leading dimension m.
__global__ __launch_bounds__(TT) void k_trsm_prep(const uint32_t *T, int64_t ldt, int trans,
                                                  int lower, int64_t m, uint32_t p, double pinv,
                                                  const uint32_t *dinv, uint32_t *Tn)
{
    const int64_t total = m * m;
    for (int64_t e = (int64_t)blockIdx.x * TT + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * TT) {
        const int64_t i = e / m, j = e - i * m;
        uint32_t v = 0;
        if (i == j) v = 1;
        else if (lower ? j < i : j > i) v = mulmod(dinv[i], op_t(T, ldt, trans, i, j), p, pinv);
        Tn[e] = v;
    }
}

// B(i, j) <- alpha dinv_i B(i, j) mod p.
__global__ __launch_bounds__(TT) void k_trsm_scale(uint32_t *B, int64_t ldb, int64_t m,
                                                   int64_t n, uint32_t p, double pinv,
                                                   uint32_t alpha, const uint32_t *dinv)
{
    const int64_t total = m * n;
    for (int64_t e = (int64_t)blockIdx.x * TT + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * TT) {
        const int64_t i = e / n, j = e - i * n;
        uint32_t *bp = B + i * ldb + j;
        *bp = mulmod(mulmod(alpha, dinv[i], p, pinv), *bp, p, pinv);
    }
}

// Diagonal block: rows [r0, r0 + bs) of the unit triangular system T' X = B,
// bs <= TRSM_BS, every other row's contribution already subtracted.  One
// thread per column of B holds the block's column in registers and
// substitutes in the triangle's order (forward for lower, backward for
// upper); the block of T' sits in LDS and every lane reads the same word.
// EXACT: values centered in binary64, x_i = r(b_i - sum_l t_il x_l) with one
// reduction r per row, exact while TRSM_BS (p/2)^2 + p/2 <= 2^53 (the
// delayed reduction of Section 2.1.2 on the substitution's dot products);
// otherwise 32-bit residues and a reduction per product.  Rows past bs are
// zero in registers and in LDS and do not change the others.
template <bool EXACT>
__global__ __launch_bounds__(TT) void k_trsm_diag(const uint32_t *Tn, int64_t m, int lower,
                                                  int64_t r0, int bs, uint32_t *B, int64_t ldb,
                                                  int64_t n, uint32_t p, double pinv)
{
    constexpr int BS = TRSM_BS;
    __shared__ double sT[EXACT ? BS * BS : 1];
    __shared__ uint32_t sU[EXACT ? 1 : BS * BS];
    const uint32_t half = (p - 1) / 2;
    const double pd = (double)p;
    for (int e = threadIdx.x; e < BS * BS; e += TT) {
        const int i = e / BS, l = e % BS;
        const bool in = i < bs && l < bs && (lower ? l < i : l > i);
        const uint32_t t = in ? Tn[(r0 + i) * m + r0 + l] : 0u;
        if (EXACT) sT[e] = (double)center(t, p, half);
        else sU[e] = t ? p - t : 0u; // -t mod p
    }
    __syncthreads();
    const int64_t j = (int64_t)blockIdx.x * TT + threadIdx.x;
    if (j >= n) return;
    uint32_t *col = B + r0 * ldb + j;
    if (EXACT) {
        double x[BS];
#pragma unroll
        for (int i = 0; i < BS; ++i)
            x[i] = i < bs ? (double)center(col[(int64_t)i * ldb], p, half) : 0.0;
#pragma unroll
        for (int s = 0; s < BS; ++s) {
            const int i = lower ? s : BS - 1 - s;
            double acc = x[i];
#pragma unroll
            for (int t = 0; t < s; ++t) {
                const int l = lower ? t : BS - 1 - t;
                acc = __builtin_fma(-sT[i * BS + l], x[l], acc);
            }
            x[i] = __builtin_fma(-__builtin_rint(acc * pinv), pd, acc); // |x_i| <= p/2 + 1
        }
#pragma unroll
        for (int i = 0; i < BS; ++i)
            if (i < bs) col[(int64_t)i * ldb] = canon_f64(x[i], pd, pinv, p);
    } else {
        uint32_t x[BS];
#pragma unroll
        for (int i = 0; i < BS; ++i) x[i] = i < bs ? col[(int64_t)i * ldb] : 0u;
#pragma unroll
        for (int s = 0; s < BS; ++s) {
            const int i = lower ? s : BS - 1 - s;
            uint32_t acc = x[i];
#pragma unroll
            for (int t = 0; t < s; ++t) {
                const int l = lower ? t : BS - 1 - t;
                acc = addmod(acc, mulmod(sU[i * BS + l], x[l], p, pinv), p);
            }
            x[i] = acc;
        }
#pragma unroll
        for (int i = 0; i < BS; ++i)
            if (i < bs) col[(int64_t)i * ldb] = x[i];
    }
}

int grid_for(int64_t total)
{
    int64_t g = (total + TT - 1) / TT;
    if (g > 65536) g = 65536;
    return g < 1 ? 1 : (int)g;
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
                            uint32_t p, const uint32_t *dinv, uint32_t *Tn, hipStream_t st)
{
    hipLaunchKernelGGL(k_trsm_prep, dim3(grid_for(m * m)), dim3(TT), 0, st, T, ldt, trans, lower,
                       m, p, 1.0 / (double)p, dinv, Tn);
    return hipGetLastError();
}

hipError_t launch_trsm_scale(uint32_t *B, int64_t ldb, int64_t m, int64_t n, uint32_t p,
                             uint32_t alpha, const uint32_t *dinv, hipStream_t st)
{
    hipLaunchKernelGGL(k_trsm_scale, dim3(grid_for(m * n)), dim3(TT), 0, st, B, ldb, m, n, p,
                       1.0 / (double)p, alpha, dinv);
    return hipGetLastError();
}

hipError_t launch_trsm_diag(const uint32_t *Tn, int64_t m, int lower, int64_t r0, int bs,
                            uint32_t *B, int64_t ldb, int64_t n, uint32_t p, int exact,
                            hipStream_t st)
{
    const dim3 grid((unsigned)((n + TT - 1) / TT));
    if (exact)
        hipLaunchKernelGGL(k_trsm_diag<true>, grid, dim3(TT), 0, st, Tn, m, lower, r0, bs, B, ldb,
                           n, p, 1.0 / (double)p);
    else
        hipLaunchKernelGGL(k_trsm_diag<false>, grid, dim3(TT), 0, st, Tn, m, lower, r0, bs, B,
                           ldb, n, p, 1.0 / (double)p);
    return hipGetLastError();
}

} // namespace ff
