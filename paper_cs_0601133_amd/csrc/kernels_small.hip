// Small products on the FP64 path in one launch.
//
// For small m, n and k the general FP64 path (pack the operands to doubles,
// GEMM, with few tiles a K split and its reduction pass) is three launches
// of a few microseconds each on a mostly idle chip.  Here one workgroup of
// four waves computes a 32 x 32 tile of C straight from the uint32
// residues: each 64-deep K stage is read coalesced, centered (Section 2.1.2)
// and converted to binary64 on its way into LDS, the products run on
// v_mfma_f64_16x16x4 with the reduction delayed by the same K-block as the
// general path (eq. (2) with the binary64 exactness limit), and alpha, beta
// and the final reduction are applied in the epilogue.  The words of the
// next four K stages are in flight in registers while a stage is
// multiplied (all of K up to 256 is requested at the start).
#include "ff_device.h"
#include "ff_internal.h"

namespace ff {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int ST = 32;   // C tile edge
constexpr int SKS = 64;  // K per stage
constexpr int STH = 256; // threads: four waves, one 16 x 16 block each

// Position of this thread's i-th word of the A stage (32 rows x 64) and
// of the B stage (64 x 32 columns): consecutive threads take consecutive
// addresses for either storage order.
__device__ __forceinline__ void a_pos(int ta, int t, int i, int &r, int &kk)
{
    if (ta) { r = t & 31; kk = (t >> 5) + 8 * i; }
    else { kk = t & 63; r = (t >> 6) + 4 * i; }
}
__device__ __forceinline__ void b_pos(int tb, int t, int i, int &c, int &kk)
{
    if (tb) { kk = t & 63; c = (t >> 6) + 4 * i; }
    else { c = t & 31; kk = (t >> 5) + 8 * i; }
}

// This thread's words of the stage at k0, from addresses clamped into the
// operands: the loads carry no condition (entries outside the operands are
// zeroed when the stage is stored to LDS), so they are all in flight
// together.
__device__ __forceinline__ void load_stage(const F64Small &J, int m0, int n0, int k0,
                                           uint32_t (&ra)[8], uint32_t (&rb)[8])
{
    const int t = threadIdx.x;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        int r, kk;
        a_pos(J.ta, t, i, r, kk);
        const int gr = min(m0 + r, J.m - 1), gk = min(k0 + kk, J.k - 1);
        ra[i] = J.ta ? J.A[(int64_t)gk * J.lda + gr] : J.A[(int64_t)gr * J.lda + gk];
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        int c, kk;
        b_pos(J.tb, t, i, c, kk);
        const int gc = min(n0 + c, J.n - 1), gk = min(k0 + kk, J.k - 1);
        rb[i] = J.tb ? J.B[(int64_t)gc * J.ldb + gk] : J.B[(int64_t)gk * J.ldb + gc];
    }
}

// acc <- acc mod p, centered up to the quotient estimate (|acc| <= p/2 + 2)
__device__ __forceinline__ void fold(v4d &acc, double pd, double pinv)
{
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[r] = __builtin_fma(-__builtin_rint(acc[r] * pinv), pd, acc[r]);
}

constexpr int RING = 4; // K stages whose words are loaded ahead (all of K <= 256 at once)

__global__ __launch_bounds__(STH) void k_fgemm_f64_small(F64Small J)
{
    __shared__ double sA[ST][SKS + 1]; // (row, k)
    __shared__ double sB[SKS][ST + 1]; // (k, column)
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int m0 = blockIdx.y * ST, n0 = blockIdx.x * ST;
    const int wr = (w >> 1) * 16, wc = (w & 1) * 16;
    const uint32_t half = (J.p - 1) / 2;

    // two accumulators (even and odd steps) halve the dependent chain; the
    // K-block counts the products of both
    v4d acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
    int since_fold = 0;
    uint32_t ra[RING][8], rb[RING][8];
#pragma unroll
    for (int q = 0; q < RING; ++q)
        if (q * SKS < J.k) load_stage(J, m0, n0, q * SKS, ra[q], rb[q]);
    for (int g0 = 0; g0 < J.k; g0 += RING * SKS) {
#pragma unroll
        for (int q = 0; q < RING; ++q) {
            const int k0 = g0 + q * SKS;
            if (k0 >= J.k) break;
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                int r, kk;
                a_pos(J.ta, t, i, r, kk);
                const bool in = m0 + r < J.m && k0 + kk < J.k;
                sA[r][kk] = in ? (double)center(ra[q][i], J.p, half) : 0.0;
            }
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                int c, kk;
                b_pos(J.tb, t, i, c, kk);
                const bool in = n0 + c < J.n && k0 + kk < J.k;
                sB[kk][c] = in ? (double)center(rb[q][i], J.p, half) : 0.0;
            }
            __syncthreads();
            // this ring slot takes the stage RING ahead
            if (k0 + RING * SKS < J.k) load_stage(J, m0, n0, k0 + RING * SKS, ra[q], rb[q]);
            const int steps = min(SKS, J.k - k0 + 3) / 4; // zero padding past k adds nothing
            const double *pa = &sA[wr + (lane & 15)][lane >> 4];
            const double *pb = &sB[lane >> 4][wc + (lane & 15)];
            if (J.fold_steps >= 2) {
                // pairs of steps, one per accumulator; a fold comes before
                // any pair that would exceed the K-block
                int s = 0;
                for (; s + 2 <= steps; s += 2) {
                    if (since_fold + 2 > J.fold_steps) {
                        fold(acc0, J.pd, J.pinv);
                        fold(acc1, J.pd, J.pinv);
                        since_fold = 0;
                    }
                    acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(pa[4 * s], pb[4 * s * (ST + 1)],
                                                                acc0, 0, 0, 0);
                    acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(
                        pa[4 * (s + 1)], pb[4 * (s + 1) * (ST + 1)], acc1, 0, 0, 0);
                    since_fold += 2;
                }
                if (s < steps) {
                    if (since_fold + 1 > J.fold_steps) {
                        fold(acc0, J.pd, J.pinv);
                        fold(acc1, J.pd, J.pinv);
                        since_fold = 0;
                    }
                    acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(pa[4 * s], pb[4 * s * (ST + 1)],
                                                                acc0, 0, 0, 0);
                    since_fold += 1;
                }
            } else {
                // a K-block of 4..7 products: fold after every step
                for (int s = 0; s < steps; ++s) {
                    acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(pa[4 * s], pb[4 * s * (ST + 1)],
                                                                acc0, 0, 0, 0);
                    fold(acc0, J.pd, J.pinv);
                }
            }
            __syncthreads(); // every wave is done with the stage before it is overwritten
        }
    }

    // Epilogue: the lane holds column lane%16 of rows lane/16 + 4r.
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int gr = m0 + wr + (lane >> 4) + 4 * r;
        const int gc = n0 + wc + (lane & 15);
        if (gr < J.m && gc < J.n) {
            // each accumulator is reduced first (|.| <= p/2 + 2), so the sum
            // is exact whatever the carries
            const double e0 = __builtin_fma(-__builtin_rint(acc0[r] * J.pinv), J.pd, acc0[r]);
            const double e1 = __builtin_fma(-__builtin_rint(acc1[r] * J.pinv), J.pd, acc1[r]);
            const uint32_t v = canon_f64(e0 + e1, J.pd, J.pinv, J.p);
            uint32_t out = mulmod(J.alpha, v, J.p, J.pinv);
            uint32_t *cp = J.C + (int64_t)gr * J.ldc + gc;
            if (J.beta) out = addmod(out, mulmod(J.beta, *cp, J.p, J.pinv), J.p);
            *cp = out;
        }
    }
}

} // namespace

hipError_t launch_f64_small(const F64Small &J, hipStream_t st)
{
    if (J.m <= 0 || J.n <= 0 || J.k <= 0 || J.fold_steps < 1) return hipErrorInvalidValue;
    const dim3 grid((unsigned)((J.n + ST - 1) / ST), (unsigned)((J.m + ST - 1) / ST));
    hipLaunchKernelGGL(k_fgemm_f64_small, grid, dim3(STH), 0, st, J);
    return hipGetLastError();
}

} // namespace ff
