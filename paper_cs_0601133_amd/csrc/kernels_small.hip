// Small products on the FP64 path in one launch.
//
// For small m, n and k the general FP64 path (pack the operands to doubles,
// GEMM, with few tiles a K split and its reduction pass) is three launches
// of a few microseconds each on a mostly idle chip.  Here one workgroup
// computes a 16 x 16 block of C straight from the uint32 residues, its four
// waves splitting K: wave w takes the 64-deep K stages w, w + 4, w + 8, ..
// Each stage is read coalesced, centered (Section 2.1.2) and converted to
// binary64 on its way into the wave's own LDS area, and multiplied on
// v_mfma_f64_16x16x4 with the reduction delayed by the same K-block as the
// general path (eq. (2) with the binary64 exactness limit).  The four
// partial blocks, each reduced, meet in LDS; alpha, beta and the final
// reduction are applied there.  The words of a wave's next two stages are in
// flight in registers while a stage is multiplied (all of K up to 512 is
// requested at the start).
#include "ff_device.h"
#include "ff_internal.h"

namespace ff {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int ST = 16;        // C block edge (one MFMA block)
constexpr int SKS = 64;       // K per stage
constexpr int NW = 4;         // waves, splitting K
constexpr int STH = 64 * NW;  // threads
constexpr int RING = 2;       // stages of one wave loaded ahead

// Position of this lane's i-th word (i < 16) of a stage: A is 16 rows x 64,
// B is 64 x 16 columns; consecutive lanes take consecutive addresses for
// either storage order.
__device__ __forceinline__ void a_pos(int ta, int l, int i, int &r, int &kk)
{
    if (ta) { r = l & 15; kk = (l >> 4) + 4 * i; }
    else { kk = l; r = i; }
}
__device__ __forceinline__ void b_pos(int tb, int l, int i, int &c, int &kk)
{
    if (tb) { kk = l; c = i; }
    else { c = l & 15; kk = (l >> 4) + 4 * i; }
}

// This lane's words of the stage at k0, from addresses clamped into the
// operands: the loads carry no condition (entries outside the operands are
// zeroed when the stage is stored to LDS), so they are all in flight
// together.
__device__ __forceinline__ void load_stage(const F64Small &J, int m0, int n0, int k0, int l,
                                           uint32_t (&ra)[16], uint32_t (&rb)[16])
{
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        int r, kk;
        a_pos(J.ta, l, i, r, kk);
        const int gr = min(m0 + r, J.m - 1), gk = min(k0 + kk, J.k - 1);
        ra[i] = J.ta ? J.A[(int64_t)gk * J.lda + gr] : J.A[(int64_t)gr * J.lda + gk];
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        int c, kk;
        b_pos(J.tb, l, i, c, kk);
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

__global__ __launch_bounds__(STH) void k_fgemm_f64_small(F64Small J)
{
    __shared__ double sA[NW][ST][SKS + 1]; // per wave: (row, k)
    __shared__ double sB[NW][SKS][ST + 1]; // per wave: (k, column)
    __shared__ double sR[NW][ST * ST];     // per wave: partial block, reduced
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int m0 = blockIdx.y * ST, n0 = blockIdx.x * ST;
    const uint32_t half = (J.p - 1) / 2;
    const int nst = (J.k + SKS - 1) / SKS;
    // thread t finishes entry (t / 16, t % 16) of the block; its entry of C
    // is requested now (clamped into C, no branch) so that the read is done
    // by the time the products are
    const int gr = m0 + (t >> 4), gc = n0 + (t & 15);
    const uint32_t cin = J.beta ? J.C[(int64_t)min(gr, J.m - 1) * J.ldc + min(gc, J.n - 1)] : 0u;

    // two accumulators (even and odd steps) halve the dependent chain; the
    // K-block counts the products of both
    v4d acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
    int since_fold = 0;
    uint32_t ra[RING][16], rb[RING][16];
#pragma unroll
    for (int q = 0; q < RING; ++q) {
        const int st = w + NW * q;
        if (st < nst) load_stage(J, m0, n0, st * SKS, lane, ra[q], rb[q]);
    }
    const double *pa = &sA[w][lane & 15][lane >> 4];
    const double *pb = &sB[w][lane >> 4][lane & 15];
    // rounds of NW stages (one per wave); the trip counts are the same in
    // every wave, so every wave reaches every barrier
    for (int g0 = 0; g0 < nst; g0 += NW * RING) {
#pragma unroll
        for (int q = 0; q < RING; ++q) {
            const int round0 = g0 + NW * q;
            if (round0 >= nst) break;
            const int st = round0 + w; // this wave's stage
            const bool act = st < nst;
            const int k0 = st * SKS;
            if (act) {
#pragma unroll
                for (int i = 0; i < 16; ++i) {
                    int r, kk;
                    a_pos(J.ta, lane, i, r, kk);
                    const bool in = m0 + r < J.m && k0 + kk < J.k;
                    sA[w][r][kk] = in ? (double)center(ra[q][i], J.p, half) : 0.0;
                }
#pragma unroll
                for (int i = 0; i < 16; ++i) {
                    int c, kk;
                    b_pos(J.tb, lane, i, c, kk);
                    const bool in = n0 + c < J.n && k0 + kk < J.k;
                    sB[w][kk][c] = in ? (double)center(rb[q][i], J.p, half) : 0.0;
                }
            }
            __syncthreads();
            if (act) {
                // this ring slot takes the wave's stage RING rounds ahead
                if (st + NW * RING < nst)
                    load_stage(J, m0, n0, (st + NW * RING) * SKS, lane, ra[q], rb[q]);
                const int steps = min(SKS, J.k - k0 + 3) / 4; // zero padding adds nothing
                if (J.fold_steps >= 2) {
                    // pairs of steps, one per accumulator; a fold comes
                    // before any pair that would exceed the K-block
                    int s = 0;
                    for (; s + 2 <= steps; s += 2) {
                        if (since_fold + 2 > J.fold_steps) {
                            fold(acc0, J.pd, J.pinv);
                            fold(acc1, J.pd, J.pinv);
                            since_fold = 0;
                        }
                        acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(
                            pa[4 * s], pb[4 * s * (ST + 1)], acc0, 0, 0, 0);
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
                        acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(
                            pa[4 * s], pb[4 * s * (ST + 1)], acc0, 0, 0, 0);
                        since_fold += 1;
                    }
                } else {
                    // a K-block of 4..7 products: fold after every step
                    for (int s = 0; s < steps; ++s) {
                        acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(
                            pa[4 * s], pb[4 * s * (ST + 1)], acc0, 0, 0, 0);
                        fold(acc0, J.pd, J.pinv);
                    }
                }
            }
            __syncthreads(); // every wave is done with its stage before it is overwritten
        }
    }

    // Partial blocks: the lane holds column lane%16 of rows lane/16 + 4r;
    // each accumulator is reduced first (|.| <= p/2 + 2), so every sum below
    // is exact whatever the carries.
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const double e0 = __builtin_fma(-__builtin_rint(acc0[r] * J.pinv), J.pd, acc0[r]);
        const double e1 = __builtin_fma(-__builtin_rint(acc1[r] * J.pinv), J.pd, acc1[r]);
        sR[w][((lane >> 4) + 4 * r) * ST + (lane & 15)] = e0 + e1;
    }
    __syncthreads();
    if (gr < J.m && gc < J.n) {
        double x = 0.0;
#pragma unroll
        for (int v = 0; v < NW; ++v) x += sR[v][t];
        const uint32_t val = canon_f64(x, J.pd, J.pinv, J.p);
        uint32_t out = mulmod(J.alpha, val, J.p, J.pinv);
        if (J.beta) out = addmod(out, mulmod(J.beta, cin, J.p, J.pinv), J.p);
        J.C[(int64_t)gr * J.ldc + gc] = out;
    }
}

} // namespace

hipError_t launch_f64_small(const F64Small &J, hipStream_t st)
{
    if (J.m <= 0 || J.n <= 0 || J.k <= 0 || J.fold_steps < 1) return hipErrorInvalidValue;
    if ((J.m + ST - 1) / ST > 65535) return hipErrorInvalidValue;
    const dim3 grid((unsigned)((J.n + ST - 1) / ST), (unsigned)((J.m + ST - 1) / ST));
    hipLaunchKernelGGL(k_fgemm_f64_small, grid, dim3(STH), 0, st, J);
    return hipGetLastError();
}

} // namespace ff
