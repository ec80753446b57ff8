// INT8 matrix-core fgemm with digit pairing.
//
// With residues split into S signed 7-bit digits (a = sum a_i R^i), the
// digit-product sums E_t = sum_{i+j=t} A_i B_j of the plain digit kernel
// take S^2 matrix-core products.  Karatsuba's identity for one pair of
// digits, a_i b_j + a_j b_i = (a_i + a_j)(b_i + b_j) - a_i b_i - a_j b_j,
// gives the same result from S(S+1)/2 products: the S diagonal products
// D_i = A_i B_i and, for every pair i < j, the product of the digit sums
// (A_i + A_j)(B_i + B_j), accumulated per weight t = i + j into K_t.  A sum
// of two 7-bit digits lies in [-128, 126], so the sum planes (written by the
// slicer after the digit planes) are int8 operands like the digits.  The
// epilogue recombines sum_t R^t K_t + sum_i D_i (R^(2i) - sum_{j != i}
// R^(i+j)) modulo p with weights computed on the host.
//
// Each operand plane enters exactly one product, so a wave reads two
// fragments per matrix-core step (the plain kernel reuses each fragment S
// times): the pairing trades S^2 - S(S+1)/2 products for S(S-1)/2 more
// planes to move.
#include "ff_device.h"
#include "ff_internal.h"
#include "ff_ring.h"

namespace ff {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int PKS = 32; // K bytes per LDS stage: one 32-deep matrix-core step

template <int S>
struct PCfg {
    static constexpr int NP = S * (S + 1) / 2; // planes per operand
    static constexpr int NSET = 3 * S - 3;     // D_0 .. D_{S-1}, K_1 .. K_{2S-3}
    static constexpr int WGM = S >= 5 ? 2 : 4, WGN = 2;
    static constexpr int BM = 32 * WGM, BN = 32 * WGN;
    static constexpr int NW = WGM * WGN;
    static constexpr int A_BYTES = NP * BM * PKS, B_BYTES = NP * BN * PKS;
    static constexpr int STAGE = A_BYTES + B_BYTES;
    static constexpr int CHUNKS = STAGE / 1024;
    static constexpr int PER_WAVE = (CHUNKS + NW - 1) / NW;
    static constexpr int FIT = LDS_LIMIT / STAGE;
    static constexpr int NST = FIT > 4 ? 4 : FIT;
    static_assert(NST >= 2, "two stages must fit in LDS");
    static_assert(STAGE % 1024 == 0 && (BM * PKS) % 1024 == 0 && (BN * PKS) % 1024 == 0,
                  "stages are whole 1 KB chunks");
    static constexpr int WPE = NW / 4 > 0 ? NW / 4 : 1; // waves per SIMD
};

// Accumulator set of operand plane x: D_x for a digit plane, K_{i+j} for
// the sum plane of the pair (i, j) (pairs in lexicographic order).
template <int S>
__host__ __device__ constexpr int plane_set(int x)
{
    if (x < S) return x;
    int q = x - S;
    for (int i = 0; i < S; ++i)
        for (int j = i + 1; j < S; ++j) {
            if (q == 0) return S + (i + j) - 1;
            --q;
        }
    return -1;
}

template <class C>
__device__ __forceinline__ int issue_pstage(const I8Job &J, int tm, int tn, int kt,
                                            char *lds_stage, int wave, int lane)
{
    const char *Abase = (const char *)J.Ad + (int64_t)tm * C::BM * J.KP + (int64_t)kt * C::BM * PKS;
    const char *Bbase = (const char *)J.Bd + (int64_t)tn * C::BN * J.KP + (int64_t)kt * C::BN * PKS;
    constexpr int ABLK = C::BM * PKS, BBLK = C::BN * PKS;
    int issued = 0;
#pragma unroll
    for (int i = 0; i < C::PER_WAVE; ++i) {
        const int c = wave + i * C::NW;
        if (C::CHUNKS % C::NW == 0 || c < C::CHUNKS) {
            const int off = c * 1024;
            const char *src;
            if (off < C::A_BYTES) {
                const int d = off / ABLK;
                src = Abase + (int64_t)d * J.a_plane + (off - d * ABLK);
            } else {
                const int o = off - C::A_BYTES;
                const int d = o / BBLK;
                src = Bbase + (int64_t)d * J.b_plane + (o - d * BBLK);
            }
            __builtin_amdgcn_global_load_lds((const void *)(src + lane * 16),
                                             (lds_ptr)(lds_stage + off), 16, 0, 0);
            ++issued;
        }
    }
    return issued;
}

__device__ __forceinline__ uint32_t mod_i32p(int32_t e, uint32_t p, double pd, double pinv)
{
    const double x = (double)e;
    const double r = __builtin_fma(-__builtin_rint(x * pinv), pd, x);
    int64_t ri = (int64_t)r; // |ri| <= p/2 + 1
    ri += ri < 0 ? (int64_t)p : 0;
    ri += ri < 0 ? (int64_t)p : 0;
    ri -= ri >= (int64_t)p ? (int64_t)p : 0;
    return (uint32_t)ri;
}

template <int S>
__global__ __attribute__((amdgpu_flat_work_group_size(64 * PCfg<S>::NW, 64 * PCfg<S>::NW),
                          amdgpu_waves_per_eu(PCfg<S>::WPE, PCfg<S>::WPE)))
void k_fgemm_i8_pair(I8Job J)
{
    using C = PCfg<S>;
    constexpr int NST = C::NST;
    __shared__ __attribute__((aligned(1024))) char smem[NST * C::STAGE];
    const int G = J.tiles_m * J.tiles_n;
    int tm, tn;
    grouped_tile_rt(xcd_remap(blockIdx.x, G), J.tiles_m, J.tiles_n, J.gm, &tm, &tn);
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm0 = (wave / C::WGN) * 32, wn0 = (wave % C::WGN) * 32;

    v16i acc[C::NSET];
#pragma unroll
    for (int t = 0; t < C::NSET; ++t)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[t][v] = 0;

    const int nk = J.KP / PKS;
    int per_stage = 0;
#pragma unroll
    for (int st = 0; st < NST - 1; ++st)
        per_stage = issue_pstage<C>(J, tm, tn, st < nk ? st : nk - 1, smem + st * C::STAGE,
                                    wave, lane);
    const int cidx = lane >> 5; // which 16-byte half of the 32-deep step
    for (int kt = 0; kt < nk; ++kt) {
        // stage kt has landed once at most NST-2 later stages' loads of this
        // wave are outstanding; after the barrier every wave's part is in
        // LDS and the slot of stage kt-1 is free
        wait_vm((NST - 2) * per_stage);
        ring_barrier();
        const char *cur = smem + (kt % NST) * C::STAGE;
        const int nxt = kt + NST - 1;
        issue_pstage<C>(J, tm, tn, nxt < nk ? nxt : nk - 1, smem + (nxt % NST) * C::STAGE,
                        wave, lane);
#pragma unroll
        for (int x = 0; x < C::NP; ++x) {
            const v4i a = *(const v4i *)(cur + x * C::BM * PKS +
                                         (cidx * C::BM + wm0 + (lane & 31)) * 16);
            const v4i b = *(const v4i *)(cur + C::A_BYTES + x * C::BN * PKS +
                                         (cidx * C::BN + wn0 + (lane & 31)) * 16);
            acc[plane_set<S>(x)] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, acc[plane_set<S>(x)],
                                                                        0, 0, 0);
        }
    }
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");

    // Epilogue: lane holds column lane%32 and rows 8*(v/4) + 4*(lane/32) +
    // v%4 of the wave's 32 x 32 block; the recombination modes are those of
    // the plain digit kernel, over the NSET weighted sets.
    // (C is read for all 16 entries first, clamped into C so that no branch
    // surrounds the loads: one memory round trip instead of one per entry
    // behind each store.)
    const int m0 = tm * C::BM + wm0, n0 = tn * C::BN + wn0;
    uint32_t cin[16];
    if (J.beta) {
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int row = m0 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
            const int col = n0 + (lane & 31);
            cin[v] = J.C[(int64_t)min(row, J.m - 1) * J.ldc + min(col, J.n - 1)];
        }
    }
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const int row = m0 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
        const int col = n0 + (lane & 31);
        if (row < J.m && col < J.n) {
            uint32_t r;
            if (J.epi_direct) {
                double sum = 0.0;
#pragma unroll
                for (int t = 0; t < C::NSET; ++t)
                    sum = __builtin_fma(J.wc[t], (double)acc[t][v], sum);
                r = canon_f64(sum, J.pd, J.pinv, J.p);
            } else if (J.fp_epi) {
                double sum = 0.0;
#pragma unroll
                for (int t = 0; t < C::NSET; ++t) {
                    const double x = (double)acc[t][v];
                    const double e = __builtin_fma(-__builtin_rint(x * J.pinv), J.pd, x);
                    sum = __builtin_fma(J.wc[t], e, sum);
                }
                r = canon_f64(sum, J.pd, J.pinv, J.p);
            } else {
                r = 0;
#pragma unroll
                for (int t = 0; t < C::NSET; ++t)
                    r = addmod(r, mulmod(J.w[t], mod_i32p(acc[t][v], J.p, J.pd, J.pinv), J.p,
                                         J.pinv),
                               J.p);
            }
            if (J.beta) r = addmod(r, mulmod(J.beta, cin[v], J.p, J.pinv), J.p);
            J.C[(int64_t)row * J.ldc + col] = r;
        }
    }
}

template <int S>
hipError_t run_pair(const I8Job &J, hipStream_t st)
{
    hipLaunchKernelGGL(k_fgemm_i8_pair<S>, dim3(J.tiles_m * J.tiles_n),
                       dim3(64 * PCfg<S>::NW), 0, st, J);
    return hipGetLastError();
}

} // namespace

hipError_t launch_i8_pair(const I8Job &J, hipStream_t st)
{
    if (J.tiles_m * J.tiles_n <= 0) return hipSuccess;
    switch (J.s) {
    case 2: return run_pair<2>(J, st);
    case 3: return run_pair<3>(J, st);
    case 4: return run_pair<4>(J, st);
    case 5: return run_pair<5>(J, st);
    default: return hipErrorInvalidValue;
    }
}

} // namespace ff
