// Operand reads of the slicing and packing kernels.
//
// A unit is row r of the logical rows x K operand (A as m x k, B^T as
// n x k) with its 16 columns 16*kc .. 16*kc + 15, zero outside the operand.
// Blocks of 256 threads cover 256 units:
//   * K-contiguous storage (trans == 0): a block covers 64 rows x 4 chunks.
//     It reads the 64 x 64 tile with 16 lanes per row (256 contiguous bytes,
//     16-byte loads when aligned) into LDS, and each thread then takes its
//     unit from there;
//   * row-contiguous storage (trans == 1): thread q of the operand takes row
//     q % rows_pad and chunk q / rows_pad; consecutive threads read
//     consecutive addresses.
// Either way consecutive threads hold consecutive rows of one chunk, so the
// packed words they write are contiguous.
#pragma once

#include "ff_internal.h"

namespace ff {

constexpr int UNIT_THREADS = 256;

// Blocks of UNIT_THREADS that cover an operand (rows_pad a multiple of 64).
__host__ __device__ inline int unit_blocks(const SliceJob &J)
{
    const int nchunk = J.KP / 16;
    if (J.trans) return (int)(((int64_t)J.rows_pad * nchunk + UNIT_THREADS - 1) / UNIT_THREADS);
    return (J.rows_pad / 64) * ((nchunk + 3) / 4);
}

typedef uint32_t UnitTile[64][65]; // padded: column reads hit distinct banks

// Raw words of this thread's unit in block b (the whole block must call
// it).  Returns false if the thread has no unit.
__device__ __forceinline__ bool load_unit(const SliceJob &J, int b, UnitTile &tile,
                                          uint32_t *v, int &r, int &kc)
{
    const int nchunk = J.KP / 16;
    const int t = threadIdx.x;
    const uint32_t *X = (const uint32_t *)J.X;
    if (J.trans) {
        const int64_t q = (int64_t)b * UNIT_THREADS + t;
        if (q >= (int64_t)J.rows_pad * nchunk) return false;
        r = (int)(q % J.rows_pad);
        kc = (int)(q / J.rows_pad);
        const int k0 = kc * 16;
        const bool row_ok = r < J.rows;
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const bool ok = row_ok && (k0 + e) < J.K;
            v[e] = ok ? X[(int64_t)(k0 + e) * J.ldx + r] : 0u;
        }
        return true;
    }
    const int nrb = J.rows_pad / 64;
    const int r0 = (b % nrb) * 64, kc0 = (b / nrb) * 4;
    const bool vec = (J.ldx & 3) == 0 && (((uintptr_t)X) & 15) == 0;
    const int g = t & 15;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int rr = (t >> 4) + 16 * i;
        const int rg = r0 + rr, kg = kc0 * 16 + 4 * g;
        uint32_t w[4] = {0u, 0u, 0u, 0u};
        if (rg < J.rows) {
            const uint32_t *src = X + (int64_t)rg * J.ldx + kg;
            if (vec && kg + 3 < J.K) {
                const uint4 q = *(const uint4 *)src;
                w[0] = q.x; w[1] = q.y; w[2] = q.z; w[3] = q.w;
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e) w[e] = kg + e < J.K ? src[e] : 0u;
            }
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) tile[rr][4 * g + e] = w[e];
    }
    __syncthreads();
    r = r0 + (t & 63);
    kc = kc0 + (t >> 6);
#pragma unroll
    for (int e = 0; e < 16; ++e) v[e] = tile[t & 63][(t >> 6) * 16 + e];
    return kc < nchunk;
}

} // namespace ff
