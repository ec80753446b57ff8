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

// K-contiguous storage: this thread's share of the 64 x 64 tile of block b
// (rows r0 + t/16 + 16i, columns 16*kc0 + 4*(t%16) ..), zero outside the
// operand.  Issues the global loads only.
__device__ __forceinline__ void load_raw(const SliceJob &J, int b, uint32_t (&w)[4][4])
{
    const uint32_t *X = (const uint32_t *)J.X;
    const int nrb = J.rows_pad / 64;
    const int r0 = (b % nrb) * 64, kc0 = (b / nrb) * 4;
    const bool vec = (J.ldx & 3) == 0 && (((uintptr_t)X) & 15) == 0;
    const int t = threadIdx.x, g = t & 15;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int rg = r0 + (t >> 4) + 16 * i, kg = kc0 * 16 + 4 * g;
#pragma unroll
        for (int e = 0; e < 4; ++e) w[i][e] = 0u;
        if (rg < J.rows) {
            const uint32_t *src = X + (int64_t)rg * J.ldx + kg;
            if (vec && kg + 3 < J.K) {
                const uint4 q = *(const uint4 *)src;
                w[i][0] = q.x; w[i][1] = q.y; w[i][2] = q.z; w[i][3] = q.w;
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e) w[i][e] = kg + e < J.K ? src[e] : 0u;
            }
        }
    }
}

// K-contiguous storage: the words of load_raw through the LDS tile to this
// thread's unit (the whole block must call it).  Returns false if the
// thread has no unit.
__device__ __forceinline__ bool unit_from_raw(const SliceJob &J, int b, UnitTile &tile,
                                              const uint32_t (&w)[4][4], uint32_t *v, int &r,
                                              int &kc)
{
    const int nrb = J.rows_pad / 64;
    const int r0 = (b % nrb) * 64, kc0 = (b / nrb) * 4;
    const int t = threadIdx.x, g = t & 15;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int e = 0; e < 4; ++e) tile[(t >> 4) + 16 * i][4 * g + e] = w[i][e];
    __syncthreads();
    r = r0 + (t & 63);
    kc = kc0 + (t >> 6);
#pragma unroll
    for (int e = 0; e < 16; ++e) v[e] = tile[t & 63][(t >> 6) * 16 + e];
    return kc < J.KP / 16;
}

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
    uint32_t w[4][4];
    load_raw(J, b, w);
    return unit_from_raw(J, b, tile, w, v, r, kc);
}

// Sum of two words of four signed bytes, byte by byte modulo 256 (no carry
// from one byte into the next): the low seven bits of each byte are added,
// and the top bit is the sum of the top bits and that carry, modulo 2.
__device__ __forceinline__ uint32_t add_bytes(uint32_t x, uint32_t y)
{
    const uint32_t low = (x & 0x7F7F7F7Fu) + (y & 0x7F7F7F7Fu);
    return low ^ ((x ^ y) & 0x80808080u);
}

// Writes the S balanced digits of the 16 values of unit (r, kc) into the
// packed planes at D (layout of the digit slicer: the 16-byte group (r, kc)
// of digit d at d*plane + (r/RT)*RT*KP + kc*RT*16 + (r%RT)*16); with
// J.pairs, planes S .. S(S+1)/2 - 1 then take the digit sums d_i + d_j,
// i < j (7-bit digits: the sums fit a signed byte).  v is consumed.
__device__ __forceinline__ void write_digits(const SliceJob &J, int8_t *D, int32_t *v, int r,
                                             int kc)
{
    const int bits = J.S == 1 ? 8 : J.bits;
    const int sh = 32 - bits;
    int8_t *dst = D + (int64_t)(r / J.RT) * J.RT * J.KP + (int64_t)kc * J.RT * 16 +
                  (int64_t)(r % J.RT) * 16;
    if (!J.pairs) {
        for (int d = 0; d < J.S; ++d) {
            uint32_t w[4] = {0, 0, 0, 0};
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                // balanced digit: the value in [-R/2, R/2) congruent to v mod
                // R, i.e. the low `bits` bits sign-extended
                const int dig = (int)((uint32_t)v[e] << sh) >> sh;
                v[e] = (v[e] - dig) >> bits; // exact division by R
                w[e >> 2] |= (uint32_t)(dig & 0xFF) << (8 * (e & 3));
            }
            *(uint4 *)(dst + (int64_t)d * J.plane) = make_uint4(w[0], w[1], w[2], w[3]);
        }
        return;
    }
    // digit pairing (S <= 5): the digits stay in registers for the sums
    uint4 dw[5];
#pragma unroll
    for (int d = 0; d < 5; ++d) {
        uint32_t w[4] = {0, 0, 0, 0};
        if (d < J.S) {
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const int dig = (int)((uint32_t)v[e] << sh) >> sh;
                v[e] = (v[e] - dig) >> bits;
                w[e >> 2] |= (uint32_t)(dig & 0xFF) << (8 * (e & 3));
            }
            *(uint4 *)(dst + (int64_t)d * J.plane) = make_uint4(w[0], w[1], w[2], w[3]);
        }
        dw[d] = make_uint4(w[0], w[1], w[2], w[3]);
    }
    int pl = J.S;
#pragma unroll
    for (int i = 0; i < 5; ++i)
#pragma unroll
        for (int j = i + 1; j < 5; ++j)
            if (j < J.S) {
                *(uint4 *)(dst + (int64_t)pl * J.plane) =
                    make_uint4(add_bytes(dw[i].x, dw[j].x), add_bytes(dw[i].y, dw[j].y),
                               add_bytes(dw[i].z, dw[j].z), add_bytes(dw[i].w, dw[j].w));
                ++pl;
            }
}

// Writes the 16 values of unit (r, kc) as binary64 into the packed operand
// at D (layout of the FP64 packing: element (r, k) at double offset
// (r/RT)*RT*KP + (k/16)*RT*16 + ((r%RT)/16)*256 + ((k%16)/2)*32 + (r%16)*2 +
// k%2; 16 consecutive rows write 256 contiguous bytes per 16-byte word).
__device__ __forceinline__ void write_f64(const SliceJob &J, double *D, const double *v, int r,
                                          int kc)
{
    typedef double v2d_ __attribute__((ext_vector_type(2)));
    double *dst = D + (int64_t)(r / J.RT) * J.RT * J.KP + (int64_t)kc * J.RT * 16 +
                  (int64_t)((r % J.RT) >> 4) * 256 + (r & 15) * 2;
#pragma unroll
    for (int c = 0; c < 8; ++c) *(v2d_ *)(dst + c * 32) = v2d_{v[2 * c], v[2 * c + 1]};
}

} // namespace ff
