// Digit slicer of the INT8 path: operand -> packed signed digit planes.
//
// A centered residue c (|c| <= p/2) is written c = sum_{i<S} d_i R^i with
// R = 2^bits and digits d_i in [-R/2, R/2 - 1] (one direct int8 plane when c
// already fits int8).  The planes are zero padded and packed: for a row
// tile of RT rows and the K range padded to KP, the 16-byte group (row r,
// k/16) of digit d sits at
//     d*plane + (r/RT)*RT*KP + (k/16)*RT*16 + (r%RT)*16,
// the layout the INT8 GEMM copies into LDS stage by stage.
#include "ff_device.h"
#include "ff_internal.h"
#include "ff_operand.h"

namespace ff {

namespace {

__device__ __forceinline__ void slice_block(const SliceJob &J, int b, UnitTile &tile)
{
    uint32_t u[16];
    int r, kc;
    if (!load_unit(J, b, tile, u, r, kc)) return;
    const uint32_t half = (J.p - 1) / 2;
    int32_t v[16];
#pragma unroll
    for (int e = 0; e < 16; ++e)
        v[e] = J.in_mode == IN_SIGNED ? (int32_t)u[e] : center(u[e], J.p, half);

    write_digits(J, J.D, v, r, kc);
}

// Both operands of one product in one launch: blocks [0, blocks_a) slice
// a, the rest b.
__global__ __launch_bounds__(UNIT_THREADS) void k_slice2(SliceJob a, SliceJob b, int blocks_a)
{
    __shared__ UnitTile tile;
    const int blk = blockIdx.x;
    if (blk < blocks_a)
        slice_block(a, blk, tile);
    else
        slice_block(b, blk - blocks_a, tile);
}

__global__ __launch_bounds__(UNIT_THREADS) void k_slice_batched(
    const SliceJob *__restrict__ jobs, int njobs)
{
    __shared__ UnitTile tile;
    int lo = 0, hi = njobs - 1;
    const int b = blockIdx.x;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].block_start <= b) lo = mid; else hi = mid - 1;
    }
    const SliceJob J = jobs[lo];
    slice_block(J, b - J.block_start, tile);
}

} // namespace

hipError_t launch_slice2(const SliceJob &a, const SliceJob &b, hipStream_t st)
{
    const int na = unit_blocks(a), nb = unit_blocks(b);
    hipLaunchKernelGGL(k_slice2, dim3((unsigned)(na + nb)), dim3(UNIT_THREADS), 0, st, a, b, na);
    return hipGetLastError();
}

hipError_t launch_slice_batched(const SliceJob *dev_jobs, int njobs,
                                int total_blocks, hipStream_t st)
{
    hipLaunchKernelGGL(k_slice_batched, dim3(total_blocks), dim3(UNIT_THREADS), 0, st,
                       dev_jobs, njobs);
    return hipGetLastError();
}

int slice_blocks(const SliceJob &J) { return unit_blocks(J); }

} // namespace ff
