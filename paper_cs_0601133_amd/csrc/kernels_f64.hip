// FP64 matrix-core fgemm: the "Zpz-double" design of Sections 2.1.2 and 3.1
// (residues converted to integer-valued doubles, products summed exactly by
// the floating-point unit, reduction delayed) on gfx950's v_mfma_f64_16x16x4.
//
// Two kernels, as in the paper's scheme of converting the operands once and
// then calling a floating-point matrix product:
//   * packing: each operand is centered (|c| <= p/2) and written as doubles
//     in a tile-packed layout (the F64Job comment in ff_internal.h), zero
//     padded, transposition resolved;
//   * GEMM: every K stage of a row tile is one contiguous block, copied
//     straight into an LDS ring by global_load_lds (no register staging, no
//     conversion work in the loop) and read back as one 16-byte word per lane
//     and two matrix-core steps.  Each wave owns 64 x 64 outputs (16 blocks
//     of 16 x 16) whose accumulators stay in VGPRs (the file is built with
//     the MFMA VGPR form), so the periodic reduction x - p*rint(x/p) costs no
//     register moves.  It runs often enough to keep every partial sum an
//     integer of magnitude <= kblock*max|ab| + p + 2 <= 2^53, hence exact in
//     whatever order the matrix core adds.  The epilogue makes the residue
//     canonical and applies alpha and beta modulo p.
#include "ff_device.h"
#include "ff_internal.h"
#include "ff_operand.h"
#include "ff_ring.h"

namespace ff {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef double v2d __attribute__((ext_vector_type(2)));

// Compiled configurations: id, WGM, WGN, NST, waves per SIMD, GM.
#define FF_F64_TILES(X)                                                        \
    X(0, 2, 2, 4, 1, 8)                                                        \
    X(1, 4, 2, 3, 2, 8)                                                        \
    X(2, 2, 2, 2, 2, 8)                                                        \
    X(3, 2, 4, 3, 2, 8)

namespace {

// ---------------------------------------------------------------------------
// Packing: operand -> centered doubles
// ---------------------------------------------------------------------------
// The thread's unit (row r, K columns 16*kc .. +15) becomes eight 16-byte
// words; 16 consecutive rows write 256 contiguous bytes per word.
__device__ __forceinline__ void pack_block(const SliceJob &J, int b, UnitTile &tile)
{
    uint32_t u[16];
    int r, kc;
    if (!load_unit(J, b, tile, u, r, kc)) return;
    const uint32_t half = (J.p - 1) / 2;
    double v[F64_BK];
#pragma unroll
    for (int e = 0; e < F64_BK; ++e)
        v[e] = (double)(J.in_mode == IN_SIGNED ? (int32_t)u[e] : center(u[e], J.p, half));
    static_assert(F64_BK == 16, "one unit is one K chunk of the packed layout");
    write_f64(J, (double *)J.D, v, r, kc);
}

// Both operands of one product in one launch: blocks [0, blocks_a) pack a,
// the rest b.
__global__ __launch_bounds__(UNIT_THREADS) void k_pack_f64_2(SliceJob a, SliceJob b, int blocks_a)
{
    __shared__ UnitTile tile;
    const int blk = blockIdx.x;
    if (blk < blocks_a)
        pack_block(a, blk, tile);
    else
        pack_block(b, blk - blocks_a, tile);
}

__global__ __launch_bounds__(UNIT_THREADS) void k_pack_f64_batched(
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
    pack_block(J, b - J.block_start, tile);
}

// ---------------------------------------------------------------------------
// GEMM on packed doubles
// ---------------------------------------------------------------------------
template <int WGM, int WGN, int NST>
struct F64Cfg {
    static constexpr int BM = 64 * WGM;
    static constexpr int BN = 64 * WGN;
    static constexpr int NW = WGM * WGN;
    static constexpr int A_BYTES = BM * F64_BK * 8;
    static constexpr int B_BYTES = BN * F64_BK * 8;
    static constexpr int STAGE = A_BYTES + B_BYTES;
    static constexpr int CHUNKS = STAGE / 1024; // 1 KB per wave load
    static constexpr int PER_WAVE = (CHUNKS + NW - 1) / NW;
    static constexpr int BYTES = NST * STAGE;
    static_assert(NST >= 2, "ring needs two slots");
    static_assert(BYTES <= LDS_LIMIT, "ring exceeds LDS");
};

template <class C>
__device__ __forceinline__ int issue_stage(const F64Job &J, int tm, int tn, int kt,
                                           char *lds_stage, int wave, int lane)
{
    const char *Abase = (const char *)(J.Ad + (int64_t)tm * C::BM * J.KP + (int64_t)kt * C::BM * F64_BK);
    const char *Bbase = (const char *)(J.Bd + (int64_t)tn * C::BN * J.KP + (int64_t)kt * C::BN * F64_BK);
    int issued = 0;
#pragma unroll
    for (int i = 0; i < C::PER_WAVE; ++i) {
        const int c = wave + i * C::NW;
        if (C::CHUNKS % C::NW == 0 || c < C::CHUNKS) {
            const int off = c * 1024;
            const char *src = off < C::A_BYTES ? Abase + off : Bbase + (off - C::A_BYTES);
            __builtin_amdgcn_global_load_lds((const void *)(src + lane * 16),
                                             (lds_ptr)(lds_stage + off), 16, 0, 0);
            ++issued;
        }
    }
    return issued;
}

__device__ __forceinline__ void fold(v4d (&acc)[4][4], double pd, double pinv)
{
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const double x = acc[i][j][r];
                acc[i][j][r] = __builtin_fma(-__builtin_rint(x * pinv), pd, x);
            }
}

// One output tile.  FINE: reduce after every 4-product matrix-core step
// (fewer than 16 products fit below 2^53), else every fold_stages stages.
// SPLIT: schedule for two waves per SIMD (see the loop).
template <int WGM, int WGN, int NST, bool SPLIT, bool FINE>
__device__ __forceinline__ void f64_tile(const F64Job &J, int tm, int tn, char *smem, int split)
{
    using C = F64Cfg<WGM, WGN, NST>;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm0 = (wave / WGN) * 64, wn0 = (wave % WGN) * 64;

    v4d acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};

    // K stages [k0, k1) of this tile (all of K unless the launch splits K)
    const int nkall = J.KP / F64_BK;
    const int k0 = J.kt_split ? split * J.kt_split : 0;
    const int k1 = J.kt_split && k0 + J.kt_split < nkall ? k0 + J.kt_split : nkall;
    const int nk = k1 - k0;
    int per_stage = 0;
#pragma unroll
    for (int st = 0; st < NST - 1; ++st)
        per_stage = issue_stage<C>(J, tm, tn, k0 + (st < nk ? st : nk - 1), smem + st * C::STAGE,
                                   wave, lane);

    // Fragment offsets inside a stage: in 16-row block b (2048 bytes), lane
    // l reads the 16-byte word of row l%16 holding K values 4(l/16) + 2h, +1.
    const int frag = (2 * (lane >> 4)) * 256 + (lane & 15) * 16;
    int since = 0;
    for (int kt = 0; kt < nk; ++kt) {
        // Stage kt has landed once at most the NST-2 later stages' loads of
        // this wave are outstanding; after the barrier every wave's part is
        // in LDS, and the slot of stage kt-1 is free for stage kt+NST-1.
        wait_vm((NST - 2) * per_stage);
        ring_barrier();
        const char *cur = smem + (kt % NST) * C::STAGE;
        v2d a[2][4], b[2][4];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
#pragma unroll
            for (int i = 0; i < 4; ++i)
                a[h][i] = *(const v2d *)(cur + ((wm0 >> 4) + i) * 2048 + frag + h * 256);
#pragma unroll
            for (int j = 0; j < 4; ++j)
                b[h][j] = *(const v2d *)(cur + C::A_BYTES + ((wn0 >> 4) + j) * 2048 + frag + h * 256);
        }
        const int nxt = kt + NST - 1;
        issue_stage<C>(J, tm, tn, k0 + (nxt < nk ? nxt : nk - 1), smem + (nxt % NST) * C::STAGE,
                       wave, lane);
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int s = 0; s < 2; ++s) {
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[h][i][s], b[h][j][s],
                                                                         acc[i][j], 0, 0, 0);
                if (FINE) fold(acc, J.pd, J.pinv);
            }
        if (!FINE) {
            // Schedule: the next stage's loads spread between the
            // matrix-core instructions.  With one wave per SIMD all fragment
            // reads go first; with two, the second half's reads wait for the
            // first half's matrix-core work (the other wave hides their
            // latency) so that fewer fragment registers are live.
            constexpr int NMF = 64, NLD = C::PER_WAVE;
            if (SPLIT) {
                constexpr int GAP = (NMF / 2) / (NLD + 1);
                __builtin_amdgcn_sched_group_barrier(0x100, 8, 0);
#pragma unroll
                for (int q = 0; q < NLD; ++q) {
                    __builtin_amdgcn_sched_group_barrier(0x008, GAP, 0);
                    __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);
                }
                __builtin_amdgcn_sched_group_barrier(0x008, NMF / 2 - NLD * GAP, 0);
                __builtin_amdgcn_sched_group_barrier(0x100, 8, 0);
                __builtin_amdgcn_sched_group_barrier(0x008, NMF / 2, 0);
            } else {
                constexpr int GAP = NMF / (NLD + 1);
                __builtin_amdgcn_sched_group_barrier(0x100, 16, 0);
#pragma unroll
                for (int q = 0; q < NLD; ++q) {
                    __builtin_amdgcn_sched_group_barrier(0x008, GAP, 0);
                    __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);
                }
                __builtin_amdgcn_sched_group_barrier(0x008, NMF - NLD * GAP, 0);
            }
            if (++since == J.fold_stages) {
                fold(acc, J.pd, J.pinv);
                since = 0;
            }
        }
    }
    // drain the (dummy) loads still in flight before the ring is left
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    // every wave is done with the ring before a persistent workgroup reuses it
    __syncthreads();

    // Epilogue: in each 16 x 16 block the lane holds column lane%16 of rows
    // lane/16 + 4r, r = 0..3 (v_mfma_f64_16x16x4 result layout).
    // C is read a block row (16 entries) at a time before that row's
    // stores, clamped into C so that no branch surrounds the loads: one
    // memory round trip per block row, not one per entry behind each store
    // (a load after a store to C cannot be moved above it).
    const int m0 = tm * C::BM, n0 = tn * C::BN;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        uint32_t cin[4][4];
        if (J.beta && !J.part) {
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int gr = m0 + wm0 + i * 16 + (lane >> 4) + 4 * r;
                    const int gc = n0 + wn0 + j * 16 + (lane & 15);
                    cin[j][r] = J.C[(int64_t)min(gr, J.m - 1) * J.ldc + min(gc, J.n - 1)];
                }
        }
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int gr = m0 + wm0 + i * 16 + (lane >> 4) + 4 * r;
                const int gc = n0 + wn0 + j * 16 + (lane & 15);
                if (gr < J.m && gc < J.n) {
                    const uint32_t v = canon_f64(acc[i][j][r], J.pd, J.pinv, J.p);
                    if (J.part) {
                        J.part[((int64_t)split * J.m + gr) * J.n + gc] = v;
                        continue;
                    }
                    uint32_t out = mulmod(J.alpha, v, J.p, J.pinv);
                    if (J.beta) out = addmod(out, mulmod(J.beta, cin[j][r], J.p, J.pinv), J.p);
                    J.C[(int64_t)gr * J.ldc + gc] = out;
                }
            }
    }
}

// FINE (reduction after every matrix-core step) is a separate instantiation
// chosen on the host: its extra live values would make the common kernel
// spill.
template <int WGM, int WGN, int NST, int WPE, bool FINE>
__global__ __attribute__((amdgpu_flat_work_group_size(64 * WGM * WGN, 64 * WGM * WGN),
                          amdgpu_waves_per_eu(WPE, WPE)))
void k_fgemm_f64(F64Job J)
{
    __shared__ __attribute__((aligned(1024))) char smem[F64Cfg<WGM, WGN, NST>::BYTES];
    const int G = J.tiles_m * J.tiles_n;
    const int split = (int)blockIdx.x / G; // 0 unless the launch splits K
    const int t = xcd_remap((int)blockIdx.x - split * G, G);
    int tm, tn;
    grouped_tile_rt(t, J.tiles_m, J.tiles_n, J.gm, &tm, &tn);
    f64_tile<WGM, WGN, NST, (WPE > 1), FINE>(J, tm, tn, smem, split);
}

// Every job of the table must have fold_stages == 0 iff FINE.
template <int WGM, int WGN, int NST, int WPE, bool FINE>
__global__ __attribute__((amdgpu_flat_work_group_size(64 * WGM * WGN, 64 * WGM * WGN),
                          amdgpu_waves_per_eu(WPE, WPE)))
void k_fgemm_f64_batched(const F64Job *__restrict__ jobs, int njobs, int total, int persistent,
                         unsigned *ctr)
{
    __shared__ __attribute__((aligned(1024))) char smem[F64Cfg<WGM, WGN, NST>::BYTES];
    __shared__ int s_tile;
    int g = persistent ? 0 : (int)blockIdx.x;
    for (;;) {
        if (persistent) {
            if (threadIdx.x == 0) s_tile = (int)atomicAdd(&ctr[0], 1u);
            __syncthreads();
            g = __builtin_amdgcn_readfirstlane(s_tile); // uniform: job fields stay scalar
            __syncthreads();
        }
        if (g >= total) break;
        int lo = 0, hi = njobs - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (jobs[mid].tile_start <= g) lo = mid; else hi = mid - 1;
        }
        const F64Job J = jobs[lo];
        int tm, tn;
        grouped_tile_rt(g - J.tile_start, J.tiles_m, J.tiles_n, J.gm, &tm, &tn);
        f64_tile<WGM, WGN, NST, (WPE > 1), FINE>(J, tm, tn, smem, 0);
        if (!persistent) break;
    }
    if (persistent && threadIdx.x == 0) {
        // The last workgroup out leaves the counters at zero for the next
        // launch (and for graph replays).
        __threadfence();
        const unsigned done = atomicAdd(&ctr[1], 1u);
        if (done == gridDim.x - 1) {
            atomicExch(&ctr[0], 0u);
            atomicExch(&ctr[1], 0u);
        }
    }
}

template <int WGM, int WGN, int NST, int WPE>
hipError_t run_single(const F64Job &J, hipStream_t st)
{
    const int nk = J.KP / F64_BK;
    const int splits = J.kt_split ? (nk + J.kt_split - 1) / J.kt_split : 1;
    const int G = J.tiles_m * J.tiles_n * splits;
    if (J.fold_stages > 0)
        hipLaunchKernelGGL((k_fgemm_f64<WGM, WGN, NST, WPE, false>), dim3(G),
                           dim3(64 * WGM * WGN), 0, st, J);
    else
        hipLaunchKernelGGL((k_fgemm_f64<WGM, WGN, NST, WPE, true>), dim3(G),
                           dim3(64 * WGM * WGN), 0, st, J);
    return hipGetLastError();
}

template <int WGM, int WGN, int NST, int WPE>
hipError_t run_batched(const F64Job *jobs, int njobs, int total, int persistent, unsigned *ctr,
                       int fine, hipStream_t st)
{
    int grid = total;
    if (persistent) {
        int dev = 0, cus = 256;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        // workgroups resident per CU: WPE waves on each of the 4 SIMDs
        const int per_cu = (4 * WPE) / (WGM * WGN) > 0 ? (4 * WPE) / (WGM * WGN) : 1;
        grid = cus * per_cu < total ? cus * per_cu : total;
        if (grid < 1) grid = 1;
    }
    if (fine)
        hipLaunchKernelGGL((k_fgemm_f64_batched<WGM, WGN, NST, WPE, true>), dim3(grid),
                           dim3(64 * WGM * WGN), 0, st, jobs, njobs, total, persistent, ctr);
    else
        hipLaunchKernelGGL((k_fgemm_f64_batched<WGM, WGN, NST, WPE, false>), dim3(grid),
                           dim3(64 * WGM * WGN), 0, st, jobs, njobs, total, persistent, ctr);
    return hipGetLastError();
}

const F64Tile kTiles[] = {
#define FF_ROW(id, WGM, WGN, NST, WPE, GM) {id, WGM, WGN, NST, WPE, GM},
    FF_F64_TILES(FF_ROW)
#undef FF_ROW
};

} // namespace

int f64_tile_count() { return (int)(sizeof(kTiles) / sizeof(kTiles[0])); }
const F64Tile &f64_tile(int id) { return kTiles[id]; }
int f64_default_tile() { return 1; }

hipError_t launch_f64(int tile, const F64Job &J, hipStream_t st)
{
    switch (tile) {
#define FF_CASE(id, WGM, WGN, NST, WPE, GM) \
    case id: return run_single<WGM, WGN, NST, WPE>(J, st);
        FF_F64_TILES(FF_CASE)
#undef FF_CASE
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_f64_batched(int tile, const F64Job *jobs, int njobs, int total, int persistent,
                              unsigned *ctr, int fine, hipStream_t st)
{
    switch (tile) {
#define FF_CASE(id, WGM, WGN, NST, WPE, GM) \
    case id: return run_batched<WGM, WGN, NST, WPE>(jobs, njobs, total, persistent, ctr, fine, st);
        FF_F64_TILES(FF_CASE)
#undef FF_CASE
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_pack_f64_2(const SliceJob &a, const SliceJob &b, hipStream_t st)
{
    const int na = unit_blocks(a), nb = unit_blocks(b);
    hipLaunchKernelGGL(k_pack_f64_2, dim3((unsigned)(na + nb)), dim3(UNIT_THREADS), 0, st, a, b,
                       na);
    return hipGetLastError();
}

hipError_t launch_pack_f64_batched(const SliceJob *dev_jobs, int njobs, int total_blocks,
                                   hipStream_t st)
{
    hipLaunchKernelGGL(k_pack_f64_batched, dim3(total_blocks), dim3(UNIT_THREADS), 0, st,
                       dev_jobs, njobs);
    return hipGetLastError();
}

int pack_blocks(const SliceJob &J) { return unit_blocks(J); }

} // namespace ff
