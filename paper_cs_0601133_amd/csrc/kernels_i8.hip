// INT8 matrix-core fgemm on signed digits.
//
// A centered residue c (|c| <= p/2) is written c = sum_{i<S} d_i R^i with
// R = 2^bits and digits d_i in [-R/2, R/2 - 1] (one direct int8 plane when
// c already fits int8).  Then
//     sum_l a_l b_l = sum_t R^t E_t,   E_t = sum_{i+j=t} sum_l a_{l,i} b_{l,j},
// and each E_t is an exact int32 sum of digit products as long as
// S * K * max|d_a| * max|d_b| < 2^31 (the int32 analogue of the accumulation
// bound of Section 2.1.2).  The digit products run on v_mfma_i32_32x32x32_i8;
// the epilogue reduces each E_t modulo p and forms
//     C <- sum_t (alpha R^t mod p) (E_t mod p) + beta C   (mod p).
//
// Digit planes (written by kernels_slice.hip) are packed: for a row tile of
// RT rows and the K range padded to KP, the 16-byte group (row r, k/16) of
// digit d sits at
//     d*plane + (r/RT)*RT*KP + (k/16)*RT*16 + (r%RT)*16,
// so the (RT x 64)-byte stage a workgroup needs is one contiguous block and
// is copied straight into LDS by global_load_lds_dwordx4 in the order the
// matrix-core operands are read back.
#include "ff_device.h"
#include "ff_internal.h"
#include "ff_ring.h"

namespace ff {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

namespace {

// ---------------------------------------------------------------------------
// GEMM on digit planes
// ---------------------------------------------------------------------------



// Geometry of one K stage (64 bytes of K) for SE digits per operand.
template <int SE, int TM, int TN, int WGM, int WGN, int KS>
struct Cfg {
    static constexpr int BM = WGM * 32 * TM;
    static constexpr int BN = WGN * 32 * TN;
    static constexpr int NT = 64 * WGM * WGN;
    static constexpr int NW = WGM * WGN;
    static constexpr int NSET = 2 * SE - 1;
    static constexpr int A_BYTES = SE * BM * KS;
    static constexpr int B_BYTES = SE * BN * KS;
    static constexpr int STAGE = A_BYTES + B_BYTES;
    static constexpr int CHUNKS = STAGE / 1024;           // 1 KB per wave load
    static constexpr int PER_WAVE = (CHUNKS + NW - 1) / NW; // loads per wave (max)
    static_assert(STAGE % 1024 == 0, "stage must be whole 1 KB chunks");
    static_assert((BM * KS) % 1024 == 0 && (BN * KS) % 1024 == 0, "digit blocks");
    static_assert(BM % 64 == 0 && BN % 64 == 0, "the slicer covers row tiles in blocks of 64");
    static constexpr int H = KS / 32; // 32-deep matrix-core steps per stage
};

// Stages in the LDS ring: as many as fit in the CU's LDS share of one of
// OCC resident workgroups (at most 6, at least 2); NST - 1 stages are in
// flight while one is consumed.
template <int S, int TM, int TN, int WGM, int WGN, int KS, int OCC>
struct Ring {
    static constexpr int STAGE = Cfg<S, TM, TN, WGM, WGN, KS>::STAGE;
    static constexpr int FIT = (LDS_LIMIT / OCC - (OCC > 1 ? 512 : 0)) / STAGE;
    static constexpr int NST = FIT > 6 ? 6 : (FIT < 2 ? 2 : FIT);
    static constexpr int BYTES = NST * STAGE;
};

// Issue the direct-to-LDS loads of stage kt; returns how many this wave
// issued.
template <class C>
__device__ __forceinline__ int issue_stage(const I8Job &J, int tm, int tn, int kt,
                                           char *lds_stage, int wave, int lane)
{
    constexpr int KS = C::H * 32;
    const char *Abase = (const char *)J.Ad + (int64_t)tm * C::BM * J.KP + (int64_t)kt * C::BM * KS;
    const char *Bbase = (const char *)J.Bd + (int64_t)tn * C::BN * J.KP + (int64_t)kt * C::BN * KS;
    constexpr int ABLK = C::BM * KS, BBLK = C::BN * KS;
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

__device__ __forceinline__ uint32_t mod_i32(int32_t e, uint32_t p, double pd, double pinv)
{
    const double x = (double)e;
    const double r = __builtin_fma(-__builtin_rint(x * pinv), pd, x);
    int64_t ri = (int64_t)r; // |ri| <= p/2 + 1
    ri += ri < 0 ? (int64_t)p : 0;
    ri += ri < 0 ? (int64_t)p : 0;
    ri -= ri >= (int64_t)p ? (int64_t)p : 0;
    return (uint32_t)ri;
}

// Matrix-core fragments of one K stage: lane l holds the 16-byte group (row
// l%32, K half l/32) of each digit block of its rows (a) and columns (b).
template <int SE, int TM, int TN, int H>
struct Frags {
    v4i a[H][SE][TM];
    v4i b[H][SE][TN];
};

template <class C, int SE, int TM, int TN>
__device__ __forceinline__ void read_frags(Frags<SE, TM, TN, C::H> &f, const char *cur, int wm0,
                                           int wn0, int lane)
{
    constexpr int KS = C::H * 32;
#pragma unroll
    for (int h = 0; h < C::H; ++h) {
        const int cidx = 2 * h + (lane >> 5);
#pragma unroll
        for (int d = 0; d < SE; ++d) {
#pragma unroll
            for (int i = 0; i < TM; ++i)
                f.a[h][d][i] = *(const v4i *)(cur + d * C::BM * KS +
                                              (cidx * C::BM + wm0 + 32 * i + (lane & 31)) * 16);
#pragma unroll
            for (int j = 0; j < TN; ++j)
                f.b[h][d][j] = *(const v4i *)(cur + C::A_BYTES + d * C::BN * KS +
                                              (cidx * C::BN + wn0 + 32 * j + (lane & 31)) * 16);
        }
    }
}

template <class C, int SE, int TM, int TN>
__device__ __forceinline__ void mfma_stage(v16i (&acc)[C::NSET][TM][TN],
                                           const Frags<SE, TM, TN, C::H> &f)
{
#pragma unroll
    for (int h = 0; h < C::H; ++h)
#pragma unroll
        for (int da = 0; da < SE; ++da)
#pragma unroll
            for (int db = 0; db < SE; ++db)
#pragma unroll
                for (int i = 0; i < TM; ++i)
#pragma unroll
                    for (int j = 0; j < TN; ++j)
                        acc[da + db][i][j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(
                            f.a[h][da][i], f.b[h][db][j], acc[da + db][i][j], 0, 0, 0);
}

// Schedule of one stage: the fragment reads first, then the stage loads
// spread between the matrix-core instructions so that no burst of memory
// instructions holds up the matrix core.
template <class C, int SE, int TM, int TN>
__device__ __forceinline__ void stage_schedule()
{
    constexpr int NDS = C::H * SE * (TM + TN);
    constexpr int NMF = C::H * SE * SE * TM * TN;
    constexpr int NLD = C::PER_WAVE;
    constexpr int GAP = NMF / (NLD + 1);
    __builtin_amdgcn_sched_group_barrier(0x100, NDS, 0);
#pragma unroll
    for (int q = 0; q < NLD; ++q) {
        __builtin_amdgcn_sched_group_barrier(0x008, GAP, 0);
        __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);
    }
    __builtin_amdgcn_sched_group_barrier(0x008, NMF - NLD * GAP, 0);
}

// One output tile with SE digits per operand; smem holds NST stages of the
// layout for SE digits (the ring is sized for the configuration's maximum).
// PIPE: the fragments of stage kt+1 are read while stage kt's matrix-core
// work runs (two fragment sets in registers), so the LDS reads that follow
// every barrier no longer stall the matrix core.
template <int SE, int TM, int TN, int WGM, int WGN, int KS, int NST, bool PIPE>
__device__ __forceinline__ void i8_tile(const I8Job &J, int tm, int tn, char *smem)
{
    using C = Cfg<SE, TM, TN, WGM, WGN, KS>;
    using F = Frags<SE, TM, TN, C::H>;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm0 = (wave / WGN) * 32 * TM, wn0 = (wave % WGN) * 32 * TN;

    v16i acc[C::NSET][TM][TN];
#pragma unroll
    for (int t = 0; t < C::NSET; ++t)
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j)
#pragma unroll
                for (int v = 0; v < 16; ++v) acc[t][i][j][v] = 0;

    const int nk = J.KP / KS;
    if constexpr (!PIPE) {
        // prologue: stages 0 .. NST-2 in flight (stage indices past the end
        // are clamped: those loads refill a free slot with data nobody reads)
        int per_stage = 0;
#pragma unroll
        for (int st = 0; st < NST - 1; ++st)
            per_stage = issue_stage<C>(J, tm, tn, st < nk ? st : nk - 1, smem + st * C::STAGE,
                                       wave, lane);
        for (int kt = 0; kt < nk; ++kt) {
            // Stage kt has landed once at most the NST-2 later stages' loads
            // of this wave are outstanding; after the barrier every wave's
            // part is in LDS, and the slot of stage kt-1 is free for stage
            // kt+NST-1.
            wait_vm((NST - 2) * per_stage);
            ring_barrier();
            F f;
            read_frags<C>(f, smem + (kt % NST) * C::STAGE, wm0, wn0, lane);
            const int nxt = kt + NST - 1;
            issue_stage<C>(J, tm, tn, nxt < nk ? nxt : nk - 1, smem + (nxt % NST) * C::STAGE,
                           wave, lane);
            mfma_stage<C>(acc, f);
            stage_schedule<C, SE, TM, TN>();
        }
    } else {
        // prologue: all NST slots in flight; stage 0's fragments in f0
        int per_stage = 0;
#pragma unroll
        for (int st = 0; st < NST; ++st)
            per_stage = issue_stage<C>(J, tm, tn, st < nk ? st : nk - 1, smem + st * C::STAGE,
                                       wave, lane);
        wait_vm((NST - 1) * per_stage);
        ring_barrier();
        F f0, f1;
        read_frags<C>(f0, smem, wm0, wn0, lane);
        // One step: stage kt's matrix-core work on cur while stage kt+1's
        // fragments are read into nxt.  Before the barrier each wave has
        // its earlier fragment reads back (lgkmcnt(0)) and its loads of
        // stage kt+1 landed (stages up to kt+NST-1 were issued, at most
        // NST-2 later ones may still be in flight); after it, the slot of
        // stage kt (its fragments are in registers on every wave) takes
        // stage kt+NST.  On the last step the read of "stage kt+1" hits a
        // slot that holds a clamped copy nobody uses.
        auto step = [&](int kt, F &cur, F &nxt) {
            asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
            wait_vm((NST - 2) * per_stage);
            ring_barrier();
            const int nst = kt + NST;
            issue_stage<C>(J, tm, tn, nst < nk ? nst : nk - 1, smem + (kt % NST) * C::STAGE,
                           wave, lane);
            read_frags<C>(nxt, smem + ((kt + 1) % NST) * C::STAGE, wm0, wn0, lane);
            mfma_stage<C>(acc, cur);
            stage_schedule<C, SE, TM, TN>();
        };
        int kt = 0;
        for (; kt + 1 < nk; kt += 2) {
            step(kt, f0, f1);
            step(kt + 1, f1, f0);
        }
        if (kt < nk) step(kt, f0, f1);
    }
    // drain the (dummy) loads still in flight before the ring is left
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    // every wave is done with the ring before a persistent workgroup reuses it
    __syncthreads();

    // Epilogue.  32 x 32 accumulator layout: lane holds column lane%32 and
    // rows 8*(v/4) + 4*(lane/32) + v%4, v = 0..15.  With epi_direct the
    // digit sums are recombined in one exact binary64 sum with centered
    // weights; with fp_epi each E_t is first reduced (centered) in binary64;
    // otherwise 64-bit integers with a reduction per term.
    //
    // The entries of C of each 32 x 32 block are requested together before
    // its recombination: a load placed after a store to C cannot be moved
    // above it (the addresses may alias for all the compiler knows), so
    // reading each entry next to its store would wait out one memory round
    // trip per entry; requested together, their latency overlaps the
    // recombination (one round trip per block, 16 registers).
    const int m0 = tm * C::BM, n0 = tn * C::BN;
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) {
            uint32_t cin[16];
            if (J.beta) {
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    const int row = m0 + wm0 + 32 * i + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
                    const int col = n0 + wn0 + 32 * j + (lane & 31);
                    // clamped into C: no branch around the load (an entry
                    // outside C is read from the edge and never used)
                    cin[v] = J.C[(int64_t)min(row, J.m - 1) * J.ldc + min(col, J.n - 1)];
                }
            }
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int row = m0 + wm0 + 32 * i + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
                const int col = n0 + wn0 + 32 * j + (lane & 31);
                if (row < J.m && col < J.n) {
                    uint32_t r;
                    if (J.epi_direct) {
                        double sum = 0.0;
#pragma unroll
                        for (int t = 0; t < C::NSET; ++t)
                            sum = __builtin_fma(J.wc[t], (double)acc[t][i][j][v], sum);
                        r = canon_f64(sum, J.pd, J.pinv, J.p);
                    } else if (J.fp_epi) {
                        double sum = 0.0;
#pragma unroll
                        for (int t = 0; t < C::NSET; ++t) {
                            const double x = (double)acc[t][i][j][v];
                            const double e = __builtin_fma(-__builtin_rint(x * J.pinv), J.pd, x);
                            sum = __builtin_fma(J.wc[t], e, sum);
                        }
                        r = canon_f64(sum, J.pd, J.pinv, J.p);
                    } else {
                        r = 0;
#pragma unroll
                        for (int t = 0; t < C::NSET; ++t)
                            r = addmod(r, mulmod(J.w[t], mod_i32(acc[t][i][j][v], J.p, J.pd, J.pinv),
                                                 J.p, J.pinv), J.p);
                    }
                    if (J.beta) r = addmod(r, mulmod(J.beta, cin[v], J.p, J.pinv), J.p);
                    J.C[(int64_t)row * J.ldc + col] = r;
                }
            }
        }
}

// Waves per SIMD implied by the workgroup size and the number of resident
// workgroups per CU.
template <int WGM, int WGN, int OCC>
struct Wpe {
    static constexpr int v = (WGM * WGN * OCC) / 4 > 0 ? (WGM * WGN * OCC) / 4 : 1;
};

template <int S, int TM, int TN, int WGM, int WGN, int KS, bool PIPE, int OCC>
__global__ __attribute__((amdgpu_flat_work_group_size(64 * WGM * WGN, 64 * WGM * WGN),
                          amdgpu_waves_per_eu(Wpe<WGM, WGN, OCC>::v, Wpe<WGM, WGN, OCC>::v)))
void k_fgemm_i8(I8Job J)
{
    using R = Ring<S, TM, TN, WGM, WGN, KS, OCC>;
    __shared__ __attribute__((aligned(1024))) char smem[R::BYTES];
    const int G = J.tiles_m * J.tiles_n;
    const int t = xcd_remap(blockIdx.x, G);
    int tm, tn;
    grouped_tile_rt(t, J.tiles_m, J.tiles_n, J.gm, &tm, &tn);
    i8_tile<S, TM, TN, WGM, WGN, KS, R::NST, PIPE>(J, tm, tn, smem);
}

// Batched: a job may use fewer digits than the configuration's S; the tile
// body is specialised per digit count so that no matrix-core instruction is
// predicated.
template <int S, int TM, int TN, int WGM, int WGN, int KS, int NST, bool PIPE>
__device__ __forceinline__ void i8_tile_any(const I8Job &J, int tm, int tn, char *smem)
{
    if constexpr (S >= 1) {
        if (J.s == S) {
            i8_tile<S, TM, TN, WGM, WGN, KS, NST, PIPE>(J, tm, tn, smem);
            return;
        }
    }
    if constexpr (S > 1) i8_tile_any<S - 1, TM, TN, WGM, WGN, KS, NST, PIPE>(J, tm, tn, smem);
}

// UNI: every job has S digits; only the S-digit tile body is compiled.
template <int S, int TM, int TN, int WGM, int WGN, int KS, bool PIPE, int OCC, bool UNI>
__global__ __attribute__((amdgpu_flat_work_group_size(64 * WGM * WGN, 64 * WGM * WGN),
                          amdgpu_waves_per_eu(Wpe<WGM, WGN, OCC>::v, Wpe<WGM, WGN, OCC>::v)))
void k_fgemm_i8_batched(const I8Job *__restrict__ jobs, int njobs, int total,
                        int persistent, unsigned *ctr)
{
    using R = Ring<S, TM, TN, WGM, WGN, KS, OCC>;
    __shared__ __attribute__((aligned(1024))) char smem[R::BYTES];
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
        const I8Job J = jobs[lo];
        int tm, tn;
        grouped_tile_rt(g - J.tile_start, J.tiles_m, J.tiles_n, J.gm, &tm, &tn);
        if constexpr (UNI)
            i8_tile<S, TM, TN, WGM, WGN, KS, R::NST, PIPE>(J, tm, tn, smem);
        else
            i8_tile_any<S, TM, TN, WGM, WGN, KS, R::NST, PIPE>(J, tm, tn, smem);
        if (!persistent) break;
    }
    if (persistent && threadIdx.x == 0) {
        __threadfence();
        const unsigned done = atomicAdd(&ctr[1], 1u);
        if (done == gridDim.x - 1) {
            atomicExch(&ctr[0], 0u);
            atomicExch(&ctr[1], 0u);
        }
    }
}

// A job table whose jobs all have S digits (the symmetric product's block
// rows): one workgroup per tile, tiles renumbered so that neighbours in a
// job's tile order share an XCD, and only the S-digit tile body compiled
// (the general table kernel's dispatch over digit counts costs registers).
template <int S, int TM, int TN, int WGM, int WGN, int KS, bool PIPE, int OCC>
__global__ __attribute__((amdgpu_flat_work_group_size(64 * WGM * WGN, 64 * WGM * WGN),
                          amdgpu_waves_per_eu(Wpe<WGM, WGN, OCC>::v, Wpe<WGM, WGN, OCC>::v)))
void k_fgemm_i8_jobs(const I8Job *__restrict__ jobs, int njobs, int total)
{
    using R = Ring<S, TM, TN, WGM, WGN, KS, OCC>;
    __shared__ __attribute__((aligned(1024))) char smem[R::BYTES];
    const int g = xcd_remap((int)blockIdx.x, total);
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].tile_start <= g) lo = mid; else hi = mid - 1;
    }
    const I8Job J = jobs[lo];
    int tm, tn;
    grouped_tile_rt(g - J.tile_start, J.tiles_m, J.tiles_n, J.gm, &tm, &tn);
    i8_tile<S, TM, TN, WGM, WGN, KS, R::NST, PIPE>(J, tm, tn, smem);
}

template <int S, int TM, int TN, int WGM, int WGN, int KS, bool PIPE, int OCC>
hipError_t run_jobs(const I8Job *jobs, int njobs, int total, hipStream_t st)
{
    hipLaunchKernelGGL((k_fgemm_i8_jobs<S, TM, TN, WGM, WGN, KS, PIPE, OCC>), dim3(total),
                       dim3(64 * WGM * WGN), 0, st, jobs, njobs, total);
    return hipGetLastError();
}

template <int S, int TM, int TN, int WGM, int WGN, int KS, bool PIPE, int OCC>
hipError_t run_single(const I8Job &J, hipStream_t st)
{
    const int G = J.tiles_m * J.tiles_n;
    hipLaunchKernelGGL((k_fgemm_i8<S, TM, TN, WGM, WGN, KS, PIPE, OCC>), dim3(G),
                       dim3(64 * WGM * WGN), 0, st, J);
    return hipGetLastError();
}

template <int S, int TM, int TN, int WGM, int WGN, int KS, bool PIPE, int OCC>
hipError_t run_batched(const I8Job *jobs, int njobs, int total, int persistent,
                       unsigned *ctr, hipStream_t st, bool uniform)
{
    int grid = total;
    if (persistent) {
        int dev = 0, cus = 256;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        cus *= OCC; // resident workgroups
        grid = cus < total ? cus : total;
        if (grid < 1) grid = 1;
    }
    if (uniform)
        hipLaunchKernelGGL((k_fgemm_i8_batched<S, TM, TN, WGM, WGN, KS, PIPE, OCC, true>),
                           dim3(grid), dim3(64 * WGM * WGN), 0, st, jobs, njobs, total,
                           persistent, ctr);
    else
        hipLaunchKernelGGL((k_fgemm_i8_batched<S, TM, TN, WGM, WGN, KS, PIPE, OCC, false>),
                           dim3(grid), dim3(64 * WGM * WGN), 0, st, jobs, njobs, total,
                           persistent, ctr);
    return hipGetLastError();
}

} // namespace

// Compiled configurations: id, S, TM, TN, WGM, WGN, KS, GM, PIPE, OCC.  Each
// (WGM x WGN) workgroup of 64-lane waves owns a (WGM*32*TM) x (WGN*32*TN)
// tile of C; 2S-1 accumulator sets of TM*TN 32x32 blocks live in each wave;
// KS bytes of K per LDS stage; GM tile rows per group of the tile order;
// PIPE: fragment reads of the next stage overlap the current stage; OCC
// workgroups share a CU (their phases drift apart, so one workgroup's
// epilogue and stage barriers overlap the other's matrix-core work).
#define FF_I8_TILES(X)                                                            \
    X(0, 1, 2, 2, 2, 2, 64, 8, 0, 1)  /* 128 x 128, 4 waves,   64 acc */             \
    X(1, 1, 2, 2, 4, 2, 64, 8, 0, 1)  /* 256 x 128, 8 waves,   64 acc */             \
    X(2, 1, 2, 2, 4, 2, 32, 8, 0, 1)  /* 256 x 128, 8 waves, half stages */          \
    X(3, 2, 1, 2, 4, 2, 32, 8, 0, 1)  /* 128 x 128, 8 waves,   96 acc, half stages */\
    X(4, 2, 1, 2, 4, 2, 64, 8, 0, 1)  /* 128 x 128, 8 waves,   96 acc */             \
    X(5, 3, 1, 2, 4, 2, 32, 8, 0, 1)  /* 128 x 128, 8 waves,  160 acc, half stages */\
    X(6, 3, 1, 2, 4, 2, 64, 8, 0, 1)  /* 128 x 128, 8 waves,  160 acc */             \
    X(7, 3, 1, 1, 4, 2, 64, 8, 0, 1)  /* 128 x  64, 8 waves,   80 acc */             \
    X(8, 4, 1, 1, 4, 2, 64, 8, 0, 1)  /* 128 x  64, 8 waves,  112 acc */             \
    X(9, 4, 1, 1, 4, 2, 64, 4, 0, 1)  /* 128 x  64, 8 waves,  groups of 4 */         \
    X(10, 4, 1, 1, 2, 4, 64, 8, 0, 1) /*  64 x 128, 8 waves,  112 acc */             \
    X(11, 4, 1, 1, 4, 2, 32, 4, 0, 1) /* 128 x  64, half stages, groups of 4 */      \
    X(12, 5, 1, 1, 4, 2, 64, 8, 0, 1) /* 128 x  64, 8 waves,  144 acc */             \
    X(13, 4, 1, 1, 4, 2, 32, 8, 0, 1) /* 128 x  64, half stages */                   \
    X(14, 4, 1, 1, 4, 2, 32, 8, 1, 1) /* 128 x  64, half stages, pipelined */        \
    X(15, 4, 1, 1, 4, 2, 64, 8, 1, 1) /* 128 x  64, pipelined */                     \
    X(16, 3, 1, 2, 4, 2, 32, 8, 1, 1) /* 128 x 128, half stages, pipelined */        \
    X(17, 1, 2, 2, 4, 2, 32, 8, 1, 1) /* 256 x 128, half stages, pipelined */        \
    X(18, 2, 1, 2, 4, 2, 32, 8, 1, 1) /* 128 x 128, half stages, pipelined */        \
    X(19, 1, 2, 4, 4, 2, 64, 8, 0, 1) /* 256 x 256, 8 waves,  128 acc */             \
    X(20, 1, 2, 2, 2, 2, 64, 4, 1, 2) /* 128 x 128, 4 waves, 2 per CU, pipelined */  \
    X(21, 1, 4, 2, 2, 4, 64, 4, 1, 1) /* 256 x 256, 8 waves, 128 acc, pipelined */

namespace {
const I8Tile k_tiles[] = {
#define FF_ROW(id, S, TM, TN, WGM, WGN, KS, GM, PIPE, OCC) \
    I8Tile{id, S, TM, TN, WGM, WGN, KS, GM, PIPE, OCC},
    FF_I8_TILES(FF_ROW)
#undef FF_ROW
};
// Default configuration per slice count (index = S).
const int k_default[6] = {-1, 20, 4, 6, 15, 12};
} // namespace

int i8_tile_count() { return (int)(sizeof(k_tiles) / sizeof(k_tiles[0])); }
const I8Tile &i8_tile(int id) { return k_tiles[id]; }
int i8_default_tile(int S) { return (S >= 1 && S <= 5) ? k_default[S] : -1; }

hipError_t launch_i8(int tile, const I8Job &J, hipStream_t st)
{
    switch (tile) {
#define FF_CASE(id, S, TM, TN, WGM, WGN, KS, GM, PIPE, OCC)                         \
    case id: return run_single<S, TM, TN, WGM, WGN, KS, PIPE, OCC>(J, st);
        FF_I8_TILES(FF_CASE)
#undef FF_CASE
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_i8_jobs(int tile, const I8Job *jobs, int njobs, int total, hipStream_t st)
{
    if (total <= 0) return hipSuccess;
    switch (tile) {
#define FF_CASE(id, S, TM, TN, WGM, WGN, KS, GM, PIPE, OCC)                         \
    case id: return run_jobs<S, TM, TN, WGM, WGN, KS, PIPE, OCC>(jobs, njobs, total, st);
        FF_I8_TILES(FF_CASE)
#undef FF_CASE
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_i8_batched(int tile, const I8Job *jobs, int njobs, int total,
                             int persistent, unsigned *ctr, hipStream_t st, bool uniform_s)
{
    switch (tile) {
#define FF_CASE(id, S, TM, TN, WGM, WGN, KS, GM, PIPE, OCC)                         \
    case id:                                                                          \
        return run_batched<S, TM, TN, WGM, WGN, KS, PIPE, OCC>(jobs, njobs, total, persistent, ctr, \
                                                              st, uniform_s);
        FF_I8_TILES(FF_CASE)
#undef FF_CASE
    default: return hipErrorInvalidValue;
    }
}


} // namespace ff
