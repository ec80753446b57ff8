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
// Digit planes are stored "packed": for a row tile of RT rows and the K
// range padded to KP, the 16-byte group (row r, k/16) of digit d sits at
//     d*plane + (r/RT)*RT*KP + (k/16)*RT*16 + (r%RT)*16,
// so the (RT x 64)-byte stage a workgroup needs is one contiguous block and
// is copied straight into LDS by global_load_lds_dwordx4 in the order the
// matrix-core operands are read back.
#include "ff_device.h"
#include "ff_internal.h"

namespace ff {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));
typedef __attribute__((address_space(3))) void *lds_ptr;

namespace {

// ---------------------------------------------------------------------------
// Slicer: operand -> packed digit planes (zero padded)
// ---------------------------------------------------------------------------
constexpr int SLICE_THREADS = 256;

__device__ __forceinline__ void slice_one(const SliceJob &J, int64_t q)
{
    const int nchunk = J.KP / 16;
    if (q >= (int64_t)J.rows_pad * nchunk) return;
    const int r = (int)(q % J.rows_pad);
    const int kc = (int)(q / J.rows_pad);
    const int k0 = kc * 16;
    const uint32_t half = (J.p - 1) / 2;

    int32_t v[16];
    const bool row_ok = r < J.rows;
    if (!J.trans) {
        const uint32_t *src = (const uint32_t *)J.X + (int64_t)r * J.ldx + k0;
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const bool ok = row_ok && (k0 + e) < J.K;
            const uint32_t u = ok ? src[e] : 0u;
            v[e] = !ok ? 0 : (J.in_mode == IN_SIGNED ? (int32_t)u : center(u, J.p, half));
        }
    } else {
        const uint32_t *src = (const uint32_t *)J.X + (int64_t)k0 * J.ldx + r;
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const bool ok = row_ok && (k0 + e) < J.K;
            const uint32_t u = ok ? src[(int64_t)e * J.ldx] : 0u;
            v[e] = !ok ? 0 : (J.in_mode == IN_SIGNED ? (int32_t)u : center(u, J.p, half));
        }
    }

    const int bits = J.S == 1 ? 8 : J.bits;
    const int Rh = 1 << (bits - 1), mask = (1 << bits) - 1;
    int8_t *dst = J.D + (int64_t)(r / J.RT) * J.RT * J.KP + (int64_t)kc * J.RT * 16 +
                  (int64_t)(r % J.RT) * 16;
    for (int d = 0; d < J.S; ++d) {
        uint32_t w[4] = {0, 0, 0, 0};
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int dig = ((v[e] + Rh) & mask) - Rh; // balanced digit
            v[e] = (v[e] - dig) >> bits;                // exact division by R
            w[e >> 2] |= (uint32_t)(dig & 0xFF) << (8 * (e & 3));
        }
        *(uint4 *)(dst + (int64_t)d * J.plane) = make_uint4(w[0], w[1], w[2], w[3]);
    }
}

__global__ __launch_bounds__(SLICE_THREADS) void k_slice(SliceJob J)
{
    slice_one(J, (int64_t)blockIdx.x * SLICE_THREADS + threadIdx.x);
}

__global__ __launch_bounds__(SLICE_THREADS) void k_slice_batched(
    const SliceJob *__restrict__ jobs, int njobs)
{
    int lo = 0, hi = njobs - 1;
    const int b = blockIdx.x;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].block_start <= b) lo = mid; else hi = mid - 1;
    }
    const SliceJob J = jobs[lo];
    slice_one(J, (int64_t)(b - J.block_start) * SLICE_THREADS + threadIdx.x);
}

// ---------------------------------------------------------------------------
// GEMM on digit planes
// ---------------------------------------------------------------------------
template <int S, int TM, int TN, int WGM, int WGN>
struct Cfg {
    static constexpr int BM = WGM * 32 * TM;
    static constexpr int BN = WGN * 32 * TN;
    static constexpr int NT = 64 * WGM * WGN;
    static constexpr int NW = WGM * WGN;
    static constexpr int NSET = 2 * S - 1;
    static constexpr int A_BYTES = S * BM * I8_BK; // one stage, all digits
    static constexpr int B_BYTES = S * BN * I8_BK;
    static constexpr int STAGE = A_BYTES + B_BYTES;
    static constexpr int CHUNKS = STAGE / 1024; // 1 KB per wave load
    static_assert(STAGE % 1024 == 0, "stage must be whole 1 KB chunks");
    static_assert((BM * I8_BK) % 1024 == 0 && (BN * I8_BK) % 1024 == 0, "digit blocks");
};

// Issue the direct-to-LDS loads of stage kt.
template <class C>
__device__ __forceinline__ void issue_stage(const I8Job &J, int tm, int tn,
                                            int kt, int s, char *lds_stage,
                                            int wave, int lane)
{
    const char *Abase = (const char *)J.Ad + (int64_t)tm * C::BM * J.KP + (int64_t)kt * C::BM * I8_BK;
    const char *Bbase = (const char *)J.Bd + (int64_t)tn * C::BN * J.KP + (int64_t)kt * C::BN * I8_BK;
    constexpr int ABLK = C::BM * I8_BK, BBLK = C::BN * I8_BK;
    for (int c = wave; c < C::CHUNKS; c += C::NW) {
        const int off = c * 1024;
        const char *src;
        int d;
        if (off < C::A_BYTES) {
            d = off / ABLK;
            src = Abase + (int64_t)d * J.a_plane + (off - d * ABLK);
        } else {
            const int o = off - C::A_BYTES;
            d = o / BBLK;
            src = Bbase + (int64_t)d * J.b_plane + (o - d * BBLK);
        }
        if (d < s)
            __builtin_amdgcn_global_load_lds((const void *)(src + lane * 16),
                                             (lds_ptr)(lds_stage + off), 16, 0, 0);
    }
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

template <int S, int TM, int TN, int WGM, int WGN>
__device__ void i8_tile(const I8Job &J, int tm, int tn, char *smem)
{
    using C = Cfg<S, TM, TN, WGM, WGN>;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm0 = (wave / WGN) * 32 * TM, wn0 = (wave % WGN) * 32 * TN;
    const int s = J.s;

    v16i acc[C::NSET][TM][TN];
#pragma unroll
    for (int t = 0; t < C::NSET; ++t)
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j)
#pragma unroll
                for (int v = 0; v < 16; ++v) acc[t][i][j][v] = 0;

    const int nk = J.KP / I8_BK;
    issue_stage<C>(J, tm, tn, 0, s, smem, wave, lane);

    for (int kt = 0; kt < nk; ++kt) {
        char *cur = smem + (kt & 1) * C::STAGE;
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();
        if (kt + 1 < nk)
            issue_stage<C>(J, tm, tn, kt + 1, s, smem + ((kt + 1) & 1) * C::STAGE, wave, lane);
#pragma unroll
        for (int h = 0; h < I8_BK / 32; ++h) {
            const int cidx = 2 * h + (lane >> 5);
            v4i a[S][TM], b[S][TN];
#pragma unroll
            for (int d = 0; d < S; ++d) {
                if (d < s) {
#pragma unroll
                    for (int i = 0; i < TM; ++i)
                        a[d][i] = *(const v4i *)(cur + d * C::BM * I8_BK +
                                                 (cidx * C::BM + wm0 + 32 * i + (lane & 31)) * 16);
#pragma unroll
                    for (int j = 0; j < TN; ++j)
                        b[d][j] = *(const v4i *)(cur + C::A_BYTES + d * C::BN * I8_BK +
                                                 (cidx * C::BN + wn0 + 32 * j + (lane & 31)) * 16);
                }
            }
#pragma unroll
            for (int da = 0; da < S; ++da)
#pragma unroll
                for (int db = 0; db < S; ++db) {
                    if (da < s && db < s) {
#pragma unroll
                        for (int i = 0; i < TM; ++i)
#pragma unroll
                            for (int j = 0; j < TN; ++j)
                                acc[da + db][i][j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(
                                    a[da][i], b[db][j], acc[da + db][i][j], 0, 0, 0);
                    }
                }
        }
    }
    // Every wave must be done with the last stage before smem is reused by
    // the next tile of a persistent workgroup.
    __syncthreads();

    // Epilogue.  32 x 32 accumulator layout: lane holds column lane%32 and
    // rows 8*(v/4) + 4*(lane/32) + v%4, v = 0..15.
    const int m0 = tm * C::BM, n0 = tn * C::BN;
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int row = m0 + wm0 + 32 * i + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
                const int col = n0 + wn0 + 32 * j + (lane & 31);
                if (row < J.m && col < J.n) {
                    uint32_t r = 0;
#pragma unroll
                    for (int t = 0; t < C::NSET; ++t)
                        if (t < 2 * s - 1)
                            r = addmod(r, mulmod(J.w[t], mod_i32(acc[t][i][j][v], J.p, J.pd, J.pinv),
                                                 J.p, J.pinv), J.p);
                    uint32_t *cp = J.C + (int64_t)row * J.ldc + col;
                    if (J.beta) r = addmod(r, mulmod(J.beta, *cp, J.p, J.pinv), J.p);
                    *cp = r;
                }
            }
}

// Waves per SIMD implied by the workgroup size (one workgroup per CU).
template <int WGM, int WGN>
struct Wpe {
    static constexpr int v = (WGM * WGN) / 4 > 0 ? (WGM * WGN) / 4 : 1;
};

template <int S, int TM, int TN, int WGM, int WGN>
__global__ __attribute__((amdgpu_flat_work_group_size(64 * WGM * WGN, 64 * WGM * WGN),
                          amdgpu_waves_per_eu(Wpe<WGM, WGN>::v, Wpe<WGM, WGN>::v)))
void k_fgemm_i8(I8Job J)
{
    using C = Cfg<S, TM, TN, WGM, WGN>;
    __shared__ __attribute__((aligned(1024))) char smem[2 * C::STAGE];
    const int G = J.tiles_m * J.tiles_n;
    const int t = xcd_remap(blockIdx.x, G);
    int tm, tn;
    grouped_tile<8>(t, J.tiles_m, J.tiles_n, &tm, &tn);
    i8_tile<S, TM, TN, WGM, WGN>(J, tm, tn, smem);
}

template <int S, int TM, int TN, int WGM, int WGN>
__global__ __attribute__((amdgpu_flat_work_group_size(64 * WGM * WGN, 64 * WGM * WGN),
                          amdgpu_waves_per_eu(Wpe<WGM, WGN>::v, Wpe<WGM, WGN>::v)))
void k_fgemm_i8_batched(const I8Job *__restrict__ jobs, int njobs, int total,
                        int persistent, unsigned *ctr)
{
    using C = Cfg<S, TM, TN, WGM, WGN>;
    __shared__ __attribute__((aligned(1024))) char smem[2 * C::STAGE];
    __shared__ int s_tile;
    int g = persistent ? 0 : (int)blockIdx.x;
    for (;;) {
        if (persistent) {
            if (threadIdx.x == 0) s_tile = (int)atomicAdd(&ctr[0], 1u);
            __syncthreads();
            g = s_tile;
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
        grouped_tile<8>(g - J.tile_start, J.tiles_m, J.tiles_n, &tm, &tn);
        i8_tile<S, TM, TN, WGM, WGN>(J, tm, tn, smem);
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

template <int S, int TM, int TN, int WGM, int WGN>
hipError_t run_single(const I8Job &J, hipStream_t st)
{
    const int G = J.tiles_m * J.tiles_n;
    hipLaunchKernelGGL((k_fgemm_i8<S, TM, TN, WGM, WGN>), dim3(G), dim3(64 * WGM * WGN),
                       0, st, J);
    return hipGetLastError();
}

template <int S, int TM, int TN, int WGM, int WGN>
hipError_t run_batched(const I8Job *jobs, int njobs, int total, int persistent,
                       unsigned *ctr, hipStream_t st)
{
    int grid = total;
    if (persistent) {
        int dev = 0, cus = 256;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        grid = cus < total ? cus : total;
        if (grid < 1) grid = 1;
    }
    hipLaunchKernelGGL((k_fgemm_i8_batched<S, TM, TN, WGM, WGN>), dim3(grid),
                       dim3(64 * WGM * WGN), 0, st, jobs, njobs, total, persistent, ctr);
    return hipGetLastError();
}

} // namespace

// Compiled configurations: id, S, TM, TN, WGM, WGN.  Each (WGM x WGN)
// workgroup of 64-lane waves owns a (WGM*32*TM) x (WGN*32*TN) tile of C;
// 2S-1 accumulator sets of TM*TN 32x32 blocks live in each wave.
#define FF_I8_TILES(X)                                                            \
    X(0, 1, 2, 2, 2, 2)  /* 128 x 128, 4 waves,   64 acc */                        \
    X(1, 1, 2, 2, 4, 2)  /* 256 x 128, 8 waves,   64 acc */                        \
    X(2, 1, 2, 4, 2, 2)  /* 128 x 256, 4 waves,  128 acc */                        \
    X(3, 2, 2, 2, 2, 2)  /* 128 x 128, 4 waves,  192 acc */                        \
    X(4, 2, 1, 2, 4, 2)  /* 128 x 128, 8 waves,   96 acc */                        \
    X(5, 3, 1, 2, 4, 1)  /* 128 x  64, 4 waves,  160 acc */                        \
    X(6, 3, 1, 2, 4, 2)  /* 128 x 128, 8 waves,  160 acc */                        \
    X(7, 3, 1, 1, 4, 2)  /* 128 x  64, 8 waves,   80 acc */                        \
    X(8, 4, 1, 1, 4, 2)  /* 128 x  64, 8 waves,  112 acc */                        \
    X(9, 4, 1, 1, 2, 2)  /*  64 x  64, 4 waves,  112 acc */                        \
    X(10, 4, 1, 1, 2, 4) /*  64 x 128, 8 waves,  112 acc */                        \
    X(11, 5, 1, 1, 4, 1) /* 128 x  32, 4 waves,  144 acc */                        \
    X(12, 5, 1, 1, 4, 2) /* 128 x  64, 8 waves,  144 acc */

namespace {
const I8Tile k_tiles[] = {
#define FF_ROW(id, S, TM, TN, WGM, WGN) I8Tile{id, S, TM, TN, WGM, WGN},
    FF_I8_TILES(FF_ROW)
#undef FF_ROW
};
// Default configuration per slice count (index = S).
const int k_default[6] = {-1, 0, 4, 6, 8, 12};
} // namespace

int i8_tile_count() { return (int)(sizeof(k_tiles) / sizeof(k_tiles[0])); }
const I8Tile &i8_tile(int id) { return k_tiles[id]; }
int i8_default_tile(int S) { return (S >= 1 && S <= 5) ? k_default[S] : -1; }

hipError_t launch_i8(int tile, const I8Job &J, hipStream_t st)
{
    switch (tile) {
#define FF_CASE(id, S, TM, TN, WGM, WGN)                                            \
    case id: return run_single<S, TM, TN, WGM, WGN>(J, st);
        FF_I8_TILES(FF_CASE)
#undef FF_CASE
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_i8_batched(int tile, const I8Job *jobs, int njobs, int total,
                             int persistent, unsigned *ctr, hipStream_t st)
{
    switch (tile) {
#define FF_CASE(id, S, TM, TN, WGM, WGN)                                            \
    case id: return run_batched<S, TM, TN, WGM, WGN>(jobs, njobs, total, persistent, ctr, st);
        FF_I8_TILES(FF_CASE)
#undef FF_CASE
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_slice(const SliceJob &J, hipStream_t st)
{
    const int64_t total = (int64_t)J.rows_pad * (J.KP / 16);
    const int64_t grid = (total + SLICE_THREADS - 1) / SLICE_THREADS;
    hipLaunchKernelGGL(k_slice, dim3((unsigned)grid), dim3(SLICE_THREADS), 0, st, J);
    return hipGetLastError();
}

hipError_t launch_slice_batched(const SliceJob *dev_jobs, int njobs,
                                int total_blocks, hipStream_t st)
{
    hipLaunchKernelGGL(k_slice_batched, dim3(total_blocks), dim3(SLICE_THREADS), 0, st,
                       dev_jobs, njobs);
    return hipGetLastError();
}

int slice_blocks(const SliceJob &J)
{
    const int64_t total = (int64_t)J.rows_pad * (J.KP / 16);
    return (int)((total + SLICE_THREADS - 1) / SLICE_THREADS);
}

} // namespace ff
