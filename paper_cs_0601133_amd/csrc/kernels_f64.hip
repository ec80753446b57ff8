// FP64 matrix-core fgemm: the "Zpz-double" design of Sections 2.1.2 and 3.1
// (residues held as integer-valued doubles, products summed exactly by the
// floating-point unit, reduction delayed) on gfx950's v_mfma_f64_16x16x4.
//
// Per workgroup: a 128 x 128 tile of C, 4 waves of 64 x 64, K in steps of 16.
// Global -> registers (uint32 residues, centered on the way) -> LDS as
// doubles (double buffered) -> MFMA operands.  Every fold_every MFMA steps
// (4 products each) the accumulators are reduced to x - p*rint(x/p), which
// keeps every partial sum an integer of magnitude <= kblock*max|ab| + p + 2
// <= 2^53 and hence exact whatever order the matrix core adds in.  The
// epilogue makes the residue canonical and applies alpha and beta modulo p.
#include "ff_device.h"
#include "ff_internal.h"

namespace ff {

typedef double v4d __attribute__((ext_vector_type(4)));

namespace {

constexpr int LDP = F64_BM + 16; // padded LDS row, in doubles

// One stage's operand words as loaded (raw) with in-matrix flags; they are
// converted after the stage's MFMAs so that the loads' latency overlaps them.
struct F64Regs {
    uint32_t a[8];
    uint32_t b[8];
    uint32_t oka, okb; // bit q: element q lies inside the matrix
};

// Operand element (clamped address, always in bounds) -> centered value, or
// 0 outside the matrix.  The loads are unconditional so that all of a
// stage's loads are in flight together.
template <int MODE>
__device__ __forceinline__ int32_t cvt(uint32_t raw, bool ok, uint32_t p, uint32_t half)
{
    const int32_t v = MODE == IN_SIGNED ? (int32_t)raw : center(raw, p, half);
    return ok ? v : 0;
}

template <int TA, int TB, int MODE>
__device__ __forceinline__ void load_stage(const F64Job &J, int m0, int n0,
                                           int k0, int tid, uint32_t half,
                                           F64Regs &R)
{
    const uint32_t *A = (const uint32_t *)J.A;
    const uint32_t *B = (const uint32_t *)J.B;
    const int km = J.k - 1, mm = J.m - 1, nm = J.n - 1;
    uint32_t oka = 0, okb = 0;
    if (!TA) { // A is m x k: lanes run along k
        const int kg = k0 + (tid & 15);
        const int kc = kg < km ? kg : km;
        const int r0 = m0 + (tid >> 4);
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int r = r0 + 16 * q;
            R.a[q] = A[(int64_t)(r < mm ? r : mm) * J.lda + kc];
            oka |= (uint32_t)(r < J.m && kg < J.k) << q;
        }
    } else { // A is k x m: lanes run along m
        const int r = m0 + (tid & 127), kq = k0 + (tid >> 7);
        const int rc = r < mm ? r : mm;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int kg = kq + 2 * q;
            R.a[q] = A[(int64_t)(kg < km ? kg : km) * J.lda + rc];
            oka |= (uint32_t)(r < J.m && kg < J.k) << q;
        }
    }
    if (!TB) { // B is k x n: lanes run along n
        const int c = n0 + (tid & 127), kq = k0 + (tid >> 7);
        const int cc = c < nm ? c : nm;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int kg = kq + 2 * q;
            R.b[q] = B[(int64_t)(kg < km ? kg : km) * J.ldb + cc];
            okb |= (uint32_t)(c < J.n && kg < J.k) << q;
        }
    } else { // B is n x k: lanes run along k
        const int kg = k0 + (tid & 15);
        const int kc = kg < km ? kg : km;
        const int c0 = n0 + (tid >> 4);
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int c = c0 + 16 * q;
            R.b[q] = B[(int64_t)(c < nm ? c : nm) * J.ldb + kc];
            okb |= (uint32_t)(c < J.n && kg < J.k) << q;
        }
    }
    R.oka = oka;
    R.okb = okb;
}

template <int TA, int TB, int MODE>
__device__ __forceinline__ void store_stage(int tid, const F64Regs &R, uint32_t p,
                                            uint32_t half, double (*sA)[LDP],
                                            double (*sB)[LDP])
{
#define VA(q) (double)cvt<MODE>(R.a[q], (R.oka >> (q)) & 1u, p, half)
#define VB(q) (double)cvt<MODE>(R.b[q], (R.okb >> (q)) & 1u, p, half)
    if (!TA) {
        const int kk = tid & 15, r0 = tid >> 4;
#pragma unroll
        for (int q = 0; q < 8; ++q) sA[kk][r0 + 16 * q] = VA(q);
    } else {
        const int r = tid & 127, kq = tid >> 7;
#pragma unroll
        for (int q = 0; q < 8; ++q) sA[kq + 2 * q][r] = VA(q);
    }
    if (!TB) {
        const int c = tid & 127, kq = tid >> 7;
#pragma unroll
        for (int q = 0; q < 8; ++q) sB[kq + 2 * q][c] = VB(q);
    } else {
        const int kk = tid & 15, c0 = tid >> 4;
#pragma unroll
        for (int q = 0; q < 8; ++q) sB[kk][c0 + 16 * q] = VB(q);
    }
#undef VA
#undef VB
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

// One 128 x 128 output tile.  smem: 2 stages x (A, B) x 16 x LDP doubles.
template <int TA, int TB, int MODE>
__device__ void f64_tile(const F64Job &J, int tm, int tn, double *smem)
{
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int m0 = tm * F64_BM, n0 = tn * F64_BN;
    const int wm0 = (wave >> 1) * 64, wn0 = (wave & 1) * 64;
    const uint32_t half = (J.p - 1) / 2;
    double(*sA)[F64_BK][LDP] = (double(*)[F64_BK][LDP])smem;
    double(*sB)[F64_BK][LDP] = (double(*)[F64_BK][LDP])(smem + 2 * F64_BK * LDP);

    v4d acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};

    const int nk = (J.k + F64_BK - 1) / F64_BK;
    F64Regs R;
    load_stage<TA, TB, MODE>(J, m0, n0, 0, tid, half, R);
    store_stage<TA, TB, MODE>(tid, R, J.p, half, sA[0], sB[0]);
    __syncthreads();

    int cnt = 0;
    for (int kt = 0; kt < nk; ++kt) {
        const int buf = kt & 1;
        if (kt + 1 < nk) load_stage<TA, TB, MODE>(J, m0, n0, (kt + 1) * F64_BK, tid, half, R);
#pragma unroll
        for (int ks = 0; ks < F64_BK / 4; ++ks) {
            const int kr = ks * 4 + (lane >> 4);
            double a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = sA[buf][kr][wm0 + i * 16 + (lane & 15)];
#pragma unroll
            for (int j = 0; j < 4; ++j) b[j] = sB[buf][kr][wn0 + j * 16 + (lane & 15)];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
            if (++cnt == J.fold_every) {
                fold(acc, J.pd, J.pinv);
                cnt = 0;
            }
        }
        if (kt + 1 < nk) store_stage<TA, TB, MODE>(tid, R, J.p, half, sA[buf ^ 1], sB[buf ^ 1]);
        __syncthreads();
    }

    // Epilogue: in each 16 x 16 block the lane holds column lane%16 of rows
    // lane/16 + 4r, r = 0..3 (v_mfma_f64_16x16x4 result layout).
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = m0 + wm0 + i * 16 + (lane >> 4) + 4 * r;
                const int col = n0 + wn0 + j * 16 + (lane & 15);
                if (row < J.m && col < J.n) {
                    const uint32_t v = canon_f64(acc[i][j][r], J.pd, J.pinv, J.p);
                    uint32_t out = mulmod(J.alpha, v, J.p, J.pinv);
                    uint32_t *cp = J.C + (int64_t)row * J.ldc + col;
                    if (J.beta) out = addmod(out, mulmod(J.beta, *cp, J.p, J.pinv), J.p);
                    *cp = out;
                }
            }
}

constexpr size_t F64_SMEM = sizeof(double) * 2 * 2 * F64_BK * LDP;

template <int TA, int TB, int MODE>
__global__ __launch_bounds__(F64_THREADS) void k_fgemm_f64(F64Job J)
{
    __shared__ double smem[F64_SMEM / sizeof(double)];
    const int G = J.tiles_m * J.tiles_n;
    const int t = xcd_remap(blockIdx.x, G);
    int tm, tn;
    grouped_tile<8>(t, J.tiles_m, J.tiles_n, &tm, &tn);
    f64_tile<TA, TB, MODE>(J, tm, tn, smem);
}

// Runtime flags -> instantiation.
template <template <int, int, int> class K, class... Args>
hipError_t f64_dispatch(int ta, int tb, int mode, Args... args)
{
    const int key = ta * 4 + tb * 2 + mode;
    switch (key) {
    case 0: return K<0, 0, 0>::go(args...);
    case 1: return K<0, 0, 1>::go(args...);
    case 2: return K<0, 1, 0>::go(args...);
    case 3: return K<0, 1, 1>::go(args...);
    case 4: return K<1, 0, 0>::go(args...);
    case 5: return K<1, 0, 1>::go(args...);
    case 6: return K<1, 1, 0>::go(args...);
    default: return K<1, 1, 1>::go(args...);
    }
}

__device__ __forceinline__ int find_job_f64(const F64Job *jobs, int njobs, int g)
{
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].tile_start <= g) lo = mid; else hi = mid - 1;
    }
    return lo;
}

template <int TA, int TB, int MODE>
__global__ __launch_bounds__(F64_THREADS) void k_fgemm_f64_batched(
    const F64Job *__restrict__ jobs, int njobs, int total, int persistent,
    unsigned *ctr)
{
    __shared__ double smem[F64_SMEM / sizeof(double)];
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
        const int j = find_job_f64(jobs, njobs, g);
        const F64Job J = jobs[j];
        const int local = g - J.tile_start;
        int tm, tn;
        grouped_tile<8>(local, J.tiles_m, J.tiles_n, &tm, &tn);
        f64_tile<TA, TB, MODE>(J, tm, tn, smem);
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

template <int TA, int TB, int MODE>
struct SingleF64 {
    static hipError_t go(const F64Job &job, hipStream_t st)
    {
        const int G = job.tiles_m * job.tiles_n;
        hipLaunchKernelGGL((k_fgemm_f64<TA, TB, MODE>), dim3(G), dim3(F64_THREADS), 0, st, job);
        return hipGetLastError();
    }
};

template <int TA, int TB, int MODE>
struct BatchedF64 {
    static hipError_t go(const F64Job *jobs, int njobs, int total, int persistent,
                         unsigned *ctr, int grid, hipStream_t st)
    {
        hipLaunchKernelGGL((k_fgemm_f64_batched<TA, TB, MODE>), dim3(grid), dim3(F64_THREADS),
                           0, st, jobs, njobs, total, persistent, ctr);
        return hipGetLastError();
    }
};

} // namespace

hipError_t launch_f64(const F64Job &job, hipStream_t st)
{
    return f64_dispatch<SingleF64>(job.transA, job.transB, job.in_mode, job, st);
}

// A batched table must share transposes and input mode (the first job's).
hipError_t launch_f64_batched(const F64Job *dev_jobs, int njobs, int total_tiles,
                              int persistent, unsigned *ctr, int ta, int tb, int mode,
                              hipStream_t st)
{
    int grid = total_tiles;
    if (persistent) {
        int dev = 0, cus = 256;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        grid = cus * 2 < total_tiles ? cus * 2 : total_tiles;
        if (grid < 1) grid = 1;
    }
    return f64_dispatch<BatchedF64>(ta, tb, mode, (const F64Job *)dev_jobs, njobs, total_tiles,
                                    persistent, ctr, grid, st);
}

} // namespace ff
