// Kernels of the LQUP factorisation over Z/pZ (Section 5.1).
//
// The factorisation is row recursive (lqup.cpp): blocks of up to 64 rows are
// factored by one workgroup (k_lqup_panel), the rest of the work is the
// triangular solve and the fgemm update of the recursion, plus the column
// exchanges the pivots require (k_lqup_swap), the gathering of the pivot rows
// (k_lqup_gather) and a search for pivots past the panel's window
// (k_lqup_first_nonzero).
#include "ff_device.h"
#include "ff_internal.h"

namespace ff {

namespace {

constexpr int PR = LQUP_PANEL;    // rows of a panel
constexpr int PW = LQUP_WINDOW;   // columns of the panel's window
constexpr int PT = 1024;          // threads: PW columns x PG row groups
constexpr int PG = PT / PW;       // row groups
constexpr int PQ = PR / PG;       // rows per group
static_assert(PR == 64 && PW == 64, "panel: column tid % 64, rows 4 (tid / 64) + q");

__device__ __forceinline__ double reduce_c(double x, double pd, double pinv)
{
    return __builtin_fma(-__builtin_rint(x * pinv), pd, x);
}

// Inverse of a unit a modulo p (extended Euclid); 0 if a is not a unit.
// Remainders stay below p < 2^31 (32-bit division steps); the Bezout
// coefficients need 64 bits.
__device__ __forceinline__ uint32_t inv_mod(uint32_t a, uint32_t p)
{
    uint32_t r0 = p, r1 = a % p;
    int64_t s0 = 0, s1 = 1;
    while (r1 != 0) {
        const uint32_t q = r0 / r1, r2 = r0 - q * r1;
        const int64_t s2 = s0 - (int64_t)q * s1;
        r0 = r1; r1 = r2; s0 = s1; s1 = s2;
    }
    if (r0 != 1) return 0;
    return (uint32_t)(s0 < 0 ? s0 + (int64_t)p : s0);
}

// One panel: rows [i0, i0 + nr) (nr <= 64) over the window of columns
// [k, k + W) (W <= 64), every entry already reduced by the pivots above.
// Thread (c, g) owns column c of the window and the contiguous rows
// 4g .. 4g + 3; the walk over rows unrolls and a group whose rows are all
// above the pivot row skips the update (the test is uniform per wave).
// Within a group the four rows' updates are computed without a branch per
// row and kept where they apply: with a branch each row waited for its own
// multiplier from LDS before its chain of dependent steps (50 -> 43 us per
// panel without).
// Rows are processed in order: a row pivots on its first nonzero entry at or
// after column t (the next pivot index), exchanged into column t inside the
// panel; a row with no such entry is dependent if the window reaches the
// last column (whole), else the panel stops there (the caller searches the
// columns past the window).  A window of 64 columns holds the pivots of
// all 64 rows when they are independent there (the usual case); a
// 128-column window (twice the update work per row) measured 13% slower
// over a whole factorisation at 4096.
//
// Elimination is fraction free: below pivot row r (pivot value pi, entry a
// of row r2 in column t) row r2 <- pi row r2 - a row r on the columns after
// t, and a stays in column t.  Every row below a pivot is scaled by the same
// factor S_t = pi_0 ... pi_{t-1} (products of the values found), so a / pi
// is the exact multiplier and the true row is the stored one divided by
// S_t; the inverses are taken once at the end, in parallel, instead of one
// per pivot on the critical path.
//
// EXACT: entries as centered doubles, pi x - a y exact while
// 2 (p/2 + 2)^2 <= 2^53; otherwise canonical residues and mulmod.
//
// out: [0] pivots t, [1] rows processed, [2] stuck, [3 + r] = pivot index
// of processed row r or -1 (dependent), [3 + 64 + j] = window column that
// pivot j came from (== j: no exchange).
//
// fail (may be null): set to 1 unless every row of the panel pivots in its
// own column (the full-rank guess of the caller's fast path).
template <bool EXACT>
__global__ __launch_bounds__(PT) void k_lqup_panel(uint32_t *A, int64_t lda, int64_t i0, int nr,
                                                   int64_t k, int W, int whole, uint32_t p,
                                                   double pinv, int32_t *out, int32_t *fail)
{
    // published pivot row, column t and search results, double-buffered by
    // row parity so that a row's writes never meet the previous row's reads
    // (one barrier per row unless a column exchange is needed)
    __shared__ double s_row[2][PW];
    __shared__ double s_col[2][PR];
    __shared__ double s_swap[2][PR];   // column exchange
    __shared__ uint32_t s_piv[PR];     // pivot values (fraction-free, canonical)
    __shared__ uint32_t s_inv[PR];     // their inverses
    __shared__ uint32_t s_invS[PR + 1]; // inverse scale after j pivots
    __shared__ int s_first[2][PW / 64];
    __shared__ int s_rowpiv[PR];       // pivot index of a row, -1 dependent, -2 untouched
    __shared__ int s_before[PR];       // pivots above the row when it was processed
    const int tid = threadIdx.x, lane = tid & 63;
    // g is the wave index (PW = 64): uniform, so tests on it are scalar
    const int c = tid % PW, g = __builtin_amdgcn_readfirstlane(tid / PW), r0g = PQ * g;
    const uint32_t half = (p - 1) / 2;
    const double pd = (double)p;

    double v[PQ];
#pragma unroll
    for (int q = 0; q < PQ; ++q) {
        const int r = r0g + q;
        uint32_t u = 0;
        if (r < nr && c < W) u = A[(i0 + r) * lda + k + c];
        v[q] = EXACT ? (double)center(u, p, half) : (double)u;
    }
    if (tid < PR) {
        s_rowpiv[tid] = -2;
        s_before[tid] = 0;
    }
    __syncthreads();

    int t = 0, nproc = 0, stuck = 0, exchanged = 0;
    // every loop has a constant trip count (it unrolls; v[] stays in
    // registers); rows past nr and rows after a stop are skipped by tests
    // that are uniform across the workgroup
#pragma unroll
    for (int r = 0; r < PR; ++r) {
        if (stuck || r >= nr) continue;
        const int gr = r / PQ, qr = r % PQ, pb = r & 1;
        // row r: publish it, and find its first nonzero at or after column t;
        // column t is published at the same time, on the guess (almost always
        // right) that it holds the pivot, so that one barrier serves both
        if (g == gr) {
            s_row[pb][c] = v[qr];
            const bool nz = c >= t && c < W && v[qr] != 0.0;
            const uint64_t bal = __ballot(nz);
            if (lane == 0) s_first[pb][c / 64] = bal ? (c - lane) + __builtin_ctzll(bal) : PW;
        }
        if (c == t) {
#pragma unroll
            for (int q = 0; q < PQ; ++q) s_col[pb][r0g + q] = v[q];
        }
        __syncthreads();
        int cmin = PW;
#pragma unroll
        for (int ww = 0; ww < PW / 64; ++ww) cmin = min(cmin, s_first[pb][ww]);
        if (cmin >= PW) {
            if (!whole) {
                stuck = 1;
            } else {
                if (tid == 0) { s_rowpiv[r] = -1; s_before[r] = t; }
                ++nproc; // dependent row: zero from column t on
            }
            continue;
        }
        if (cmin != t) {
            exchanged = 1;
            // exchange columns t and cmin in every row of the panel, then
            // publish the new column t and row r's two changed entries
            if (c == t) {
#pragma unroll
                for (int q = 0; q < PQ; ++q) s_swap[0][r0g + q] = v[q];
            }
            if (c == cmin) {
#pragma unroll
                for (int q = 0; q < PQ; ++q) s_swap[1][r0g + q] = v[q];
            }
            __syncthreads();
            if (c == t) {
#pragma unroll
                for (int q = 0; q < PQ; ++q) v[q] = s_swap[1][r0g + q];
#pragma unroll
                for (int q = 0; q < PQ; ++q) s_col[pb][r0g + q] = v[q];
            }
            if (c == cmin) {
#pragma unroll
                for (int q = 0; q < PQ; ++q) v[q] = s_swap[0][r0g + q];
            }
            if (g == gr && (c == t || c == cmin)) s_row[pb][c] = v[qr];
            __syncthreads();
        }
        if (tid == 0) {
            s_rowpiv[r] = t;
            s_before[r] = t;
            out[3 + PR + t] = cmin;
        }
        const double pv = s_col[pb][r];
        if (tid == 0) {
            const double pc = EXACT ? (pv < 0 ? pv + pd : pv) : pv;
            s_piv[t] = (uint32_t)pc;
        }
        // rows below r, columns after t (groups entirely above r skip).  The
        // group's multipliers are read together and every row's update is
        // computed, then kept where it applies (no branch per row: the
        // rows' dependent chains overlap instead of running one by one)
        if (g >= gr) {
            const double y = s_row[pb][c];
            double a[PQ];
#pragma unroll
            for (int q = 0; q < PQ; ++q) a[q] = s_col[pb][r0g + q];
            const bool colok = c > t && c < W;
#pragma unroll
            for (int q = 0; q < PQ; ++q) {
                const int r2 = r0g + q;
                double nv;
                if (EXACT) {
                    nv = reduce_c(__builtin_fma(pv, v[q], -a[q] * y), pd, pinv);
                } else {
                    const uint32_t x1 = mulmod((uint32_t)pv, (uint32_t)v[q], p, pinv);
                    const uint32_t x2 = mulmod((uint32_t)a[q], (uint32_t)y, p, pinv);
                    nv = (double)(x1 >= x2 ? x1 - x2 : x1 + p - x2);
                }
                v[q] = colok && r2 > r && r2 < nr ? nv : v[q];
            }
        }
        ++t;
        ++nproc;
    }
    __syncthreads();
    // inverses of the pivots, and of the scales S_j = pi_0 ... pi_{j-1}
    if (tid < t) s_inv[tid] = inv_mod(s_piv[tid], p);
    __syncthreads();
    if (tid < 64) {
        // inclusive prefix product over lanes < t, then shifted by one
        uint32_t x = lane < t ? s_inv[lane] : 1u;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const uint32_t y = __shfl_up(x, d, 64);
            if (lane >= d) x = mulmod(x, y, p, pinv);
        }
        s_invS[lane + 1] = x;
        if (lane == 0) s_invS[0] = 1u;
    }
    __syncthreads();
    // undo the scaling and store canonical residues
    if (c < W) {
        const uint32_t invc = c < t ? s_inv[c] : 0u;
#pragma unroll
        for (int q = 0; q < PQ; ++q) {
            const int r = r0g + q;
            if (r >= nr) continue;
            const int rp = s_rowpiv[r];
            const int before = rp == -2 ? t : s_before[r];
            uint32_t u;
            if (EXACT) {
                const double x = v[q];
                u = (uint32_t)(x < 0 ? x + pd : x);
            } else {
                u = (uint32_t)v[q];
            }
            if (c < before) u = mulmod(u, invc, p, pinv);         // multiplier a / pi
            else u = mulmod(u, s_invS[before], p, pinv);          // row / S
            A[(i0 + r) * lda + k + c] = u;
        }
    }
    if (tid == 0) {
        out[0] = t;
        out[1] = nproc;
        out[2] = stuck;
        if (fail && (t != nr || stuck || exchanged)) *fail = 1;
    }
    if (tid < PR) out[3 + tid] = s_rowpiv[tid];
}

// Column exchanges (c1, c2), in order, applied to every row outside
// [skip_lo, skip_hi); one thread per row.
__global__ __launch_bounds__(256) void k_lqup_swap(uint32_t *A, int64_t lda, int64_t m,
                                                   int64_t skip_lo, int64_t skip_hi,
                                                   const int64_t *pairs, int npairs)
{
    const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (r >= m || (r >= skip_lo && r < skip_hi)) return;
    uint32_t *row = A + r * lda;
    for (int j = 0; j < npairs; ++j) {
        const int64_t c1 = pairs[2 * j], c2 = pairs[2 * j + 1];
        const uint32_t x = row[c1];
        row[c1] = row[c2];
        row[c2] = x;
    }
}

// U[j][c] = A[rows[j]][c0 + c] for j < r, c < ncols.
__global__ __launch_bounds__(256) void k_lqup_gather(const uint32_t *A, int64_t lda,
                                                     const int64_t *rows, int64_t r, int64_t c0,
                                                     int64_t ncols, uint32_t *U, int64_t ldu)
{
    const int64_t j = blockIdx.y;
    const uint32_t *src = A + rows[j] * lda + c0;
    uint32_t *dst = U + j * ldu;
    for (int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x; c < ncols;
         c += (int64_t)gridDim.x * 256)
        dst[c] = src[c];
}

// out[r] = first column c in [c0, n) with A[i0 + r][c] != 0, or -1; one
// workgroup per row.
__global__ __launch_bounds__(256) void k_lqup_first_nonzero(const uint32_t *A, int64_t lda,
                                                            int64_t i0, int64_t c0, int64_t n,
                                                            int64_t *out)
{
    __shared__ int64_t s_min[4];
    const int64_t r = blockIdx.x;
    const uint32_t *row = A + (i0 + r) * lda;
    int64_t best = INT64_MAX;
    for (int64_t c = c0 + threadIdx.x; c < n; c += 256)
        if (row[c] != 0) { best = c; break; }
    // minimum over the workgroup
    for (int d = 32; d > 0; d >>= 1) {
        const int64_t o = __shfl_down(best, d, 64);
        best = o < best ? o : best;
    }
    if ((threadIdx.x & 63) == 0) s_min[threadIdx.x >> 6] = best;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t b = s_min[0];
        for (int w = 1; w < 4; ++w) b = s_min[w] < b ? s_min[w] : b;
        out[r] = b == INT64_MAX ? -1 : b;
    }
}

} // namespace

hipError_t launch_lqup_panel(uint32_t *A, int64_t lda, int64_t i0, int nr, int64_t k, int W,
                             int whole, uint32_t p, int32_t *out, hipStream_t st, int32_t *fail)
{
    if (nr < 1 || nr > PR || W < 1 || W > PW) return hipErrorInvalidValue;
    const double h = (double)(p / 2) + 2.0;
    const bool exact = 2.0 * h * h <= 9007199254740992.0;
    if (exact)
        hipLaunchKernelGGL(k_lqup_panel<true>, dim3(1), dim3(PT), 0, st, A, lda, i0, nr, k, W,
                           whole, p, 1.0 / (double)p, out, fail);
    else
        hipLaunchKernelGGL(k_lqup_panel<false>, dim3(1), dim3(PT), 0, st, A, lda, i0, nr, k, W,
                           whole, p, 1.0 / (double)p, out, fail);
    return hipGetLastError();
}

hipError_t launch_lqup_swap(uint32_t *A, int64_t lda, int64_t m, int64_t skip_lo, int64_t skip_hi,
                            const int64_t *pairs, int npairs, hipStream_t st)
{
    if (m <= 0 || npairs <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_lqup_swap, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st, A, lda,
                       m, skip_lo, skip_hi, pairs, npairs);
    return hipGetLastError();
}

// Z = I (n x n, row stride n); a grid-stride loop over the entries.
__global__ __launch_bounds__(256) void k_lqup_identity(uint32_t *Z, int64_t n)
{
    const int64_t total = n * n;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * 256)
        Z[e] = (e / n == e % n) ? 1u : 0u;
}

hipError_t launch_lqup_identity(uint32_t *Z, int64_t n, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    const unsigned g = (unsigned)std::min<int64_t>((n * n + 255) / 256, 8192);
    hipLaunchKernelGGL(k_lqup_identity, dim3(g), dim3(256), 0, st, Z, n);
    return hipGetLastError();
}

hipError_t launch_lqup_gather(const uint32_t *A, int64_t lda, const int64_t *rows, int64_t r,
                              int64_t c0, int64_t ncols, uint32_t *U, int64_t ldu, hipStream_t st)
{
    if (r <= 0 || ncols <= 0) return hipSuccess;
    if (r > 65535) return hipErrorInvalidValue;
    const unsigned gx = (unsigned)std::min<int64_t>((ncols + 255) / 256, 64);
    hipLaunchKernelGGL(k_lqup_gather, dim3(gx, (unsigned)r), dim3(256), 0, st, A, lda, rows, r,
                       c0, ncols, U, ldu);
    return hipGetLastError();
}

hipError_t launch_lqup_first_nonzero(const uint32_t *A, int64_t lda, int64_t i0, int64_t nr,
                                     int64_t c0, int64_t n, int64_t *out, hipStream_t st)
{
    if (nr <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_lqup_first_nonzero, dim3((unsigned)nr), dim3(256), 0, st, A, lda, i0, c0,
                       n, out);
    return hipGetLastError();
}

} // namespace ff
