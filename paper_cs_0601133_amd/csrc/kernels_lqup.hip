// Kernels of the LQUP factorisation over Z/pZ (Section 5.1).
//
// The factorisation is row recursive (lqup.cpp): blocks of up to 64 rows are
// factored by one workgroup (k_lqup_panel), the rest of the work is the
// triangular solve and the fgemm update of the recursion, plus the column
// exchanges the pivots require (k_lqup_swap), the gathering of the pivot rows
// (k_lqup_gather) and a search for pivots past the panel's window
// (k_lqup_first_nonzero).
#include <type_traits>

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

// Lane l's value of x, in every lane (l uniform).
__device__ __forceinline__ double readlane_d(double x, int l)
{
    const uint64_t u = __builtin_bit_cast(uint64_t, x);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), l);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Polls of a publication flag before a wave gives up (each poll is an LDS
// round trip; a step's wait is a few hundred cycles).  The polls do not
// sleep: a sleep of 64 cycles between them made a factorisation at 4096
// 1.7% slower.
constexpr int SPIN_LIMIT = 1 << 20;

__device__ __forceinline__ bool wait_flag(int *f)
{
    for (int it = 0; it < SPIN_LIMIT; ++it)
        if (__builtin_amdgcn_readfirstlane(
                __hip_atomic_load(f, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP)))
            return true;
    return false;
}

// Panel of the full-rank guess: rows [i0, i0 + nr) taken to pivot in columns
// k, k + 1, ... in order, with no exchange.  The guess holds unless a pivot
// value is 0 (or nr > W); then *fail is set and the caller redoes the
// factorisation on the general path, so this kernel needs no pivot search,
// column exchange or stop.
//
// Elimination is fraction free, as in k_lqup_panel; the synchronisation is
// not a barrier per row.  Row r is published once, into LDS slot r, by the
// wave that holds it, right after its update by row r - 1, and a release
// flag follows.  A wave waits only for the row it needs next and takes its
// multipliers from its own registers (lane r of each of its rows), so waves
// run ahead of one another.  The critical path is one row's update per step,
// plus, every PQ rows, the hand-over to the next wave through LDS.  A
// wave whose rows are all finished leaves the loop.
//
// Below pivot row r, columns c <= r are scaled by the pivot instead of being
// kept, so the multiplier in column c of row r2 ends up carrying the pivots
// c .. r2 - 1 of the steps it went through: L = stored S_c / (pi_c S_r2),
// with S_j = pi_0 ... pi_{j-1}; a U entry is stored / S_r2 as before.
//
// Workgroup b also carries the nc columns past the window, 64 of them from
// column k + W + 64 b, through the same row operations, so that the pivot
// rows' entries there leave finished (the caller's unit lower triangular
// solve for them, fused).
//
// With m2 > 0 (and nr == W) the last ceil(m2 / 16) workgroups eliminate the
// m2 rows from g0 on over the window by all nr pivot rows, as rows below
// them, 16 per workgroup, four in each of the last four waves (those stay to
// the end anyway: the workgroup's work is then that of a carrying one).  The
// multipliers are G with G T = X, T the panel's U in the window and X those
// rows' window entries (the caller's right-hand triangular solve for the
// rows below the panel, fused), stored over X.
//
// Every workgroup factors the window, which they all read, so the last one
// to finish (ctr[2], left zero) writes it, and sets *fail to 1 for a zero
// pivot, 2 if a wait gave up.
//
// With so.ad set, G and the carried columns are also written as the INT8
// digit planes of the product that follows (G times those columns, K = 64):
// the balanced digits of the centered values, in the layout of the digit
// slicer (G as the A operand, the carried columns as the transposed B
// operand), so that the product needs no slicing launch.
template <bool CARRY, bool FOLD>
__global__ __launch_bounds__(PT) void k_lqup_panel_fast(uint32_t *A, int64_t lda, int64_t i0,
                                                        int nr, int64_t k, int W, int64_t nc,
                                                        int64_t g0, int m2, uint32_t p,
                                                        double pinv, int32_t *fail, unsigned *ctr,
                                                        LqupDigits so)
{
    // digits of canonical u as the byte at dst + d plane, d < so.S
    auto put_digits = [&](uint32_t u, int8_t *dst, int64_t plane) {
        const int bits = so.S == 1 ? 8 : so.bits, sh = 32 - bits;
        int32_t v = center(u, p, (p - 1) / 2);
        for (int d = 0; d < so.S; ++d) {
            const int dig = (int)((uint32_t)v << sh) >> sh;
            v = (v - dig) >> bits;
            dst[(int64_t)d * plane] = (int8_t)dig;
        }
    };
    __shared__ double s_row[PR][PW];                // published rows, window
    __shared__ double s_rowx[CARRY ? PR : 1][64];   // and carried columns
    __shared__ int s_flag[PR];
    __shared__ uint32_t s_inv[PR], s_S[PR + 1], s_invS[PR + 1];
    __shared__ int s_bad, s_last;
    const int tid = threadIdx.x, c = tid % 64;
    const int g = __builtin_amdgcn_readfirstlane(tid / 64);
    // the wave's block of PQ rows: waves g, g + 4, g + 8, g + 12 share a SIMD
    // (g mod 4), and a block's work grows with its index, so the blocks are
    // dealt s, 7 - s, 8 + s, 15 - s to SIMD s: the same work on every SIMD
    const int wj = g / 4, ws = g % 4;
    const int gbk = 4 * wj + ((wj & 1) ? 3 - ws : ws);
    const uint32_t half = (p - 1) / 2;
    const double pd = (double)p;
    // gwg: a workgroup of the rows below, whose last four waves hold four of
    // them each (below; x[q] the window entries of row gb + q of them); xc: x
    // holds carried columns (all uniform)
    const int ng = (m2 + 15) / 16;
    const bool gwg = FOLD && (int)blockIdx.x >= (int)gridDim.x - ng;
    const bool xc = CARRY && !gwg;
    const bool below = gwg && gbk >= PG - 4;
    const int gb = 16 * ((int)blockIdx.x - ((int)gridDim.x - ng)) + PQ * (gbk - (PG - 4));
    const int64_t x0 = k + W + 64 * (int64_t)blockIdx.x;
    const int64_t xleft = nc - 64 * (int64_t)blockIdx.x;
    const int xw = xc ? (int)(xleft < 64 ? xleft : 64) : 0;

    double v[PQ], x[PQ];
#pragma unroll
    for (int q = 0; q < PQ; ++q) {
        const int r = PQ * gbk + q;
        uint32_t u = 0, ux = 0;
        if (r < nr && c < W) u = A[(i0 + r) * lda + k + c];
        if (xc && r < nr && c < xw) ux = A[(i0 + r) * lda + x0 + c];
        if (below && gb + q < m2 && c < W) ux = A[(g0 + gb + q) * lda + k + c];
        v[q] = (double)center(u, p, half);
        x[q] = (double)center(ux, p, half);
    }
    if (tid < PR) s_flag[tid] = 0;
    if (tid == 0) s_bad = 0;
    __syncthreads();
    if (gbk == 0) {
        s_row[0][c] = v[0];
        if (xc) s_rowx[0][c] = x[0];
        __hip_atomic_store(&s_flag[0], 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
    }

    int gave_up = 0;
    // step r: the rows after r, by pivot row r (column r); the rows below
    // the panel take every pivot row, the panel's own rows all but the last
    const int steps = gwg ? nr : nr - 1;
    for (int r = 0; r < steps; ++r) {
        const bool done = PQ * gbk + PQ - 1 <= r; // this wave's panel rows are finished
        if (done && !below) break;
        const int gn = (r + 1) / PQ, qn = (r + 1) % PQ;
        double y, yx = 0.0;
        if (gbk == gn && qn != 0) {
            // row r is this wave's row qn - 1
            y = qn == 1 ? v[0] : qn == 2 ? v[1] : v[2];
            if (xc) yx = qn == 1 ? x[0] : qn == 2 ? x[1] : x[2];
        } else {
            if (!gave_up) gave_up = !wait_flag(&s_flag[r]);
            y = s_row[r][c];
            if (xc) yx = s_rowx[r][c];
        }
        const double pv = readlane_d(y, r);
        const double ye = c > r && c < W ? y : 0.0;
        using I0 = std::integral_constant<int, 0>;
        using I1 = std::integral_constant<int, 1>;
        using I2 = std::integral_constant<int, 2>;
        using I3 = std::integral_constant<int, 3>;
        using I4 = std::integral_constant<int, 4>;
        // the panel's rows of this wave after r; WX: with their carried
        // columns (x), else x is left alone
        auto own_rows = [&](auto wxc) {
            constexpr bool WX = decltype(wxc)::value;
            // rows [q0, q1): the multipliers first, then each stage for all
            // rows, so that their chains of dependent operations overlap
            auto update = [&](auto q0c, auto q1c) {
                constexpr int q0 = decltype(q0c)::value, q1 = decltype(q1c)::value;
                double a[PQ], t[PQ], tx[PQ];
#pragma unroll
                for (int q = q0; q < q1; ++q) a[q] = readlane_d(v[q], r);
#pragma unroll
                for (int q = q0; q < q1; ++q) {
                    t[q] = __builtin_fma(pv, v[q], -a[q] * ye);
                    if (WX) tx[q] = __builtin_fma(pv, x[q], -a[q] * yx);
                }
#pragma unroll
                for (int q = q0; q < q1; ++q) {
                    v[q] = reduce_c(t[q], pd, pinv);
                    if (WX) x[q] = reduce_c(tx[q], pd, pinv);
                }
            };
            auto publish = [&](double w, double wx) {
                s_row[r + 1][c] = w;
                if (WX) s_rowx[r + 1][c] = wx;
            };
            if (gbk == gn) {
                // row r + 1 (this wave's row qn) first, at raised priority:
                // its entries go out before the rows after it are updated,
                // the flag after them
                __builtin_amdgcn_s_setprio(3);
                switch (qn) {
                case 0:
                    update(I0{}, I1{}); publish(v[0], x[0]); update(I1{}, I4{});
                    break;
                case 1:
                    update(I1{}, I2{}); publish(v[1], x[1]); update(I2{}, I4{});
                    break;
                case 2:
                    update(I2{}, I3{}); publish(v[2], x[2]); update(I3{}, I4{});
                    break;
                default:
                    update(I3{}, I4{}); publish(v[3], x[3]);
                    break;
                }
                __hip_atomic_store(&s_flag[r + 1], 1, __ATOMIC_RELEASE,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
            } else {
                __builtin_amdgcn_s_setprio(0);
                update(I0{}, I4{});
            }
        };
        if (!done) {
            if (xc) own_rows(std::integral_constant<bool, CARRY>{});
            else own_rows(std::false_type{});
        }
        if (FOLD && below) {
            // the wave's rows below the panel, by their own multipliers
            double a[PQ], t[PQ];
#pragma unroll
            for (int q = 0; q < PQ; ++q) a[q] = readlane_d(x[q], r);
#pragma unroll
            for (int q = 0; q < PQ; ++q) t[q] = __builtin_fma(pv, x[q], -a[q] * ye);
#pragma unroll
            for (int q = 0; q < PQ; ++q) x[q] = reduce_c(t[q], pd, pinv);
        }
    }
    __builtin_amdgcn_s_setprio(0);
    if (gave_up && c == 0) atomicOr(&s_bad, 2);
    __syncthreads();
    // pivots pi_j: row j as published (every update applied); inverses, and
    // the prefix products S_j and 1 / S_j
    if (tid < 64) {
        uint32_t pi = 1, iv = 1;
        if (tid < nr) {
            pi = canon_f64(s_row[tid][tid], pd, pinv, p);
            iv = inv_mod(pi, p);
            if (pi == 0) atomicOr(&s_bad, 1);
        }
        s_inv[tid] = iv;
        uint32_t sp = pi, si = iv; // inclusive products over lanes <= tid
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const uint32_t up = __shfl_up(sp, d, 64), ui = __shfl_up(si, d, 64);
            if (tid >= d) {
                sp = mulmod(sp, up, p, pinv);
                si = mulmod(si, ui, p, pinv);
            }
        }
        s_S[tid + 1] = sp;
        s_invS[tid + 1] = si;
        if (tid == 0) {
            s_S[0] = 1u;
            s_invS[0] = 1u;
        }
    } else if (tid == 64) {
        // (a second wave: the counter's round trip beside the inverses)
        s_last = gridDim.x == 1 || atomicAdd(&ctr[2], 1u) == gridDim.x - 1;
    }
    __syncthreads();
    if (xc) {
#pragma unroll
        for (int q = 0; q < PQ; ++q) {
            const int r = PQ * gbk + q;
            if (r < nr && c < xw) {
                const uint32_t u = mulmod(canon_f64(x[q], pd, pinv, p), s_invS[r], p, pinv);
                A[(i0 + r) * lda + x0 + c] = u;
                if (so.bd) {
                    // row j of the transposed operand, K index r
                    const int64_t j = 64 * (int64_t)blockIdx.x + c;
                    put_digits(u, so.bd + (j / so.rtb) * so.rtb * 64 + (r / 16) * so.rtb * 16 +
                                      (j % so.rtb) * 16 + r % 16, so.plane_b);
                }
            }
        }
    }
    if (below && c < W) {
        // G = stored S_c / (pi_c S_nr): every pivot row went through it
        const uint32_t f = mulmod(mulmod(s_S[c], s_inv[c], p, pinv), s_invS[nr], p, pinv);
#pragma unroll
        for (int q = 0; q < PQ; ++q)
            if (gb + q < m2) {
                const uint32_t u = mulmod(canon_f64(x[q], pd, pinv, p), f, p, pinv);
                A[(g0 + gb + q) * lda + k + c] = u;
                if (so.ad) {
                    // row i of the A operand, K index c
                    const int64_t i = gb + q;
                    put_digits(u, so.ad + (i / so.rta) * so.rta * 64 + (c / 16) * so.rta * 16 +
                                      (i % so.rta) * 16 + c % 16, so.plane_a);
                }
            }
    }
    if (!s_last) return;
    if (c < W) {
        const uint32_t colf = c < nr ? mulmod(s_S[c], s_inv[c], p, pinv) : 0u;
#pragma unroll
        for (int q = 0; q < PQ; ++q) {
            const int r = PQ * gbk + q;
            if (r >= nr) continue;
            const uint32_t f = c < r ? mulmod(colf, s_invS[r], p, pinv) : s_invS[r];
            A[(i0 + r) * lda + k + c] = mulmod(canon_f64(v[q], pd, pinv, p), f, p, pinv);
        }
    }
    if (tid == 0) {
        if (s_bad) *fail = s_bad;
        if (gridDim.x > 1) atomicExch(&ctr[2], 0u);
    }
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

bool lqup_panel_fast_ok(uint32_t p)
{
    const double h = (double)(p / 2) + 2.0;
    return 2.0 * h * h <= 9007199254740992.0;
}

hipError_t launch_lqup_panel_fast(uint32_t *A, int64_t lda, int64_t i0, int nr, int64_t k, int W,
                                  int64_t nc, int64_t g0, int m2, uint32_t p, int32_t *fail,
                                  unsigned *ctr, hipStream_t st, const LqupDigits &so)
{
    if (so.ad && (m2 <= 0 || nc <= 0 || !so.bd || nr != 64 || so.S < 1 || so.S > 5 ||
                  so.rta < 1 || so.rtb < 1 || (so.S > 1 && (so.bits < 2 || so.bits > 8))))
        return hipErrorInvalidValue;
    if (nr < 1 || nr > PR || W < 1 || W > PW || nc < 0 || m2 < 0 || m2 > (1 << 20) ||
        (m2 > 0 && nr != W) || !fail || !ctr || !lqup_panel_fast_ok(p))
        return hipErrorInvalidValue;
    // carried-column workgroups, then those of the rows below
    const int64_t nb = (nc + 63) / 64 + (m2 + 15) / 16;
    if (nb > 0x7FFFFFFF) return hipErrorInvalidValue;
    if (m2 > 0)
        hipLaunchKernelGGL((k_lqup_panel_fast<true, true>), dim3((unsigned)nb), dim3(PT), 0, st, A,
                           lda, i0, nr, k, W, nc, g0, m2, p, 1.0 / (double)p, fail, ctr, so);
    else if (nb > 0)
        hipLaunchKernelGGL((k_lqup_panel_fast<true, false>), dim3((unsigned)nb), dim3(PT), 0, st,
                           A, lda, i0, nr, k, W, nc, g0, 0, p, 1.0 / (double)p, fail, ctr,
                           LqupDigits{});
    else
        hipLaunchKernelGGL((k_lqup_panel_fast<false, false>), dim3(1), dim3(PT), 0, st, A, lda, i0,
                           nr, k, W, nc, g0, 0, p, 1.0 / (double)p, fail, ctr, LqupDigits{});
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
