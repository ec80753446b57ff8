// Planner: the host-side decisions of one fgemm call.
//
// * Centered residues (Section 2.1.2: the balanced representation halves
//   the accumulation bound).  For modulus p they lie in [-(p/2), (p-1)/2].
// * Winograd levels (Section 3.2.1): l = floor(log2(n/w)) + 1 for the
//   crossover order w, clamped at 0, or as requested.  The paper leaves w to
//   experiment; measured here, the order at which the first level pays and
//   the leaf order at which one more does differ, and both depend on the
//   leaf arithmetic, so the automatic rule takes a first level at
//   n >= w_first and each further one while the leaf order stays >= w_next
//   (w_first = w_next = w is the single-threshold rule; FF_WINOGRAD_W sets
//   that).  Each level's
//   pre-additions widen the operand range; with unreduced pre-additions (the
//   delayed form Theorem 3.1 analyses) the widest leaf operand after l levels
//   and the largest leaf product term follow from interval arithmetic over
//   the coefficient tables below.  The leaf product term bound equals
//   v_l^A v_l^B of Theorem 3.1.
// * FP64 path: kblock = largest kb with kb * max|a*b| + carry <= 2^53, the
//   binary64 exactness limit (eq. (2) read with gamma = 53 and the residue
//   carried between blocks, carry = p + 2, which bounds |x - p*rint(x/p)|
//   after one floating-point-inverse reduction).
// * INT8 path: the smallest number S of signed digits (7- or 8-bit) that
//   covers the operand range; int32 K-block = floor((2^31-1) / (S dA dB))
//   since one accumulator sums the S digit pairs of equal weight.
#include <algorithm>
#include <cstdlib>
#include <vector>

#include "ff_internal.h"

namespace ff {

namespace {

constexpr int64_t TWO53 = int64_t(1) << 53;
constexpr int64_t I32MAX = 2147483647;

// Coefficients of the seven leaf operands of one Winograd level on the four
// quadrants (11, 12, 21, 22), products P1..P7 (Appendix A).
const int PRE_A[7][4] = {
    {1, 0, 0, 0},   // A11
    {0, 1, 0, 0},   // A12
    {1, 1, -1, -1}, // S4 = A12 - (A21 + A22 - A11)
    {0, 0, 0, 1},   // A22
    {0, 0, 1, 1},   // S1 = A21 + A22
    {-1, 0, 1, 1},  // S2 = S1 - A11
    {1, 0, -1, 0},  // S3 = A11 - A21
};
const int PRE_B[7][4] = {
    {1, 0, 0, 0},   // B11
    {0, 0, 1, 0},   // B21
    {0, 0, 0, 1},   // B22
    {1, -1, -1, 1}, // T4 = T2 - B21
    {-1, 1, 0, 0},  // T1 = B12 - B11
    {1, -1, 0, 1},  // T2 = B22 - T1
    {0, -1, 0, 1},  // T3 = B22 - B12
};

struct Range { int64_t lo, hi; };

Range combine(const int *c, Range x)
{
    Range r{0, 0};
    for (int q = 0; q < 4; ++q) {
        if (c[q] > 0) { r.lo += c[q] * x.lo; r.hi += c[q] * x.hi; }
        else if (c[q] < 0) { r.lo += c[q] * x.hi; r.hi += c[q] * x.lo; }
    }
    return r;
}

int64_t mag(Range r) { return std::max(-r.lo, r.hi); }

void leaf_bounds(Range base, int L, Range *widest, int64_t *max_prod)
{
    std::vector<std::pair<Range, Range>> cur{{base, base}}, nxt;
    for (int l = 0; l < L; ++l) {
        nxt.clear();
        for (auto &pr : cur)
            for (int q = 0; q < 7; ++q)
                nxt.push_back({combine(PRE_A[q], pr.first),
                               combine(PRE_B[q], pr.second)});
        cur.swap(nxt);
    }
    Range w{0, 0};
    int64_t mp = 0;
    for (auto &pr : cur) {
        w.lo = std::min({w.lo, pr.first.lo, pr.second.lo});
        w.hi = std::max({w.hi, pr.first.hi, pr.second.hi});
        mp = std::max(mp, mag(pr.first) * mag(pr.second));
    }
    *widest = w;
    *max_prod = mp;
}

// Smallest number of signed digits of the given width covering [lo, hi];
// one direct int8 plane when the range fits int8.  0 if more than 5.
int slices_for(Range r, int bits)
{
    if (r.lo >= -128 && r.hi <= 127) return 1;
    const int64_t R = int64_t(1) << bits;
    int64_t geo = 1, pw = 1;
    for (int s = 1; s <= 5; ++s) {
        // s digits in [-R/2, R/2 - 1] cover [-(R/2) geo, (R/2 - 1) geo]
        if (-(R / 2) * geo <= r.lo && r.hi <= (R / 2 - 1) * geo) return s;
        pw *= R;
        geo += pw;
    }
    return 0;
}

int64_t digit_mag(Range r, int bits, int S)
{
    if (S == 1 && r.lo >= -128 && r.hi <= 127) return mag(r);
    return int64_t(1) << (bits - 1);
}

int64_t round_up(int64_t x, int64_t q) { return (x + q - 1) / q * q; }

int64_t ipow7(int L) { int64_t r = 1; while (L--) r *= 7; return r; }

// Winograd buffers of the leaf problem (ml x kl times kl x nl, 7^L leaves):
// int32 combinations of both sides in two ping-pong sets (the first only
// once two levels are stored: unfused, or fused from L = 3 on; the second
// from L = 2 on), and the products' two sets.
int64_t wino_buffers(int64_t ml, int64_t nl, int64_t kl, int L, bool one_pass)
{
    const int64_t nleaf = ipow7(L);
    const int64_t szA = round_up(nleaf * ml * kl * 4, 256), szB = round_up(nleaf * kl * nl * 4, 256),
                  szP = round_up(nleaf * ml * nl * 4, 256);
    const bool fused = one_pass && wino_fused_enabled();
    const bool need0 = !fused || L >= 3;
    return (need0 ? szA + szB : 0) + (L > 1 ? szA + szB + szP : 0) + szP;
}

// Tile configuration for the INT8 kernel: FF_I8_TILE (an id of the right
// slice count) overrides; else the autotuner's cache; else the default.
// One-digit products (a single accumulator set per block) take the 256 x 256
// tile (waves of 128 x 64, fewer bytes through LDS per matrix-core step)
// when its tiles fill whole rounds of one workgroup per CU; measured on
// MI355X at 8192^3, p = 251: 0.585 against 0.63 ms for the default two
// 128 x 128 workgroups per CU.
int choose_i8_tile(int S, int64_t m, int64_t n, int64_t k, const ff_opts &)
{
    const char *e = std::getenv("FF_I8_TILE");
    if (e && *e) {
        const int id = std::atoi(e);
        if (id >= 0 && id < i8_tile_count() && i8_tile(id).S == S) return id;
    }
    const int tuned = tuned_i8_tile(S, m, n, k);
    if (tuned >= 0) return tuned;
    if (S == 1 && m > 0 && n > 0) {
        constexpr int64_t CUS = 256; // MI355X
        constexpr int BIG = 21;
        const I8Tile &t = i8_tile(BIG);
        const int64_t tiles = ((m + t.bm() - 1) / t.bm()) * ((n + t.bn() - 1) / t.bn());
        if (tiles >= CUS && tiles % CUS == 0) return BIG;
    }
    return i8_default_tile(S);
}

struct Crossover {
    int64_t first, next;
};

// Measured on MI355X (square products, one level against none): INT8
// leaves of one digit never gain (the digit product costs about what the
// extra passes move); INT8 leaves of 2..5 digits gain 4-15% from n = 3072
// on with residues below 2^30, and 3-8% from 8192 on above (wider
// arithmetic in the fused pre-addition); a second INT8 level gains at most
// 1% up to 16384.  FP64 leaves: one level ties at 2048 and gains 8-40% from
// 3072 on, a second one gains from leaf order 3072 (the paper's rule with
// w = 3072).
Crossover crossover(int path, int s0, uint32_t p)
{
    const char *e = std::getenv("FF_WINOGRAD_W");
    if (e && std::atoll(e) > 0) return {std::atoll(e), std::atoll(e)};
    constexpr int64_t NEVER = int64_t(1) << 62;
    if (path == FF_PATH_FP64) return {3072, 3072};
    if (s0 <= 1) return {NEVER, NEVER};
    if (p >= (1u << 30)) return {8192, 24576};
    return {3072, 12288};
}

} // namespace

// Products small enough that the three launches of the general FP64 path
// (packing, GEMM with a K split, split reduction) cost more than one
// launch of 32 x 32 tiles over the whole K.
bool f64_small(int64_t m, int64_t n, int64_t k)
{
    // the kernel's limits: int dimensions, at most 65535 tile rows
    if (m > int64_t(65535) * 16 || n > 0x3FFFFFFF || k > 0x3FFFFFFF) return false;
    const char *e = std::getenv("FF_F64_SMALL");
    if (e && *e == '0') return false;
    if (e && *e == '1') return true;
    return m * n <= 512 * 512 && k <= 768;
}

// FF_F64_TILE (an id) overrides the default FP64 configuration.  A single
// product, or the `count` equal leaves of a Winograd batch, takes the
// 256 x 128 tile when its tiles fill whole rounds of one workgroup per CU
// (more reuse per tile), else the 128 x 128 tile, whose shorter tail wins
// there.  Measured on MI355X: 256 x 128 is 2.7% faster at 4096 (512 tiles),
// 128 x 128 is 9-24% faster at 3072, 5120 and 6144 and 7% on the seven
// 2048^2 leaves of a 4096 product; batches keep the default.
int choose_f64_tile(int64_t m, int64_t n, int64_t count)
{
    const char *e = std::getenv("FF_F64_TILE");
    if (e && *e) {
        const int id = std::atoi(e);
        if (id >= 0 && id < f64_tile_count()) return id;
    }
    if (m <= 0 || n <= 0) return f64_default_tile();
    constexpr int64_t CUS = 256; // MI355X
    const F64Tile &big = f64_tile(f64_default_tile());
    const int64_t tiles = count * ((m + big.bm() - 1) / big.bm()) * ((n + big.bn() - 1) / big.bn());
    if (tiles >= CUS && tiles % CUS == 0) return f64_default_tile();
    return 2;
}

// A single FP64 launch with fewer workgroup tiles than CUs (256) splits K so
// that about 512 workgroups run (a wave's 64 x 64 block over all of K is a
// long serial chain of matrix-core steps, and a few tiles leave most CUs
// idle).
int f64_splits(int64_t tiles, int64_t nk, int *kt_split)
{
    int64_t s = 1;
    if (tiles < 256 && nk > 1) s = std::min<int64_t>(nk, std::max<int64_t>(1, 512 / tiles));
    const int64_t per = (nk + s - 1) / s;
    *kt_split = s > 1 ? (int)per : 0;
    return s > 1 ? (int)((nk + per - 1) / per) : 1;
}

int make_plan(uint32_t p, int64_t m, int64_t n, int64_t k, const ff_opts &o,
              Plan *pl)
{
    Plan P;
    if (p < 2 || p > 0x7FFFFFFFu)
        return fail(FF_EINVAL, "modulus p must satisfy 2 <= p < 2^31");
    if (o.path < 0 || o.path > 2)
        return fail(FF_EINVAL, "unknown path");
    if (o.digit_bits != 0 && o.digit_bits != 7 && o.digit_bits != 8)
        return fail(FF_EINVAL, "digit_bits must be 0, 7 or 8");
    if (o.winograd_levels < -1 || o.winograd_levels > 3)
        return fail(FF_EINVAL, "winograd_levels must be -1..3");
    if (o.preadd_mode < 0 || o.preadd_mode > 2)
        return fail(FF_EINVAL, "preadd_mode must be 0, 1 or 2");
    if (o.digit_pairing != 0 && o.digit_pairing != 1)
        return fail(FF_EINVAL, "digit_pairing must be 0 or 1");
    if (o.digit_pairing) {
        // sums of two digits must fit int8: 7-bit digits, on the INT8 path,
        // without Winograd levels
        if (o.path == FF_PATH_FP64)
            return fail(FF_EUNSUPPORTED, "digit pairing is an INT8-path option");
        if (o.digit_bits == 8)
            return fail(FF_EUNSUPPORTED, "digit pairing needs 7-bit digits");
        if (o.winograd_levels > 0)
            return fail(FF_EUNSUPPORTED, "digit pairing runs plain products only");
    }

    const Range base{-(int64_t)(p / 2), (int64_t)((p - 1) / 2)};

    // Winograd levels: requested or from the crossover orders, for the
    // path this call takes and its digit count without Winograd.
    int L = o.digit_pairing ? 0 : o.winograd_levels;
    const int64_t dmin = std::min({m, n, k});
    int path = o.path == FF_PATH_AUTO ? FF_PATH_INT8 : o.path;
    if (L < 0) {
        int s0 = 0;
        if (path == FF_PATH_INT8)
            for (int bits : {7, 8})
                if (!o.digit_bits || bits == o.digit_bits) {
                    const int s = slices_for(base, bits);
                    if (s && (!s0 || s < s0)) s0 = s;
                }
        const Crossover w = crossover(path, s0, p);
        L = 0;
        if (dmin >= w.first) {
            L = 1;
            for (int64_t x = dmin / 2; x >= w.next && L < 3; x /= 2) ++L;
        }
    }
    // Every leaf dimension must keep at least 16 entries.
    while (L > 0 && (dmin >> L) < 16) --L;
    P.levels = L;
    P.me = m - (m % (int64_t(1) << L));
    P.ne = n - (n % (int64_t(1) << L));
    P.ke = k - (k % (int64_t(1) << L));

    // Leaf operand range, unreduced (delayed) and reduced pre-additions.
    Range wid_d, wid_r = base;
    int64_t mp_d, mp_r = mag(base) * mag(base);
    leaf_bounds(base, L, &wid_d, &mp_d);
    const bool delayed_fits = wid_d.lo >= -I32MAX && wid_d.hi <= I32MAX;

    // Path.
    P.path = path;
    const int64_t carry = (int64_t)p + 2;

    if (path == FF_PATH_FP64) {
        int64_t kb_d = delayed_fits ? (TWO53 - carry) / mp_d : 0;
        int64_t kb_r = (TWO53 - carry) / mp_r;
        bool reduce = L > 0 && kb_r > kb_d && kb_d < (P.ke >> L);
        if (o.preadd_mode == 1) reduce = false;
        if (o.preadd_mode == 2) reduce = L > 0;
        if (!reduce && !delayed_fits)
            return fail(FF_EUNSUPPORTED, "delayed pre-additions overflow 32 bits for this p");
        int64_t kb = reduce ? kb_r : kb_d;
        if (kb < 4)
            return fail(FF_EUNSUPPORTED,
                        "FP64 path: fewer than 4 products fit below 2^53 for this p");
        P.preadds_reduced = reduce;
        P.lo = reduce ? wid_r.lo : wid_d.lo;
        P.hi = reduce ? wid_r.hi : wid_d.hi;
        P.max_prod = reduce ? mp_r : mp_d;
        P.kblock = kb;
        P.tile = choose_f64_tile(P.me >> L, P.ne >> L, ipow7(L));
    } else {
        int best_s = 0, best_bits = 0, best_reduce = 0;
        for (int reduce = 0; reduce <= (L > 0 ? 1 : 0); ++reduce) {
            if (!reduce && !delayed_fits) continue;
            if (o.preadd_mode == 1 && reduce) continue;
            if (o.preadd_mode == 2 && !reduce && L > 0) continue;
            Range r = reduce ? wid_r : wid_d;
            for (int bits : {7, 8}) {
                if (o.digit_bits && bits != o.digit_bits) continue;
                if (o.digit_pairing && bits != 7) continue;
                int s = slices_for(r, bits);
                if (s == 0) continue;
                // fewer slices wins; ties keep the delayed (unreduced) form and
                // 7-bit digits
                if (best_s == 0 || s < best_s) {
                    best_s = s; best_bits = bits; best_reduce = reduce;
                }
            }
        }
        if (best_s == 0)
            return fail(FF_EUNSUPPORTED, "INT8 path: operand range needs more than 5 digits");
        Range r = best_reduce ? wid_r : wid_d;
        P.preadds_reduced = best_reduce;
        P.bits = best_bits;
        P.slices = best_s;
        P.lo = r.lo;
        P.hi = r.hi;
        P.max_prod = best_reduce ? mp_r : mp_d;
        const int64_t d = digit_mag(r, best_bits, best_s);
        P.kblock = I32MAX / ((int64_t)best_s * d * d);
        P.tile = choose_i8_tile(best_s, P.me >> L, P.ne >> L, P.ke >> L, o);
        if (o.digit_pairing && best_s >= 2) {
            // accumulators: products of one digit pair (|.| <= d^2 each) and
            // sums over the pairs of one weight of products of digit sums
            // (|.| <= (2d)^2 each)
            P.pairing = 1;
            P.tile = -1;
            const int64_t q = (int64_t)pairing_max_pairs(best_s) * 4 * d * d;
            P.kblock = std::min(I32MAX / (d * d), I32MAX / q);
        }
    }

    // Workspace.
    const int64_t ml = P.me >> L, nl = P.ne >> L, kl = P.ke >> L;
    const int64_t nleaf = ipow7(L);
    int64_t ws = 0;
    if (P.path == FF_PATH_INT8 && P.pairing) {
        const int64_t kpass = std::min<int64_t>(kl, P.kblock);
        const int64_t KP = round_up(std::max<int64_t>(kpass, 1), I8_BK);
        const int64_t mp = round_up(std::max<int64_t>(ml, 1), i8p_bm(P.slices));
        const int64_t np = round_up(std::max<int64_t>(nl, 1), i8p_bn(P.slices));
        ws += (int64_t)P.slices * (P.slices + 1) / 2 * (mp + np) * KP;
    } else if (P.path == FF_PATH_INT8) {
        const I8Tile &t = i8_tile(P.tile);
        const int64_t kpass = std::min<int64_t>(kl, P.kblock);
        const int64_t KP = round_up(std::max<int64_t>(kpass, 1), I8_BK);
        const int64_t mp = round_up(std::max<int64_t>(ml, 1), t.bm());
        const int64_t np = round_up(std::max<int64_t>(nl, 1), t.bn());
        ws += nleaf * P.slices * (mp + np) * KP;
        if (L > 0) ws += wino_buffers(ml, nl, kl, L, kpass == kl);
    } else {
        // packed double operands of every leaf
        const F64Tile &t = f64_tile(P.tile);
        const int64_t KP = round_up(std::max<int64_t>(kl, 1), F64_BK);
        const int64_t mp = round_up(std::max<int64_t>(ml, 1), t.bm());
        const int64_t np = round_up(std::max<int64_t>(nl, 1), t.bn());
        ws += nleaf * (mp + np) * KP * 8;
        if (L > 0) {
            ws += wino_buffers(ml, nl, kl, L, true);
        } else if (f64_small(m, n, k)) {
            P.small = 1;
            ws = 0; // residues are read in place
        } else {
            int kts = 0;
            const int ns = f64_splits((mp / t.bm()) * (np / t.bn()), KP / F64_BK, &kts);
            if (ns > 1) ws += 256 + (int64_t)ns * ml * nl * 4; // split partials
        }
    }
    if (L > 0) ws += nleaf * 256 + 4096; // job tables
    P.ws_bytes = ws;
    *pl = P;
    return FF_OK;
}

} // namespace ff
