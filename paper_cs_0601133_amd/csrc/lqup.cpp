// LQUP factorisation over Z/pZ (Section 5.1) and what Section 6 reads off
// it: the rank and the determinant.
//
// A = L Q U P, computed in place in the compressed form: row i keeps its
// position; with k_i pivots in the rows above it, its entries before column
// k_i are its multipliers on those pivots and the rest is U's row (pivot
// rows) or zero (dependent rows), columns in the permuted order.  Pivots are
// chosen row by row, each row on its first nonzero entry among the columns no
// pivot uses yet, exchanged into place; the factorisation is then unique.
//
// The algorithm is the row recursion the paper describes: factor the top
// half (pivots T, Y = the rest of their U rows, in the pivot rows), then for
// the bottom half [X Z] solve G T = X (the right-hand triangular solve, done
// as T^T G^T = X^T by the ftrsm driver reading X as the transposed storage
// of X^T, so G overwrites X in place), update Z <- Z - G Y with one
// fgemm, and factor Z.  Blocks of 64 rows are factored by one workgroup
// over a window of 64 columns (k_lqup_panel); the pivot rows' entries past
// the window are then finished with a unit lower triangular ftrsm and the
// panel's remaining rows with an fgemm.  When a row's window holds no pivot,
// the remaining rows of the panel are searched over all columns from the
// current rank on (k_lqup_first_nonzero): the first row with a nonzero is
// the next pivot row (a column exchange brings its entry into place), the
// rows before it are dependent.  Each panel's pivots
// decide the sizes of what follows, so the host reads them back: the call is
// synchronous.
//
// Fast path: when m <= n the factorisation first runs on the guess that
// every row is a pivot row in its own column (no dependent row, no column
// exchange), which fixes every size in advance: nothing is read back per
// panel, the pivot rows of a half are its rows in place (no gather), and
// each panel kernel records in a device flag whether the guess held for it.
// While centered products are exact in binary64 (p below about 2^26.5) a
// panel is one launch of k_lqup_panel_fast, which carries the pivot rows'
// entries past the window through its own row operations (the solve for
// them, fused; one workgroup per 64 of those columns), and nodes small
// enough (blocked_node) are factored panel by panel, each panel launch also
// solving G T = X for the node's rows below it.  For larger p each panel's
// solve for its pivot rows past the window is an ftrsm on a second stream,
// beside the right-hand solve that follows it (see Aux).
// The flag is read once at the end; if any panel saw otherwise, A is
// restored from a copy taken at the start and the factorisation runs again
// with the read-backs above.  Either way the result is the same unique
// factorisation.
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

#include "ff_runtime.h"

namespace ff {

namespace {

// A second stream and two events, borrowed per factorisation from a pool
// per device: on the fast path with the general panel kernel (large p),
// each panel's solve for its pivot rows past
// the window runs there, beside the next right-hand solve (which does not
// read those entries); the main stream waits for it before the update that
// does.  Both are latency-bound launches of a few workgroups.
struct Aux {
    hipStream_t st = nullptr;
    hipEvent_t panel = nullptr, y = nullptr;
};

std::mutex g_aux_mu;
std::map<int, std::vector<Aux>> g_aux_free;

bool aux_acquire(Aux *a)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return false;
    {
        std::lock_guard<std::mutex> lk(g_aux_mu);
        std::vector<Aux> &v = g_aux_free[dev];
        if (!v.empty()) {
            *a = v.back();
            v.pop_back();
            return true;
        }
    }
    Aux n;
    bool ok = hipStreamCreateWithFlags(&n.st, hipStreamNonBlocking) == hipSuccess;
    ok = ok && hipEventCreateWithFlags(&n.panel, hipEventDisableTiming) == hipSuccess;
    ok = ok && hipEventCreateWithFlags(&n.y, hipEventDisableTiming) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        if (n.y) (void)hipEventDestroy(n.y);
        if (n.panel) (void)hipEventDestroy(n.panel);
        if (n.st) (void)hipStreamDestroy(n.st);
        return false;
    }
    *a = n;
    return true;
}

void aux_release(const Aux &a)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return;
    std::lock_guard<std::mutex> lk(g_aux_mu);
    g_aux_free[dev].push_back(a);
}

struct Lqup {
    uint32_t p;
    int64_t m, n, lda;
    uint32_t *A;
    hipStream_t st;
    ff_opts o;              // for the inner fgemm / ftrsm calls
    int64_t k = 0;          // pivots so far
    std::vector<int64_t> piv; // pivot rows in order
    std::vector<char> dep;    // dependent rows
    std::vector<int64_t> colperm;
    bool spec = false;      // full-rank guess in force (see above)
    bool fused = false;     // its panels by k_lqup_panel_fast (p small enough)
    int64_t below = 0;      // rows after the next panel whose solve it may fold in
    bool folded = false;    // the last panel solved G T = X for those rows
    const LqupDigits *digits = nullptr; // the next panel may also write the update's digits
    bool sliced = false;    // the last panel wrote them
    int32_t *d_fail = nullptr; // set by a panel that contradicts the guess
    unsigned *ctr = nullptr;   // the stream's counter block (fused panels)
    int64_t cus = 256;         // compute units of the device
    Aux aux;                // second stream (fast path), if one was had
    bool have_aux = false;
    bool y_pending = false; // a panel's solve past its window still runs on aux.st
    // device scratch (workspace slot 2)
    uint32_t *U = nullptr;  // gathered pivot rows
    int64_t *d_rows = nullptr, *d_pairs = nullptr, *d_first = nullptr;
    int32_t *d_out = nullptr;
};

int fgemm_sub(const Lqup &c, int64_t m, int64_t n, int64_t k, const uint32_t *A, int64_t lda,
              const uint32_t *B, int64_t ldb, uint32_t *C, int64_t ldc)
{
    // C <- C - A B
    return ff_fgemm_ex(c.p, FF_NOTRANS, FF_NOTRANS, m, n, k, c.p - 1, A, lda, B, ldb, 1, C, ldc,
                       &c.o);
}

// Column exchanges (pairs of absolute columns, in order) on the rows outside
// [skip_lo, skip_hi), recorded in colperm.
int exchange(Lqup &c, const std::vector<int64_t> &pairs, int64_t skip_lo, int64_t skip_hi)
{
    if (pairs.empty()) return FF_OK;
    for (size_t j = 0; j < pairs.size(); j += 2) std::swap(c.colperm[pairs[j]], c.colperm[pairs[j + 1]]);
    int rc = upload_async(c.st, pairs.data(), pairs.size() * sizeof(int64_t), c.d_pairs);
    if (rc) return rc;
    FF_HIP_CHECK(launch_lqup_swap(c.A, c.lda, c.m, skip_lo, skip_hi, c.d_pairs,
                                  (int)(pairs.size() / 2), c.st));
    return FF_OK;
}

// The main stream waits for the last panel's solve on the second stream.
int wait_y(Lqup &c)
{
    if (!c.y_pending) return FF_OK;
    FF_HIP_CHECK(hipStreamWaitEvent(c.st, c.aux.y, 0));
    c.y_pending = false;
    return FF_OK;
}

// Fast-path panel: rows [a, b) assumed to be pivot rows in columns
// [c.k, c.k + b - a) in order; the kernel flags the guess if it fails.
int panel_guess(Lqup &c, int64_t a, int64_t b, int64_t *found)
{
    const int nr = (int)(b - a);
    const int W = (int)std::min<int64_t>(LQUP_WINDOW, c.n - c.k);
    const int whole = c.k + W == c.n;
    if (c.fused) {
        // one launch: the panel, its rows past the window and, when the
        // caller asks and the panel is 64 rows over a 64-column window, the
        // right-hand solve of the rows below it
        const int m2 = nr == W && W == LQUP_PANEL ? (int)c.below : 0;
        const int64_t nc = whole ? 0 : c.n - c.k - W;
        const bool sliced = c.digits && m2 > 0 && nc > 0;
        FF_HIP_CHECK(launch_lqup_panel_fast(c.A, c.lda, a, nr, c.k, W, nc, b, m2, c.p, c.d_fail,
                                            c.ctr, c.st, sliced ? *c.digits : LqupDigits{}));
        c.folded = m2 > 0;
        c.sliced = sliced;
    } else {
        FF_HIP_CHECK(launch_lqup_panel(c.A, c.lda, a, nr, c.k, W, whole, c.p, c.d_out, c.st,
                                       c.d_fail));
    }
    if (!c.fused && !whole && nr <= W) {
        const int64_t nc = c.n - c.k - W;
        uint32_t *T = c.A + a * c.lda + c.k;
        ff_opts o = c.o;
        if (c.have_aux) {
            FF_HIP_CHECK(hipEventRecord(c.aux.panel, c.st));
            FF_HIP_CHECK(hipStreamWaitEvent(c.aux.st, c.aux.panel, 0));
            o.stream = (void *)c.aux.st;
        }
        int rc = ff_ftrsm_ex(c.p, FF_LOWER, FF_NOTRANS, FF_UNIT, nr, nc, 1, T, c.lda,
                             c.A + a * c.lda + c.k + W, c.lda, &o);
        if (rc) return rc;
        if (c.have_aux) {
            FF_HIP_CHECK(hipEventRecord(c.aux.y, c.aux.st));
            c.y_pending = true;
        }
    }
    for (int64_t r = a; r < b; ++r) c.piv.push_back(r);
    c.k += nr;
    *found = nr;
    return FF_OK;
}

// Rows [a, b), b - a <= LQUP_PANEL; the pivots found go to *found.
int panel(Lqup &c, int64_t a, int64_t b, int64_t *found)
{
    if (c.spec) return panel_guess(c, a, b, found);
    const int64_t k_start = c.k;
    int64_t i = a;
    int32_t out[3 + 2 * LQUP_PANEL];
    int64_t first[LQUP_PANEL];
    while (i < b) {
        if (c.k == c.n) { // no column left: the other rows are dependent
            for (int64_t r = i; r < b; ++r) c.dep[r] = 1;
            break;
        }
        const int W = (int)std::min<int64_t>(LQUP_WINDOW, c.n - c.k);
        const int whole = c.k + W == c.n;
        const int nr = (int)(b - i);
        FF_HIP_CHECK(launch_lqup_panel(c.A, c.lda, i, nr, c.k, W, whole, c.p, c.d_out, c.st));
        FF_HIP_CHECK(hipMemcpyAsync(out, c.d_out, sizeof(out), hipMemcpyDeviceToHost, c.st));
        FF_HIP_CHECK(hipStreamSynchronize(c.st));
        const int t = out[0], nproc = out[1], stuck = out[2];
        std::vector<int64_t> pairs;
        for (int j = 0; j < t; ++j) {
            const int from = out[3 + LQUP_PANEL + j];
            if (from != j) {
                pairs.push_back(c.k + j);
                pairs.push_back(c.k + from);
            }
        }
        int rc = exchange(c, pairs, i, b); // the panel's own rows are done
        if (rc) return rc;
        for (int r = 0; r < nproc; ++r) {
            if (out[3 + r] >= 0) c.piv.push_back(i + r);
            else c.dep[i + r] = 1;
        }
        if (t > 0 && !whole) {
            // the pivot rows [i, i + t) past the window: U = L_pp^-1 (row),
            // L_pp the unit lower triangle of their multipliers
            const int64_t nc = c.n - c.k - W;
            uint32_t *T = c.A + i * c.lda + c.k;
            rc = ff_ftrsm_ex(c.p, FF_LOWER, FF_NOTRANS, FF_UNIT, t, nc, 1, T, c.lda,
                             c.A + i * c.lda + c.k + W, c.lda, &c.o);
            if (rc) return rc;
            if (nr - t > 0) {
                rc = fgemm_sub(c, nr - t, nc, t, c.A + (i + t) * c.lda + c.k, c.lda,
                               c.A + i * c.lda + c.k + W, c.lda,
                               c.A + (i + t) * c.lda + c.k + W, c.lda);
                if (rc) return rc;
            }
        }
        c.k += t;
        i += nproc;
        if (!stuck) continue;
        // rows [i, b) are fully reduced and row i is zero inside the window
        // from column c.k on (the rows after it may not be): the first row
        // with a nonzero entry from column c.k on is the next pivot row and
        // the rows before it are dependent
        FF_HIP_CHECK(launch_lqup_first_nonzero(c.A, c.lda, i, b - i, c.k, c.n, c.d_first, c.st));
        FF_HIP_CHECK(hipMemcpyAsync(first, c.d_first, (b - i) * sizeof(int64_t),
                                    hipMemcpyDeviceToHost, c.st));
        FF_HIP_CHECK(hipStreamSynchronize(c.st));
        int64_t j = 0;
        while (j < b - i && first[j] < 0) ++j;
        for (int64_t r = 0; r < j; ++r) c.dep[i + r] = 1;
        i += j;
        if (i < b && first[j] != c.k) {
            // bring row i's first nonzero into column c.k, in every row
            rc = exchange(c, {c.k, first[j]}, 0, 0);
            if (rc) return rc;
        }
    }
    *found = c.k - k_start;
    return FF_OK;
}

// Whether the fused fast path factors a node of s rows panel by panel
// (below): the largest nodes whose first panel launch (one workgroup per 64
// columns past its window, one per 16 rows below it) fits in one round of
// the device's CUs; past that the launch takes two rounds (n = 4096, ms per
// factorisation by node size: 128: 5.6, 512: 4.95, 2048: 4.58, 4096: 5.0).
// FF_LQUP_BLOCK (a multiple of 64 from 64 to 65536) sets the size instead.
bool blocked_node(const Lqup &c, int64_t s)
{
    const char *e = std::getenv("FF_LQUP_BLOCK");
    if (e && *e) {
        const int v = std::atoi(e);
        if (v >= LQUP_PANEL && v <= 65536 && v % LQUP_PANEL == 0) return s <= v;
    }
    const int64_t wgs = (c.n - c.k - LQUP_PANEL + 63) / 64 + (s - LQUP_PANEL + 15) / 16;
    return wgs <= c.cus;
}

// Fused fast path, rows [a, b) (a node that blocked_node accepts): the panels from
// left to right, each launch also solving G T = X for every row of the node
// below the panel (G over X, in the panel's pivot columns), then one fgemm
// for those rows past the panel's pivot columns, Z <- Z - G Y.  The same
// products as the recursion's right-hand solves and updates, without the
// solves.
int blocked(Lqup &c, int64_t a, int64_t b, int64_t *found)
{
    int64_t total = 0;
    for (int64_t i = a; i < b; i += LQUP_PANEL) {
        const int64_t e = std::min(i + LQUP_PANEL, b), k0 = c.k, m2 = b - e;
        int64_t r = 0;
        // when the update after a full panel is one plain INT8 launch, the
        // panel writes its operands' digit planes (no slicing launch)
        PreSliced ps;
        LqupDigits so;
        const int64_t past = c.n - k0 - LQUP_PANEL;
        if (e - i == LQUP_PANEL && m2 > 0 && past > 0) {
            int rc = presliced_prepare(c.p, m2, past, LQUP_PANEL, c.o, c.st, &ps);
            if (rc) return rc;
            if (ps.ok && ps.KP == LQUP_PANEL) {
                so.ad = ps.Ad;
                so.bd = ps.Bd;
                so.plane_a = ps.plane_a;
                so.plane_b = ps.plane_b;
                so.rta = ps.rta;
                so.rtb = ps.rtb;
                so.S = ps.P.slices;
                so.bits = ps.P.bits;
                c.digits = &so;
            }
        }
        c.below = m2;
        c.folded = false;
        c.sliced = false;
        int rc = panel(c, i, e, &r);
        c.below = 0;
        c.digits = nullptr;
        const bool folded = c.folded, sliced = c.sliced;
        c.folded = false;
        c.sliced = false;
        if (rc) return rc;
        total += r;
        const int64_t nc = c.n - k0;
        if (r > 0 && m2 > 0) {
            const uint32_t *U = c.A + i * c.lda + k0; // the panel's U rows (in place)
            uint32_t *X = c.A + e * c.lda + k0;
            if (!folded) {
                rc = ftrsm_run(c.p, FF_UPPER, FF_TRANS, FF_NONUNIT, r, m2, 1, U, c.lda, X, c.lda,
                               1, &c.o);
                if (rc) return rc;
            }
            if (nc > r) {
                if (sliced && folded && r == LQUP_PANEL && nc - r == past)
                    rc = presliced_run(ps, c.p, m2, nc - r, c.p - 1, 1, X + r, c.lda, c.st);
                else
                    rc = fgemm_sub(c, m2, nc - r, r, X, c.lda, U + r, c.lda, X + r, c.lda);
                if (rc) return rc;
            }
        }
    }
    *found = total;
    return FF_OK;
}

int rec(Lqup &c, int64_t a, int64_t b, int64_t *found)
{
    if (b - a <= LQUP_PANEL) return panel(c, a, b, found);
    if (c.spec && c.fused && blocked_node(c, b - a)) return blocked(c, a, b, found);
    const int64_t mid = a + round_up((b - a) / 2, LQUP_PANEL);
    const int64_t k0 = c.k;
    int64_t r1 = 0, r2 = 0;
    // a top half of one panel on the fused fast path solves G T = X for the
    // bottom half itself (at most 64 rows)
    c.below = c.spec && c.fused && mid - a == LQUP_PANEL ? b - mid : 0;
    c.folded = false;
    int rc = rec(c, a, mid, &r1);
    c.below = 0;
    const bool folded = c.folded;
    c.folded = false;
    if (rc) return rc;
    const int64_t m2 = b - mid, nc = c.n - k0;
    if (r1 > 0 && m2 > 0) {
        // T (r1 x r1 upper) and Y: the U rows of the top half's pivots (on
        // the fast path, the top half's rows themselves)
        const uint32_t *U = c.U;
        int64_t ldu = nc;
        if (c.spec) {
            U = c.A + a * c.lda + k0;
            ldu = c.lda;
        } else {
            rc = upload_async(c.st, c.piv.data() + k0, r1 * sizeof(int64_t), c.d_rows);
            if (rc) return rc;
            FF_HIP_CHECK(launch_lqup_gather(c.A, c.lda, c.d_rows, r1, k0, nc, c.U, nc, c.st));
        }
        // G T = X  <=>  T^T G^T = X^T, solved in place on X read as the
        // transposed storage of G^T
        uint32_t *X = c.A + mid * c.lda + k0;
        if (!folded) {
            rc = ftrsm_run(c.p, FF_UPPER, FF_TRANS, FF_NONUNIT, r1, m2, 1, U, ldu, X, c.lda, 1,
                           &c.o);
            if (rc) return rc;
        }
        // Y's last columns may still be in the making on the second stream
        if ((rc = wait_y(c))) return rc;
        if (nc > r1) {
            rc = fgemm_sub(c, m2, nc - r1, r1, X, c.lda, U + r1, ldu, X + r1, c.lda);
            if (rc) return rc;
        }
    }
    if ((rc = wait_y(c))) return rc;
    rc = rec(c, mid, b, &r2);
    if (rc) return rc;
    *found = r1 + r2;
    return FF_OK;
}

} // namespace

} // namespace ff

using namespace ff;

extern "C" {

int ff_flqup(uint32_t p, int64_t m, int64_t n, uint32_t *A, int64_t lda, int64_t *rank,
             int64_t *pivrows, int64_t *colperm, const ff_opts *opts)
{
    if (p < 2 || p > 0x7FFFFFFFu) return fail(FF_EINVAL, "p must be in [2, 2^31 - 1]");
    if (m < 0 || n < 0) return fail(FF_EINVAL, "negative dimension");
    if (!rank || (m > 0 && !pivrows) || (n > 0 && !colperm))
        return fail(FF_EINVAL, "null output pointer");
    if (m > 0 && n > 0 && (!A || lda < n)) return fail(FF_EINVAL, "A null or lda < n");
    if (m > 0x7FFFFFFF || n > 0x7FFFFFFF) return fail(FF_EINVAL, "dimension too large");
    for (int64_t j = 0; j < n; ++j) colperm[j] = j;
    if (m == 0 || n == 0) {
        *rank = 0;
        for (int64_t i = 0; i < m; ++i) pivrows[i] = i;
        return FF_OK;
    }
    ff_opts o = opts ? *opts : default_opts();
    int rc = check_device();
    if (rc) return rc;
    Lqup c;
    // on every return: the second stream's work is done and it goes back to
    // the pool
    struct AuxGuard {
        Lqup &c;
        ~AuxGuard()
        {
            if (!c.have_aux) return;
            (void)hipStreamSynchronize(c.aux.st);
            aux_release(c.aux);
        }
    } aux_guard{c};
    c.p = p;
    c.m = m;
    c.n = n;
    c.lda = lda;
    c.A = A;
    c.st = stream_of(&o);
    c.o = o;
    c.o.stream = (void *)c.st;
    c.o.validate = 0;
    c.dep.assign(m, 0);
    c.colperm.resize(n);
    for (int64_t j = 0; j < n; ++j) c.colperm[j] = j;
    if (o.validate) {
        unsigned *bad = nullptr;
        FF_HIP_CHECK(hipMalloc(&bad, sizeof(unsigned)));
        unsigned h = 0;
        hipError_t e = hipMemsetAsync(bad, 0, sizeof(unsigned), c.st);
        if (e == hipSuccess) e = launch_validate(A, lda, m, n, p, bad, c.st);
        if (e == hipSuccess) e = hipMemcpyAsync(&h, bad, sizeof(unsigned), hipMemcpyDeviceToHost, c.st);
        if (e == hipSuccess) e = hipStreamSynchronize(c.st);
        (void)hipFree(bad);
        if (e != hipSuccess) return fail(FF_EHIP, std::string("validate: ") + hipGetErrorString(e));
        if (h) return fail(FF_EINVAL, std::to_string(h) + " entries of A are not residues < p");
    }
    // scratch: U (r x n) for r <= min(m, n), row lists, exchange pairs,
    // panel results
    const int64_t rmax = std::min(m, n);
    const int64_t u_bytes = round_up(rmax * n * 4, 256);
    const int64_t rows_bytes = round_up(m * 8, 256), pairs_bytes = round_up(2 * std::max<int64_t>(n, 64) * 8, 256);
    const int64_t out_bytes = 1024, first_bytes = round_up(LQUP_PANEL * 8, 256);
    void *ws = nullptr;
    rc = workspace(c.st, (size_t)(u_bytes + rows_bytes + pairs_bytes + out_bytes + first_bytes),
                   &ws, 2);
    if (rc) return rc;
    char *w = (char *)ws;
    c.U = (uint32_t *)w;
    c.d_rows = (int64_t *)(w + u_bytes);
    c.d_pairs = (int64_t *)(w + u_bytes + rows_bytes);
    c.d_out = (int32_t *)(w + u_bytes + rows_bytes + pairs_bytes);
    c.d_first = (int64_t *)(w + u_bytes + rows_bytes + pairs_bytes + out_bytes);
    c.d_fail = (int32_t *)(c.d_out + 3 + 2 * LQUP_PANEL);
    int64_t found = 0;
    bool guessed = false;
    if (m <= n) {
        // fast path: keep a copy of A, clear the flag, run on the guess
        void *bk = nullptr;
        if ((rc = workspace(c.st, (size_t)(m * n * 4), &bk, 3))) return rc;
        FF_HIP_CHECK(hipMemcpy2DAsync(bk, (size_t)n * 4, A, (size_t)lda * 4, (size_t)n * 4,
                                      (size_t)m, hipMemcpyDeviceToDevice, c.st));
        FF_HIP_CHECK(launch_scale((uint32_t *)c.d_fail, 1, 1, 1, 2u, 0u, c.st));
        c.spec = true;
        c.fused = lqup_panel_fast_ok(p);
        if (c.fused) {
            if ((rc = counter_buffer(c.st, &c.ctr))) return rc;
            int dev = 0, cus = 0;
            FF_HIP_CHECK(hipGetDevice(&dev));
            FF_HIP_CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
            if (cus > 0) c.cus = cus;
        } else {
            c.have_aux = aux_acquire(&c.aux); // else everything stays on c.st
        }
        rc = rec(c, 0, m, &found);
        if (rc) return rc;
        if ((rc = wait_y(c))) return rc;
        int32_t failed = 1;
        FF_HIP_CHECK(hipMemcpyAsync(&failed, c.d_fail, sizeof(failed), hipMemcpyDeviceToHost,
                                    c.st));
        FF_HIP_CHECK(hipStreamSynchronize(c.st));
        if (failed & 2) return fail(FF_EHIP, "internal error: an LQUP panel's wait gave up");
        guessed = failed == 0;
        if (!guessed) {
            FF_HIP_CHECK(hipMemcpy2DAsync(A, (size_t)lda * 4, bk, (size_t)n * 4, (size_t)n * 4,
                                          (size_t)m, hipMemcpyDeviceToDevice, c.st));
            c.spec = false;
            c.fused = false;
            c.k = 0;
            c.piv.clear();
            c.dep.assign(m, 0);
            for (int64_t j = 0; j < n; ++j) c.colperm[j] = j;
        }
    }
    if (!guessed) {
        rc = rec(c, 0, m, &found);
        if (rc) return rc;
    }
    FF_HIP_CHECK(hipStreamSynchronize(c.st));
    *rank = c.k;
    int64_t d = 0;
    for (int64_t v : c.piv) pivrows[d++] = v;
    for (int64_t i = 0; i < m; ++i)
        if (c.dep[i]) pivrows[d++] = i;
    if (d != m) return fail(FF_EHIP, "internal error: rows not all classified");
    for (int64_t j = 0; j < n; ++j) colperm[j] = c.colperm[j];
    return FF_OK;
}

int ff_frank(uint32_t p, int64_t m, int64_t n, uint32_t *A, int64_t lda, int64_t *rank,
             const ff_opts *opts)
{
    if (m < 0 || n < 0) return fail(FF_EINVAL, "negative dimension");
    std::vector<int64_t> piv(std::max<int64_t>(m, 1)), perm(std::max<int64_t>(n, 1));
    return ff_flqup(p, m, n, A, lda, rank, piv.data(), perm.data(), opts);
}

int ff_fdet(uint32_t p, int64_t n, uint32_t *A, int64_t lda, uint32_t *det, const ff_opts *opts)
{
    if (!det) return fail(FF_EINVAL, "null output pointer");
    if (n < 0) return fail(FF_EINVAL, "negative dimension");
    if (n == 0) {
        *det = 1 % p;
        return FF_OK;
    }
    std::vector<int64_t> piv(n), perm(n);
    int64_t r = 0;
    int rc = ff_flqup(p, n, n, A, lda, &r, piv.data(), perm.data(), opts);
    if (rc) return rc;
    if (r < n) {
        *det = 0;
        return FF_OK;
    }
    // every row is a pivot row, in order: det = sign(colperm) prod A[k][k]
    ff_opts o = opts ? *opts : default_opts();
    hipStream_t st = stream_of(&o);
    std::vector<uint32_t> diag(n);
    FF_HIP_CHECK(hipMemcpy2DAsync(diag.data(), 4, A, (size_t)(lda + 1) * 4, 4, (size_t)n,
                                  hipMemcpyDeviceToHost, st));
    FF_HIP_CHECK(hipStreamSynchronize(st));
    uint64_t d = 1;
    for (int64_t k = 0; k < n; ++k) d = d * diag[k] % p;
    std::vector<char> seen(n, 0);
    int sign = 1;
    for (int64_t s = 0; s < n; ++s) {
        if (seen[s]) continue;
        int64_t len = 0;
        for (int64_t j = s; !seen[j]; j = perm[j]) {
            seen[j] = 1;
            ++len;
        }
        if (len % 2 == 0) sign = -sign;
    }
    *det = (uint32_t)(sign > 0 ? d : (p - d) % p);
    return FF_OK;
}

// A^-1 over Z/pZ (Section 6 builds the inverse on LQUP).  With full rank
// every row is a pivot row, in order, so A P = L U with (A P)[:, j] =
// A[:, colperm[j]], and A^-1 = P U^-1 L^-1: solve L Y = I (unit lower
// triangle of the compressed form), then U Z = Y (its upper triangle), and
// row colperm[j] of A^-1 is row j of Z.
int ff_finv(uint32_t p, int64_t n, uint32_t *A, int64_t lda, uint32_t *X, int64_t ldx,
            int *invertible, const ff_opts *opts)
{
    if (!invertible) return fail(FF_EINVAL, "null output pointer");
    if (n < 0) return fail(FF_EINVAL, "negative dimension");
    if (n > 65535) return fail(FF_EINVAL, "n exceeds 65535");
    if (n > 0 && (!X || ldx < n)) return fail(FF_EINVAL, "X null or ldx < n");
    *invertible = 0;
    if (n == 0) {
        *invertible = 1;
        return FF_OK;
    }
    std::vector<int64_t> piv(n), perm(n);
    int64_t r = 0;
    int rc = ff_flqup(p, n, n, A, lda, &r, piv.data(), perm.data(), opts);
    if (rc) return rc;
    if (r < n) return FF_OK;
    ff_opts o = opts ? *opts : default_opts();
    hipStream_t st = stream_of(&o);
    o.stream = (void *)st;
    o.validate = 0;
    // Z (n x n) and, for each row of A^-1, the row of Z it takes; the
    // factorisation is finished with this stream's slot-2 buffer
    const int64_t z_bytes = round_up(n * n * 4, 256);
    void *ws = nullptr;
    if ((rc = workspace(st, (size_t)(z_bytes + n * 8), &ws, 2))) return rc;
    uint32_t *Z = (uint32_t *)ws;
    int64_t *d_src = (int64_t *)((char *)ws + z_bytes);
    std::vector<int64_t> src(n);
    for (int64_t j = 0; j < n; ++j) src[perm[j]] = j;
    FF_HIP_CHECK(launch_lqup_identity(Z, n, st));
    FF_HIP_CHECK(hipMemcpyAsync(d_src, src.data(), (size_t)n * 8, hipMemcpyHostToDevice, st));
    if ((rc = ff_ftrsm_ex(p, FF_LOWER, FF_NOTRANS, FF_UNIT, n, n, 1, A, lda, Z, n, &o))) return rc;
    if ((rc = ff_ftrsm_ex(p, FF_UPPER, FF_NOTRANS, FF_NONUNIT, n, n, 1, A, lda, Z, n, &o)))
        return rc;
    FF_HIP_CHECK(launch_lqup_gather(Z, n, d_src, n, 0, n, X, ldx, st));
    // src is read by the copy above: wait before it goes
    FF_HIP_CHECK(hipStreamSynchronize(st));
    *invertible = 1;
    return FF_OK;
}

} // extern "C"
