// Triangular system with matrix right-hand side over Z/pZ (Section 4):
// B <- X with op(T) X = alpha B (mod p).
//
// Normalisation (Section 4.2): with D the diagonal of op(T), T' = D^-1 op(T)
// has a unit diagonal and T' X = alpha D^-1 B involves ring operations only.
// The solve is the block recursive algorithm of Section 4.1: split the rows
// in two at a multiple of 64, solve the part the triangle allows first,
// subtract its contribution from the other part with one fgemm
// (C <- C - A X, reduced in the GEMM epilogue), solve the other part.  The
// recursion stops at leaves of at most `leaf` rows (512 unless FF_TRSM_LEAF
// says otherwise), each solved by one kernel launch: the inverses of all
// 64 x 64 diagonal blocks are formed once up front, and the leaf kernel
// walks its 64-row sub-blocks on the FP64 matrix cores (residual, then
// inverse times residual).
//
// The paper's cascades (blocks of t_del rows solved over Z by a numerical
// trsm, updates left unreduced below t_update) save reduction passes around
// CPU BLAS calls; here the reduction of an update is fused into the fgemm
// epilogue and the leaf reduces after every 64-deep product, so the
// recursion reduces at every level at no extra pass.
#include <algorithm>
#include <cstdlib>
#include <cstring>

#include "ff_profile.h"
#include "ff_runtime.h"

namespace ff {

namespace {

// Leaf size: FF_TRSM_LEAF (a multiple of 64 up to TRSM_LEAF_MAX) or 512.
int64_t trsm_leaf_rows()
{
    const char *e = std::getenv("FF_TRSM_LEAF");
    if (e && *e) {
        const int v = std::atoi(e);
        if (v >= 64 && v <= TRSM_LEAF_MAX && v % 64 == 0) return v;
    }
    return 512;
}

struct Trsm {
    uint32_t p;
    int lower; // op(T) lower triangular
    int64_t m, n;
    const uint32_t *Tn; // ldn x ldn
    int64_t ldn;
    const uint32_t *Tinv; // ldn / 64 blocks of 64 x 64
    uint32_t *B;
    int64_t ldb;
    int bt; // B stored transposed (entry (i, j) at B[j * ldb + i])
    int64_t leaf;
    int split;
    ff_opts o; // inner fgemm options (stream set, no validation)
    hipStream_t st;
};

int solve(const Trsm &c, int64_t r0, int64_t r1)
{
    const int64_t size = r1 - r0;
    if (size <= c.leaf) {
        FF_HIP_CHECK(FF_TIMED(PROF_SLICE, c.st,
                              launch_trsm_leaf(c.Tn, c.ldn, c.Tinv, c.lower, r0, (int)size, c.B,
                                               c.ldb, c.bt, c.m, c.n, c.p, c.split, c.st)));
        return FF_OK;
    }
    // split at a multiple of 64 near the middle
    const int64_t mid = r0 + round_up(size / 2, 64);
    const uint32_t minus1 = c.p - 1;
    // rows [d0, d1) of B -= T'[d0:d1, s0:s1] X[s0:s1]; with B stored
    // transposed the same update reads Bt[:, d0:d1] -= Bt[:, s0:s1] T'[d0:d1, s0:s1]^T
    auto update = [&](int64_t d0, int64_t d1, int64_t s0, int64_t s1) {
        const uint32_t *Tb = c.Tn + d0 * c.ldn + s0;
        if (c.bt)
            return ff_fgemm_ex(c.p, 0, 1, c.n, d1 - d0, s1 - s0, minus1, c.B + s0, c.ldb, Tb,
                               c.ldn, 1, c.B + d0, c.ldb, &c.o);
        return ff_fgemm_ex(c.p, 0, 0, d1 - d0, c.n, s1 - s0, minus1, Tb, c.ldn, c.B + s0 * c.ldb,
                           c.ldb, 1, c.B + d0 * c.ldb, c.ldb, &c.o);
    };
    int rc;
    if (!c.lower) {
        // upper: rows [mid, r1) first, then B[r0:mid] -= T'[r0:mid, mid:r1] X[mid:r1]
        if ((rc = solve(c, mid, r1))) return rc;
        if ((rc = update(r0, mid, mid, r1))) return rc;
        return solve(c, r0, mid);
    }
    // lower: rows [r0, mid) first, then B[mid:r1] -= T'[mid:r1, r0:mid] X[r0:mid]
    if ((rc = solve(c, r0, mid))) return rc;
    if ((rc = update(mid, r1, r0, mid))) return rc;
    return solve(c, mid, r1);
}

} // namespace

int ftrsm_run(uint32_t p, int uplo, int transT, int diag, int64_t m, int64_t n, uint32_t alpha,
              const uint32_t *T, int64_t ldt, uint32_t *B, int64_t ldb, int bt,
              const ff_opts *opts)
{
    if (p < 2 || p > 0x7FFFFFFFu) return fail(FF_EINVAL, "p must be in [2, 2^31 - 1]");
    if ((uplo != FF_UPPER && uplo != FF_LOWER) || (transT != FF_NOTRANS && transT != FF_TRANS) ||
        (diag != FF_NONUNIT && diag != FF_UNIT))
        return fail(FF_EINVAL, "uplo, transT and diag must be FF_UPPER/FF_LOWER, "
                               "FF_NOTRANS/FF_TRANS and FF_NONUNIT/FF_UNIT");
    if (m < 0 || n < 0) return fail(FF_EINVAL, "negative dimension");
    if (m == 0 || n == 0) return FF_OK;
    if (!T || !B) return fail(FF_EINVAL, "null matrix pointer");
    if (ldt < m) return fail(FF_EINVAL, "ldt < m");
    if (ldb < (bt ? m : n)) return fail(FF_EINVAL, bt ? "ldb < m" : "ldb < n");
    if (m > 0x7FFFFFFF / 2) return fail(FF_EINVAL, "m too large");
    ff_opts o = opts ? *opts : default_opts();
    int rc = check_device();
    if (rc) return rc;
    hipStream_t st = stream_of(&o);
    alpha %= p;
    if (o.validate) {
        unsigned *bad = nullptr;
        FF_HIP_CHECK(hipMalloc(&bad, sizeof(unsigned)));
        unsigned h = 0;
        hipError_t e = hipMemsetAsync(bad, 0, sizeof(unsigned), st);
        if (e == hipSuccess) e = launch_validate(B, ldb, bt ? n : m, bt ? m : n, p, bad, st);
        if (e == hipSuccess) e = hipMemcpyAsync(&h, bad, sizeof(unsigned), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        (void)hipFree(bad);
        if (e != hipSuccess) return fail(FF_EHIP, std::string("validate: ") + hipGetErrorString(e));
        if (h) return fail(FF_EINVAL, std::to_string(h) + " entries of B are not residues < p");
    }
    if (alpha == 0) { // X = 0
        FF_HIP_CHECK(launch_scale(B, ldb, bt ? n : m, bt ? m : n, p, 0, st));
        return FF_OK;
    }
    // workspace slot 1 (the inner fgemm calls use slot 0): T', the inverses
    // of its diagonal blocks, dinv, a flag
    const int64_t ldn = round_up(m, 64);
    const int64_t tn_bytes = ldn * ldn * 4, ti_bytes = ldn * 64 * 4,
                  di_bytes = round_up(m * 4, 256);
    void *wsv = nullptr;
    if ((rc = workspace(st, (size_t)(tn_bytes + ti_bytes + di_bytes + 256), &wsv, 1))) return rc;
    uint32_t *Tn = (uint32_t *)wsv;
    uint32_t *Tinv = (uint32_t *)((char *)wsv + tn_bytes);
    uint32_t *dinv = (uint32_t *)((char *)wsv + tn_bytes + ti_bytes);
    unsigned *bad = (unsigned *)((char *)wsv + tn_bytes + ti_bytes + di_bytes);
    const int lower = (uplo == FF_LOWER) ^ (transT == FF_TRANS);
    // a unit diagonal needs no inverses (dinv stays null for the kernels).
    // Systems of at most 64 rows, and B stored transposed (the LQUP
    // recursion's right-hand solves) below 1024 rows, take the inverses in
    // the pass that scales B (one launch instead of two); the others, and
    // any solve that validates (it counts the entries without an inverse),
    // take them in a pass of their own, one thread per row, and scale B
    // after (a transposed B with the inverses given takes enough workgroups
    // to keep its loads in flight: at 2048 rows the pass that inverts took
    // 50 us for 32 MB).
    const bool unit = diag == FF_UNIT;
    const bool fused = !o.validate && ((bt && m < 1024) || m <= 64);
    if (fused && (alpha != 1 || !unit))
        FF_HIP_CHECK(launch_trsm_dscale(T, ldt, unit, B, ldb, bt, m, n, p, alpha,
                                        unit ? nullptr : dinv, st));
    if (!unit && !fused) {
        if (o.validate) FF_HIP_CHECK(hipMemsetAsync(bad, 0, sizeof(unsigned), st));
        FF_HIP_CHECK(launch_trsm_dinv(T, ldt, m, p, 0, dinv, o.validate ? bad : nullptr, st));
        if (o.validate) {
            unsigned h = 0;
            FF_HIP_CHECK(hipMemcpyAsync(&h, bad, sizeof(unsigned), hipMemcpyDeviceToHost, st));
            FF_HIP_CHECK(hipStreamSynchronize(st));
            if (h)
                return fail(FF_EINVAL,
                            std::to_string(h) + " diagonal entries of T have no inverse modulo p");
        }
    }
    const uint32_t *dv = unit ? nullptr : dinv;
    // 64-term sums of centered products (|t| <= p/2, |x| <= p/2 + 2) plus a
    // residual stay exact integers in binary64 up to 2^53
    const double h = (double)(p / 2), hx = h + 2.0;
    const int split = !(64.0 * h * hx + hx <= 9007199254740992.0);
    if (m <= 64) {
        // one diagonal block: its inverse straight from op(T); the single
        // leaf reads no T'
        FF_HIP_CHECK(launch_trsm_inv_direct(T, ldt, transT == FF_TRANS, lower, m, p, split, dv,
                                            Tinv, st));
    } else {
        FF_HIP_CHECK(launch_trsm_prep(T, ldt, transT == FF_TRANS, lower, m, ldn, p, dv, Tn, st));
        FF_HIP_CHECK(launch_trsm_inv(Tn, ldn, lower, p, split, Tinv, st));
    }
    if (!fused && (alpha != 1 || !unit)) {
        if (bt)
            FF_HIP_CHECK(launch_trsm_dscale(T, ldt, unit, B, ldb, 1, m, n, p, alpha, nullptr, st,
                                            dv));
        else
            FF_HIP_CHECK(launch_trsm_scale(B, ldb, m, n, p, alpha, dv, st));
    }
    Trsm c;
    c.p = p;
    c.lower = lower;
    c.m = m;
    c.n = n;
    c.Tn = Tn;
    c.ldn = ldn;
    c.Tinv = Tinv;
    c.B = B;
    c.ldb = ldb;
    c.bt = bt;
    c.leaf = trsm_leaf_rows();
    c.split = split;
    c.o = o;
    c.o.stream = (void *)st;
    c.o.validate = 0;
    c.st = st;
    return solve(c, 0, m);
}

} // namespace ff

using namespace ff;

extern "C" {

int ff_ftrsm_ex(uint32_t p, int uplo, int transT, int diag, int64_t m, int64_t n,
                uint32_t alpha, const uint32_t *T, int64_t ldt, uint32_t *B, int64_t ldb,
                const ff_opts *opts)
{
    return ftrsm_run(p, uplo, transT, diag, m, n, alpha, T, ldt, B, ldb, 0, opts);
}

int ff_ftrsm(uint32_t p, int uplo, int transT, int diag, int64_t m, int64_t n, uint32_t alpha,
             const uint32_t *T, int64_t ldt, uint32_t *B, int64_t ldb)
{
    return ff_ftrsm_ex(p, uplo, transT, diag, m, n, alpha, T, ldt, B, ldb, nullptr);
}

} // extern "C"
