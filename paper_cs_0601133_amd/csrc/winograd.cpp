// Winograd's variant of Strassen's algorithm over Z/pZ (Section 3.2), l
// recursive levels on top of the FP64 or INT8 leaf products.
//
// Per level the seven products P1..P7 use the operands of Appendix A:
//   P1 = A11 B11, P2 = A12 B21, P3 = S4 B22, P4 = A22 T4, P5 = S1 T1,
//   P6 = S2 T2, P7 = S3 T3, with S1 = A21 + A22, S2 = S1 - A11,
//   S3 = A11 - A21, S4 = A12 - S2, T1 = B12 - B11, T2 = B22 - T1,
//   T3 = B22 - B12, T4 = T2 - B21,
// and the result is U1 = P1 + P2, U5 = U4 + P3, U6 = U3 - P4, U7 = U3 + P5
// with U2 = P1 + P6, U3 = U2 + P7, U4 = U2 + P5.
//
// The schedule is laid out for a GPU with memory to spare rather than the
// three-temporary order of the paper's schedule table: all pre-additions of
// a level run as one kernel, all 7^l leaf products as one batched launch,
// all post-additions of a level as one kernel.  Pre-additions are either
// kept as unreduced integers (the delayed form whose growth Theorem 3.1
// bounds; the planner sizes the leaf K-block or digit count from it) or
// reduced to centered residues, whichever makes the leaves cheaper.  Leaf
// products come back reduced, so post-additions are modular additions;
// alpha and beta are applied once at the top.  Dimensions that are not
// multiples of 2^l are peeled off at the top level: the largest such
// top-left block goes through Winograd, the leftover strips are thin
// products added afterwards (the dynamic peeling of Appendix A, done once
// for all levels).
//
// With the leaf K in one pass (always on FP64 leaves, within the int32
// block on INT8 ones), the last level of pre-additions is fused with the
// preparation of the leaves' operands: the seven combinations of each
// quadrant quadruple are sliced into digit planes (INT8) or packed as
// binary64 (FP64) in registers, straight into the leaves' operands
// (FF_WINO_FUSED=0 runs them apart).
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "ff_batch.h"
#include "ff_profile.h"

namespace ff {

bool wino_fused_enabled()
{
    const char *e = std::getenv("FF_WINO_FUSED");
    return !(e && *e == '0');
}

namespace {

int64_t align256(int64_t x) { return (x + 255) & ~int64_t(255); }

int64_t pow7(int L)
{
    int64_t r = 1;
    while (L--) r *= 7;
    return r;
}

// op(X)[r0.., c0..] as a pointer with the same leading dimension.
const uint32_t *sub(const uint32_t *X, int64_t ld, int trans, int64_t r0, int64_t c0)
{
    return trans ? X + c0 * ld + r0 : X + r0 * ld + c0;
}

// Descriptors of the fused last level, both sides, from the leaf batch's
// own slicing layout (leaf q: A planes in sj[2q], B^T planes in sj[2q+1]).
// The last level reads the residues of op(A), op(B) when L == 1, else the
// int32 blocks of level L-1: A blocks 2ml x 2kl, B blocks 2kl x 2nl, both
// row-major.
int fused_slices(const BatchPrep &bp, char *ws, int L, int transA, int transB, int64_t ml,
                 int64_t nl, int64_t kl, const uint32_t *A, int64_t lda, const uint32_t *B,
                 int64_t ldb, const void *const lastIn[2], int reduce, WinoSlice w[2])
{
    const int64_t nleaf = pow7(L);
    const int64_t njobs = bp.path == FF_PATH_INT8 ? (int64_t)bp.ij.size() : (int64_t)bp.fj.size();
    if ((int64_t)bp.sj.size() != 2 * nleaf || njobs != nleaf)
        return fail(FF_EUNSUPPORTED, "fused Winograd slicing: unexpected leaf batch");
    const intptr_t a0 = (intptr_t)bp.sj[0].D, b0 = (intptr_t)bp.sj[1].D;
    const intptr_t stride = nleaf > 1 ? (intptr_t)bp.sj[2].D - a0 : 0;
    for (int64_t q = 0; q < nleaf; ++q)
        if ((intptr_t)bp.sj[2 * q].D != a0 + q * stride ||
            (intptr_t)bp.sj[2 * q + 1].D != b0 + q * stride)
            return fail(FF_EUNSUPPORTED, "fused Winograd slicing: leaf planes not evenly spaced");
    char *planes = ws + bp.off_planes;
    for (int side = 0; side < 2; ++side) {
        WinoSlice &W = w[side];
        std::memset(&W, 0, sizeof(W));
        W.J = bp.sj[side];
        W.side = side;
        W.reduce = reduce;
        W.f64 = bp.path == FF_PATH_FP64;
        W.D = (int8_t *)(planes + (side ? b0 : a0));
        W.leaf_stride = (int64_t)stride;
        W.count = (int)(nleaf / 7);
        for (int q = 0; q < 4; ++q) {
            const int64_t qr = q >> 1, qc = q & 1;
            if (L == 1) {
                W.J.in_mode = IN_RESIDUE;
                if (side == 0) { // quadrant (qr, qc) of op(A), m x k
                    W.J.X = A; W.J.ldx = lda; W.J.trans = transA;
                    W.qoff[q] = transA ? qc * kl * lda + qr * ml : qr * ml * lda + qc * kl;
                } else { // quadrant (qr, qc) of op(B), k x n, read as B^T
                    W.J.X = B; W.J.ldx = ldb; W.J.trans = transB ? 0 : 1;
                    W.qoff[q] = transB ? qc * nl * ldb + qr * kl : qr * kl * ldb + qc * nl;
                }
                W.block_stride = 0;
            } else {
                W.J.in_mode = IN_SIGNED;
                W.J.X = lastIn[side];
                if (side == 0) {
                    W.J.ldx = 2 * kl; W.J.trans = 0;
                    W.qoff[q] = qr * ml * 2 * kl + qc * kl;
                    W.block_stride = 4 * ml * kl;
                } else {
                    W.J.ldx = 2 * nl; W.J.trans = 1;
                    W.qoff[q] = qr * kl * 2 * nl + qc * nl;
                    W.block_stride = 4 * kl * nl;
                }
            }
        }
    }
    return FF_OK;
}

} // namespace

int run_winograd(uint32_t p, int transA, int transB, int64_t m, int64_t n, int64_t k,
                 uint32_t alpha, const uint32_t *A, int64_t lda, const uint32_t *B,
                 int64_t ldb, uint32_t beta, uint32_t *C, int64_t ldc, const Plan &P,
                 const ff_opts &o, hipStream_t st)
{
    const int L = P.levels;
    const int64_t me = P.me, ne = P.ne, ke = P.ke;
    const int64_t ml = me >> L, nl = ne >> L, kl = ke >> L;
    const int64_t nleaf = pow7(L);

    // Leaf batch: 7^l products of int32 operands, possibly in several K
    // passes when an int32 pass cannot hold the whole leaf K (INT8 path).
    const int64_t kpass = P.path == FF_PATH_INT8 ? std::min<int64_t>(kl, P.kblock) : kl;
    const int npass = (int)((kl + kpass - 1) / kpass);
    const bool fused = npass == 1 && wino_fused_enabled();

    // workspace layout.  Stored levels alternate between buffers 0 and 1:
    // unfused, the last level lands in buffer 0; fused, the last stored level
    // (L - 1) lands in buffer 1, so buffer 0 is needed only from L = 3 on.
    const int64_t szA = nleaf * ml * kl * 4, szB = nleaf * kl * nl * 4, szP = nleaf * ml * nl * 4;
    const bool need0 = !fused || L >= 3;
    int64_t off = 0;
    const int64_t oA0 = off; off = align256(off + (need0 ? szA : 0));
    const int64_t oA1 = off; off = align256(off + (L > 1 ? szA : 0));
    const int64_t oB0 = off; off = align256(off + (need0 ? szB : 0));
    const int64_t oB1 = off; off = align256(off + (L > 1 ? szB : 0));
    const int64_t oP0 = off; off = align256(off + szP);
    const int64_t oP1 = off; off = align256(off + (L > 1 ? szP : 0));
    const int64_t oBatch = off;

    std::vector<IJob> leaves;
    for (int64_t q = 0; q < nleaf; ++q) {
        IJob j;
        j.p = p;
        j.m = ml; j.n = nl; j.k = std::min<int64_t>(kpass, kl);
        j.alpha = 1; j.beta = 0;
        j.lda = kl; j.ldb = nl; j.ldc = nl;
        j.in_mode = IN_SIGNED;
        j.path = P.path; j.S = P.slices; j.bits = P.bits; j.kblock = P.kblock;
        leaves.push_back(j);
    }
    BatchPrep prep;
    int rc = prep_batch(leaves, P.path, P.tile, &prep);
    if (rc) return rc;
    void *wsv = nullptr;
    if ((rc = workspace(st, (size_t)(oBatch + prep.ws_bytes), &wsv))) return rc;
    char *ws = (char *)wsv;
    unsigned *ctr = nullptr;
    if ((rc = counter_buffer(st, &ctr))) return rc;

    // Pre-additions, level by level, for both sides (fused: all but the
    // last level; src is then the last level's input).
    int32_t *Abuf[2] = {(int32_t *)(ws + oA0), (int32_t *)(ws + oA1)};
    int32_t *Bbuf[2] = {(int32_t *)(ws + oB0), (int32_t *)(ws + oB1)};
    const int32_t *leafA = nullptr, *leafB = nullptr;
    const void *lastIn[2] = {nullptr, nullptr};
    const int Lpre = fused ? L - 1 : L;
    for (int side = 0; side < 2; ++side) {
        const void *src = side ? (const void *)B : (const void *)A;
        int64_t ld = side ? ldb : lda;
        int tr = side ? transB : transA;
        int64_t rows = side ? ke : me, cols = side ? ne : ke;
        int64_t count = 1;
        int32_t **buf = side ? Bbuf : Abuf;
        for (int l = 1; l <= Lpre; ++l) {
            PreLevel J;
            std::memset(&J, 0, sizeof(J));
            J.X = src; J.ldx = ld; J.trans = l == 1 ? tr : 0; J.in_residue = l == 1;
            J.count_in = (int)count;
            rows /= 2; cols /= 2;
            J.rows = (int)rows; J.cols = (int)cols;
            J.side = side;
            // reduced form: reduce at every level (keeps int32 range for any p)
            J.reduce = P.preadds_reduced;
            J.p = p;
            // levels alternate buffers; the last stored one ends in buf[0]
            // (unfused) or buf[1] (fused), and no level writes the buffer it
            // reads
            J.Y = buf[fused ? (((Lpre - l) & 1) ^ 1) : ((L - l) & 1)];
            FF_HIP_CHECK(launch_preadd(J, st));
            src = J.Y;
            count *= 7;
        }
        (side ? leafB : leafA) = (const int32_t *)src;
        lastIn[side] = src;
    }

    // Leaf products into P0 (reduced residues, alpha = 1, beta = 0).
    uint32_t *Pbuf[2] = {(uint32_t *)(ws + oP0), (uint32_t *)(ws + oP1)};
    // Leaves go to P0; post-addition level l writes P[(L - l + 1) & 1], so
    // no level reads and writes the same buffer.
    uint32_t *leafP = Pbuf[0];
    for (int pass = 0; pass < npass; ++pass) {
        const int64_t k0 = (int64_t)pass * kpass;
        const int64_t kc = std::min<int64_t>(kpass, kl - k0);
        std::vector<IJob> js = leaves;
        for (int64_t q = 0; q < nleaf; ++q) {
            // fused: the leaves' operands exist only as digit planes
            js[q].A = fused ? nullptr : leafA + q * ml * kl + k0;
            js[q].B = fused ? nullptr : leafB + q * kl * nl + k0 * nl;
            js[q].C = leafP + q * ml * nl;
            js[q].k = kc;
            js[q].beta = pass == 0 ? 0u : 1u;
        }
        BatchPrep bp;
        if ((rc = prep_batch(js, P.path, P.tile, &bp))) return rc;
        if ((rc = upload_batch(bp, ws + oBatch, st, false))) return rc;
        if (fused) {
            WinoSlice w[2];
            if ((rc = fused_slices(bp, ws + oBatch, L, transA, transB, ml, nl, kl, A, lda, B, ldb,
                                   lastIn, P.preadds_reduced, w)))
                return rc;
            FF_HIP_CHECK(FF_TIMED(PROF_SLICE, st, launch_wino_slice(w[0], w[1], st)));
        }
        if (P.path == FF_PATH_INT8 && bp.scales.empty() && bp.singles.empty() && !bp.ij.empty()) {
            // leaves of one size: one workgroup per tile (XCD-aware order),
            // no work queue
            char *bw = bp.bound_ws;
            if (!fused)
                FF_HIP_CHECK(FF_TIMED(PROF_SLICE, st,
                                      launch_slice_batched((const SliceJob *)(bw + bp.off_sj),
                                                           (int)bp.sj.size(), bp.slice_blocks,
                                                           st)));
            FF_HIP_CHECK(FF_TIMED(PROF_GEMM, st,
                                  launch_i8_jobs(bp.tile, (const I8Job *)(bw + bp.off_ij),
                                                 (int)bp.ij.size(), bp.i8_tiles, st)));
        } else if ((rc = launch_batch(bp, ctr, st, 0, !fused))) {
            return rc;
        }
    }

    // Post-additions, level by level up to C.
    const uint32_t *src = leafP;
    int64_t count = nleaf / 7, rows = ml, cols = nl;
    const double pinv = 1.0 / (double)p;
    for (int l = L; l >= 1; --l) {
        PostLevel J;
        std::memset(&J, 0, sizeof(J));
        J.P = src;
        J.count_out = (int)count;
        J.rows = (int)rows; J.cols = (int)cols;
        J.p = p; J.alpha = alpha; J.beta = beta; J.pinv = pinv;
        if (l == 1) {
            J.Y = C; J.ldy = ldc; J.block_stride = 0; J.final_level = 1;
        } else {
            J.Y = Pbuf[(L - l + 1) & 1];
            J.ldy = 2 * cols; J.block_stride = 4 * rows * cols; J.final_level = 0;
        }
        FF_HIP_CHECK(launch_postadd(J, st));
        src = J.Y;
        count /= 7; rows *= 2; cols *= 2;
    }

    // Peeled strips (plain products, residues in place).
    ff_opts so = o;
    so.winograd_levels = 0;
    so.stream = (void *)st;
    so.validate = 0;
    if (ke < k) { // C[0:me, 0:ne] += alpha * A[0:me, ke:k] * B[ke:k, 0:ne]
        rc = ff_fgemm_ex(p, transA, transB, me, ne, k - ke, alpha, sub(A, lda, transA, 0, ke),
                         lda, sub(B, ldb, transB, ke, 0), ldb, 1, C, ldc, &so);
        if (rc) return rc;
    }
    if (ne < n) { // C[0:me, ne:n]
        rc = ff_fgemm_ex(p, transA, transB, me, n - ne, k, alpha, A, lda,
                         sub(B, ldb, transB, 0, ne), ldb, beta, C + ne, ldc, &so);
        if (rc) return rc;
    }
    if (me < m) { // C[me:m, 0:n]
        rc = ff_fgemm_ex(p, transA, transB, m - me, n, k, alpha, sub(A, lda, transA, me, 0), lda,
                         B, ldb, beta, C + me * ldc, ldc, &so);
        if (rc) return rc;
    }
    return FF_OK;
}

} // namespace ff
