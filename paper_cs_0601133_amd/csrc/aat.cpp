// Symmetric product C <- alpha A D A^T + beta C over Z/pZ (the A x A^T of
// Section 6, with a diagonal D between the factors; D = I when no diagonal is
// given).  The result is symmetric, so only the lower triangle is computed
// and then mirrored: about half the work of the full product, the n^3
// (classical) of the paper's AAT(n) instead of 2 n^3.
//
// The paper obtains the saving by recursion on 2 x 2 blocks (two recursive
// squarings per diagonal block, one product for the off-diagonal block).
// Here the lower triangle is cut into GEMM jobs: below the diagonal, one job
// per block row of 8 workgroup tiles' height (tall enough for the tile order
// to reuse operand panels as a full product does); the diagonal blocks as
// strips of one tile's height, each up to the end of its diagonal tile.
// Every job reads the same digit planes (or packed doubles) of A and of
// A D, sliced once, and all jobs run as one persistent launch over their
// tiles, heaviest first; the upper triangle is then copied from the lower.
#include <algorithm>
#include <cstring>
#include <vector>

#include "ff_batch.h"
#include "ff_profile.h"

namespace ff {

namespace {

int64_t align256(int64_t x) { return (x + 255) & ~int64_t(255); }

} // namespace

} // namespace ff

using namespace ff;

extern "C" {

int ff_faat(uint32_t p, int64_t m, int64_t k, uint32_t alpha, const uint32_t *A, int64_t lda,
            const uint32_t *D, uint32_t beta, uint32_t *C, int64_t ldc, const ff_opts *opts)
{
    if (p < 2 || p > 0x7FFFFFFFu) return fail(FF_EINVAL, "p must be in [2, 2^31 - 1]");
    if (m < 0 || k < 0) return fail(FF_EINVAL, "negative dimension");
    if (m == 0) return FF_OK;
    if (!C || ldc < m) return fail(FF_EINVAL, "C null or ldc < m");
    if (k > 0 && (!A || lda < k)) return fail(FF_EINVAL, "A null or lda < k");
    if (m > 0x7FFFFFFF || k > 0x7FFFFFFF) return fail(FF_EINVAL, "dimension too large");
    ff_opts o = opts ? *opts : default_opts();
    int rc = check_device();
    if (rc) return rc;
    hipStream_t st = stream_of(&o);
    alpha %= p;
    beta %= p;
    if (o.validate) {
        // the same checks as fgemm: A's entries (and D's) are residues < p
        ff_opts vo = o;
        vo.stream = (void *)st;
        unsigned *bad = nullptr;
        FF_HIP_CHECK(hipMalloc(&bad, sizeof(unsigned)));
        unsigned h = 0;
        hipError_t e = hipMemsetAsync(bad, 0, sizeof(unsigned), st);
        if (e == hipSuccess && k > 0) e = launch_validate(A, lda, m, k, p, bad, st);
        if (e == hipSuccess && k > 0 && D) e = launch_validate(D, k, 1, k, p, bad, st);
        if (e == hipSuccess) e = launch_validate(C, ldc, m, m, p, bad, st);
        if (e == hipSuccess) e = hipMemcpyAsync(&h, bad, sizeof(unsigned), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        (void)hipFree(bad);
        if (e != hipSuccess) return fail(FF_EHIP, std::string("validate: ") + hipGetErrorString(e));
        if (h) return fail(FF_EINVAL, std::to_string(h) + " entries are not residues < p");
    }
    if (k == 0 || alpha == 0) {
        if (beta != 1) FF_HIP_CHECK(launch_scale(C, ldc, m, m, p, beta, st));
        FF_HIP_CHECK(launch_aat_mirror(C, ldc, m, st));
        return FF_OK;
    }
    ff_opts po = o;
    po.winograd_levels = 0;
    po.digit_pairing = 0; // the triangle's jobs use the regular digit kernel
    Plan P;
    if ((rc = make_plan(p, m, m, k, po, &P))) return rc;
    const int path = P.path;
    // one K pass per product on the INT8 path (else: block rows as separate
    // fgemm calls, each with its own K passes)
    const bool batched = path == FF_PATH_FP64 || k <= P.kblock;
    int tile, bm, bn, KP;
    if (path == FF_PATH_INT8) {
        tile = tuned_i8_tile(P.slices, m, m, k);
        if (tile < 0) tile = i8_default_tile(P.slices);
        bm = i8_tile(tile).bm();
        bn = i8_tile(tile).bn();
        KP = (int)round_up(k, I8_BK);
    } else {
        tile = choose_f64_tile(m, m);
        bm = f64_tile(tile).bm();
        bn = f64_tile(tile).bn();
        KP = (int)round_up(k, F64_BK);
    }
    const int64_t H = std::max(bm, bn); // block-row height: a multiple of both
    const int64_t nblk = (m + H - 1) / H; // block rows of the unbatched path
    // A D (or A itself): the second operand, stored m x k
    const uint32_t *Bop = A;
    int64_t ldb = lda;
    const int64_t ad_bytes = D ? align256(m * k * 4) : 0;
    int64_t planes = 0, a_off = 0, b_off = 0;
    const bool shared = !D && bm == bn; // one slicing serves both operands
    BatchPrep B;
    B.path = path;
    B.tile = tile;
    if (batched) {
        const int64_t mpa = round_up(m, bm), mpb = round_up(m, bn);
        const int64_t elt = path == FF_PATH_INT8 ? P.slices : 8; // bytes per (row, k)
        a_off = 0;
        planes = align256(mpa * KP * elt);
        b_off = shared ? a_off : planes;
        if (!shared) planes = align256(planes + mpb * KP * elt);
    }
    void *ws = nullptr;
    // workspace layout: [batch tables | planes | A D]
    if (!batched) {
        if ((rc = workspace(st, (size_t)std::max<int64_t>(ad_bytes, 256), &ws, 3))) return rc;
        uint32_t *AD = (uint32_t *)ws;
        if (D) {
            FF_HIP_CHECK(launch_aat_scale_cols(A, lda, D, m, k, p, AD, k, st));
            Bop = AD;
            ldb = k;
        }
        ff_opts so = o;
        so.stream = (void *)st;
        so.validate = 0;
        so.winograd_levels = 0;
        for (int64_t i = 0; i < nblk; ++i) {
            const int64_t r0 = i * H, rows = std::min(H, m - r0), cols = std::min(r0 + H, m);
            rc = ff_fgemm_ex(p, FF_NOTRANS, FF_TRANS, rows, cols, k, alpha, A + r0 * lda, lda,
                             Bop, ldb, beta, C + r0 * ldc, ldc, &so);
            if (rc) return rc;
        }
        FF_HIP_CHECK(launch_aat_mirror(C, ldc, m, st));
        return FF_OK;
    }
    // slicing (or packing) tasks, with plane offsets relative to the planes
    int blocks = 0;
    auto add_slice = [&](const uint32_t *X, int64_t ldx, int RT, int64_t off) {
        SliceJob s = path == FF_PATH_INT8
                         ? slice_job(X, ldx, (int)m, (int)k, 0, IN_RESIDUE, p, P.slices, P.bits,
                                     (int8_t *)(intptr_t)off, RT, KP)
                         : pack_job(X, ldx, (int)m, (int)k, 0, IN_RESIDUE, p,
                                    (double *)(intptr_t)off, RT, KP);
        s.block_start = blocks;
        blocks += path == FF_PATH_INT8 ? slice_blocks(s) : pack_blocks(s);
        B.sj.push_back(s);
        return s.plane;
    };
    // A D is written into the workspace after the planes; its address is
    // only known once the workspace is, so the second slicing task is
    // patched below
    const int64_t a_plane = add_slice(A, lda, bm, a_off);
    int64_t b_plane = a_plane;
    if (!shared) b_plane = add_slice(A, lda, bn, b_off);
    // jobs: below the diagonal, one job per block row of HB rows (tall
    // enough that the tile order reuses operand panels as a full product
    // would); the diagonal blocks as strips of H rows, each up to the end of
    // its own H x H diagonal tile (the work above the diagonal stays within
    // those tiles)
    struct Part { int64_t r0, rows, c0, cols; }; // C[r0.., c0..] of rows x cols
    std::vector<Part> parts;
    const int64_t HB = 8 * H;
    for (int64_t R = 0; R < m; R += HB) {
        const int64_t rows = std::min(HB, m - R);
        if (R > 0) parts.push_back({R, rows, 0, R});
        for (int64_t s0 = R; s0 < R + rows; s0 += H)
            parts.push_back({s0, std::min(H, m - s0), R, std::min(s0 + H, m) - R});
    }
    // heaviest first, so that the small strips fill the persistent queue's end
    std::stable_sort(parts.begin(), parts.end(),
                     [](const Part &a, const Part &b) { return a.rows * a.cols > b.rows * b.cols; });
    int tiles = 0;
    const bool fine = path == FF_PATH_FP64 && P.kblock < F64_BK;
    for (const Part &q : parts) {
        // r0 and c0 are multiples of the packing row tiles (H and HB are
        // multiples of both bm and bn), so a job's operands start r0 KP and
        // c0 KP elements into the packed planes
        const int64_t r0 = q.r0, rows = q.rows, c0 = q.c0, cols = q.cols;
        if (path == FF_PATH_INT8) {
            I8Job J;
            std::memset(&J, 0, sizeof(J));
            // rows r0.. of the packed operands start r0 KP bytes into each plane
            J.Ad = (const int8_t *)(intptr_t)(a_off + r0 * KP);
            J.Bd = (const int8_t *)(intptr_t)(b_off + c0 * KP);
            J.a_plane = a_plane;
            J.b_plane = b_plane;
            J.C = C + r0 * ldc + c0;
            J.ldc = ldc;
            J.m = (int)rows;
            J.n = (int)cols;
            J.KP = KP;
            J.s = P.slices;
            J.p = p;
            J.beta = beta;
            J.pd = (double)p;
            J.pinv = 1.0 / (double)p;
            i8_weights(J, alpha, P.bits);
            J.gm = i8_tile(tile).GM;
            J.tiles_m = (int)((rows + bm - 1) / bm);
            J.tiles_n = (int)((cols + bn - 1) / bn);
            J.tile_start = tiles;
            tiles += J.tiles_m * J.tiles_n;
            B.ij.push_back(J);
        } else {
            F64Job J = f64_job((const double *)(intptr_t)(a_off + r0 * KP * 8),
                               (const double *)(intptr_t)(b_off + c0 * KP * 8), C + r0 * ldc + c0,
                               ldc, rows, cols, KP, p, alpha, beta, P.kblock, tile);
            J.tile_start = tiles;
            tiles += J.tiles_m * J.tiles_n;
            B.fj.push_back(J);
        }
    }
    B.slice_blocks = blocks;
    if (path == FF_PATH_INT8) {
        B.i8_tiles = tiles;
    } else {
        B.fj_fine = fine ? 0 : (int)B.fj.size();
        B.f64_tiles[fine ? 1 : 0] = tiles;
    }
    int64_t off = 0;
    B.off_sj = off;
    off = align256(off + (int64_t)B.sj.size() * sizeof(SliceJob));
    B.off_ij = off;
    off = align256(off + (int64_t)B.ij.size() * sizeof(I8Job));
    B.off_fj = off;
    off = align256(off + (int64_t)B.fj.size() * sizeof(F64Job));
    B.table_bytes = off;
    B.off_planes = off;
    B.ws_bytes = off + planes;
    if ((rc = workspace(st, (size_t)(B.ws_bytes + ad_bytes + 256), &ws, 3))) return rc;
    if (D) {
        uint32_t *AD = (uint32_t *)((char *)ws + align256(B.ws_bytes));
        FF_HIP_CHECK(launch_aat_scale_cols(A, lda, D, m, k, p, AD, k, st));
        // the second operand is A D
        B.sj.back().X = AD;
        B.sj.back().ldx = k;
    }
    unsigned *ctr = nullptr;
    if ((rc = counter_buffer(st, &ctr))) return rc;
    if ((rc = upload_batch(B, (char *)ws, st, false))) return rc;
    if (path == FF_PATH_INT8) {
        // every job has the plan's digit count: the table kernel that
        // compiles only that tile body, one workgroup per tile
        char *w = (char *)ws;
        FF_HIP_CHECK(FF_TIMED(PROF_SLICE, st,
                              launch_slice_batched((const SliceJob *)(w + B.off_sj),
                                                   (int)B.sj.size(), B.slice_blocks, st)));
        FF_HIP_CHECK(FF_TIMED(PROF_GEMM, st,
                              launch_i8_jobs(tile, (const I8Job *)(w + B.off_ij),
                                             (int)B.ij.size(), B.i8_tiles, st)));
    } else if ((rc = launch_batch(B, ctr, st, 0))) {
        return rc;
    }
    FF_HIP_CHECK(launch_aat_mirror(C, ldc, m, st));
    return FF_OK;
}

} // extern "C"
