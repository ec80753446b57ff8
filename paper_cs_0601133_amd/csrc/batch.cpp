// Batched launches: many independent fgemm jobs (own modulus, sizes and
// pointers each) run as one digit-slicing launch plus one persistent GEMM
// launch that drains a shared tile queue, heaviest jobs first.  This is the
// shape of the multi-modular workload the paper points to for large moduli
// and for integer problems (Chinese remaindering, Sections 1 and 7), and it
// also carries the 7^l leaf products of Winograd's algorithm.
//
// The batch is described once on the host (job tables, workspace layout)
// and can then be enqueued on a stream, or captured into a HIP graph bound
// to its pointers and replayed.
#include <algorithm>
#include <cstring>
#include <vector>

#include "ff_batch.h"
#include "ff_profile.h"

namespace ff {

namespace {

int64_t align256(int64_t x) { return (x + 255) & ~int64_t(255); }

} // namespace

int prep_batch(const std::vector<IJob> &jobs, int path, int tile, BatchPrep *out)
{
    BatchPrep B;
    B.path = path;
    B.tile = tile;
    int64_t planes = 0;
    std::vector<IJob> work;
    for (const IJob &j : jobs) {
        if (j.m == 0 || j.n == 0) continue;
        if (j.k == 0 || j.alpha == 0) {
            if (j.beta != 1) B.scales.push_back(j);
            continue;
        }
        if (path == FF_PATH_INT8 && j.k > j.kblock) {
            B.singles.push_back(j);
            continue;
        }
        work.push_back(j);
    }
    if (path == FF_PATH_INT8) {
        const I8Tile &t = i8_tile(tile);
        // heaviest tiles first: cost of one tile ~ KP * s^2
        std::stable_sort(work.begin(), work.end(), [](const IJob &a, const IJob &b) {
            return a.k * a.S * a.S > b.k * b.S * b.S;
        });
        int blocks = 0, tiles = 0;
        for (const IJob &j : work) {
            if (j.S > t.S) return fail(FF_EINVAL, "batch job needs more digits than the tile");
            const int KP = (int)round_up(j.k, I8_BK);
            const int mp = (int)round_up(j.m, t.bm()), np = (int)round_up(j.n, t.bn());
            const int64_t a_off = planes;
            planes = align256(planes + (int64_t)j.S * mp * KP);
            const int64_t b_off = planes;
            planes = align256(planes + (int64_t)j.S * np * KP);
            // planes are relative offsets until the workspace is known
            SliceJob sa = slice_job(j.A, j.lda, (int)j.m, (int)j.k, j.ta, j.in_mode, j.p, j.S,
                                    j.bits, (int8_t *)(intptr_t)a_off, t.bm(), KP);
            SliceJob sb = slice_job(j.B, j.ldb, (int)j.n, (int)j.k, j.tb ? 0 : 1, j.in_mode, j.p,
                                    j.S, j.bits, (int8_t *)(intptr_t)b_off, t.bn(), KP);
            sa.block_start = blocks;
            blocks += slice_blocks(sa);
            sb.block_start = blocks;
            blocks += slice_blocks(sb);
            B.sj.push_back(sa);
            B.sj.push_back(sb);
            I8Job J;
            std::memset(&J, 0, sizeof(J));
            J.Ad = (const int8_t *)(intptr_t)a_off;
            J.Bd = (const int8_t *)(intptr_t)b_off;
            J.a_plane = sa.plane;
            J.b_plane = sb.plane;
            J.C = j.C;
            J.ldc = j.ldc;
            J.m = (int)j.m;
            J.n = (int)j.n;
            J.KP = KP;
            J.s = j.S;
            J.p = j.p;
            J.beta = j.beta;
            J.pd = (double)j.p;
            J.pinv = 1.0 / (double)j.p;
            i8_weights(J, j.alpha, j.bits);
            J.gm = t.GM;
            J.tiles_m = mp / t.bm();
            J.tiles_n = np / t.bn();
            J.tile_start = tiles;
            tiles += J.tiles_m * J.tiles_n;
            B.ij.push_back(J);
        }
        B.slice_blocks = blocks;
        B.i8_tiles = tiles;
        B.uniform_s = !work.empty();
        for (const IJob &j : work) B.uniform_s = B.uniform_s && j.S == t.S;
    } else {
        const F64Tile &t = f64_tile(tile);
        // jobs reduced per stage before jobs reduced after every step (two
        // launches), heaviest tiles first within each group
        auto fine = [](const IJob &j) { return j.kblock < F64_BK; };
        std::stable_sort(work.begin(), work.end(), [&](const IJob &a, const IJob &b) {
            if (fine(a) != fine(b)) return !fine(a);
            return a.k > b.k;
        });
        int blocks = 0, tiles = 0;
        B.fj_fine = (int)work.size();
        for (const IJob &j : work) {
            if (fine(j) && B.fj_fine == (int)work.size()) {
                B.fj_fine = (int)B.fj.size();
                B.f64_tiles[0] = tiles;
                tiles = 0;
            }
            const int KP = (int)round_up(j.k, F64_BK);
            const int64_t mp = round_up(j.m, t.bm()), np = round_up(j.n, t.bn());
            const int64_t a_off = planes;
            planes = align256(planes + mp * KP * 8);
            const int64_t b_off = planes;
            planes = align256(planes + np * KP * 8);
            // packed operands are relative offsets until the workspace is known
            SliceJob sa = pack_job(j.A, j.lda, (int)j.m, (int)j.k, j.ta, j.in_mode, j.p,
                                   (double *)(intptr_t)a_off, t.bm(), KP);
            SliceJob sb = pack_job(j.B, j.ldb, (int)j.n, (int)j.k, j.tb ? 0 : 1, j.in_mode, j.p,
                                   (double *)(intptr_t)b_off, t.bn(), KP);
            sa.block_start = blocks;
            blocks += pack_blocks(sa);
            sb.block_start = blocks;
            blocks += pack_blocks(sb);
            B.sj.push_back(sa);
            B.sj.push_back(sb);
            F64Job J = f64_job((const double *)(intptr_t)a_off, (const double *)(intptr_t)b_off,
                               j.C, j.ldc, j.m, j.n, KP, j.p, j.alpha, j.beta, j.kblock, tile);
            J.tile_start = tiles;
            tiles += J.tiles_m * J.tiles_n;
            B.fj.push_back(J);
        }
        B.slice_blocks = blocks;
        B.f64_tiles[B.fj_fine < (int)B.fj.size() ? 1 : 0] = tiles;
    }
    // workspace layout: tables, then digit planes
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
    *out = std::move(B);
    return FF_OK;
}

// Rebases plane offsets on the workspace and serialises the tables.
static void bind_tables(BatchPrep &B, char *ws)
{
    B.staging.assign(B.table_bytes, 0);
    char *planes = ws + B.off_planes;
    std::vector<SliceJob> sj = B.sj;
    for (auto &s : sj) s.D = (int8_t *)(planes + (intptr_t)s.D);
    std::vector<I8Job> ij = B.ij;
    for (auto &J : ij) {
        J.Ad = (const int8_t *)(planes + (intptr_t)J.Ad);
        J.Bd = (const int8_t *)(planes + (intptr_t)J.Bd);
    }
    std::vector<F64Job> fj = B.fj;
    for (auto &J : fj) {
        J.Ad = (const double *)(planes + (intptr_t)J.Ad);
        J.Bd = (const double *)(planes + (intptr_t)J.Bd);
    }
    if (!sj.empty()) std::memcpy(B.staging.data() + B.off_sj, sj.data(), sj.size() * sizeof(SliceJob));
    if (!ij.empty()) std::memcpy(B.staging.data() + B.off_ij, ij.data(), ij.size() * sizeof(I8Job));
    if (!fj.empty()) std::memcpy(B.staging.data() + B.off_fj, fj.data(), fj.size() * sizeof(F64Job));
    B.bound_ws = ws;
}

int upload_batch(BatchPrep &B, char *ws, hipStream_t st, bool sync)
{
    bind_tables(B, ws);
    if (B.table_bytes == 0) return FF_OK;
    if (sync) {
        FF_HIP_CHECK(hipMemcpy(ws, B.staging.data(), B.table_bytes, hipMemcpyHostToDevice));
    } else {
        int rc = upload_async(st, B.staging.data(), (size_t)B.table_bytes, ws);
        if (rc) return rc;
    }
    return FF_OK;
}

int launch_batch(BatchPrep &B, unsigned *ctr, hipStream_t st, int persistent, bool slice)
{
    char *ws = B.bound_ws;
    for (const IJob &j : B.scales)
        FF_HIP_CHECK(launch_scale(j.C, j.ldc, j.m, j.n, j.p, j.beta, st));
    if (B.path == FF_PATH_INT8 && !B.ij.empty()) {
        if (slice)
            FF_HIP_CHECK(FF_TIMED(PROF_SLICE, st,
                                  launch_slice_batched((const SliceJob *)(ws + B.off_sj),
                                                       (int)B.sj.size(), B.slice_blocks, st)));
        FF_HIP_CHECK(FF_TIMED(PROF_GEMM, st,
                              launch_i8_batched(B.tile, (const I8Job *)(ws + B.off_ij),
                                                (int)B.ij.size(), B.i8_tiles, persistent, ctr,
                                                st, B.uniform_s)));
    }
    if (B.path == FF_PATH_FP64 && !B.fj.empty()) {
        if (slice)
            FF_HIP_CHECK(FF_TIMED(PROF_SLICE, st,
                                  launch_pack_f64_batched((const SliceJob *)(ws + B.off_sj),
                                                          (int)B.sj.size(), B.slice_blocks, st)));
        const F64Job *tab = (const F64Job *)(ws + B.off_fj);
        const int nf = (int)B.fj.size() - B.fj_fine;
        if (B.fj_fine > 0)
            FF_HIP_CHECK(FF_TIMED(PROF_GEMM, st,
                                  launch_f64_batched(B.tile, tab, B.fj_fine, B.f64_tiles[0],
                                                     persistent, ctr, 0, st)));
        if (nf > 0)
            FF_HIP_CHECK(FF_TIMED(PROF_GEMM, st,
                                  launch_f64_batched(B.tile, tab + B.fj_fine, nf, B.f64_tiles[1],
                                                     persistent, ctr, 1, st)));
    }
    return FF_OK;
}

// ff_job -> internal job with its own (Winograd-free) plan.
int job_from_abi(const ff_job &a, const ff_opts &o, IJob *out)
{
    int rc = check_args(a.p, a.transA, a.transB, a.m, a.n, a.k, a.A, a.lda, a.B, a.ldb, a.C,
                        a.ldc);
    if (rc) return rc;
    IJob j;
    j.p = a.p; j.ta = a.transA; j.tb = a.transB;
    j.m = a.m; j.n = a.n; j.k = a.k;
    j.alpha = a.alpha % a.p; j.beta = a.beta % a.p;
    j.A = a.A; j.lda = a.lda; j.B = a.B; j.ldb = a.ldb; j.C = a.C; j.ldc = a.ldc;
    j.in_mode = IN_RESIDUE;
    if (j.m == 0 || j.n == 0 || j.k == 0 || j.alpha == 0) {
        j.path = o.path == FF_PATH_FP64 ? FF_PATH_FP64 : FF_PATH_INT8;
        *out = j;
        return FF_OK;
    }
    ff_opts po = o;
    po.winograd_levels = 0;
    po.digit_pairing = 0; // batches use the regular digit kernel
    Plan P;
    if ((rc = make_plan(a.p, a.m, a.n, a.k, po, &P))) return rc;
    j.path = P.path;
    j.S = P.slices;
    j.bits = P.bits;
    j.kblock = P.kblock;
    *out = j;
    return FF_OK;
}

int run_single_job(const IJob &j, const ff_opts &o, hipStream_t st)
{
    ff_opts so = o;
    so.winograd_levels = 0;
    so.stream = (void *)st;
    so.validate = 0;
    return ff_fgemm_ex(j.p, j.ta, j.tb, j.m, j.n, j.k, j.alpha, (const uint32_t *)j.A, j.lda,
                       (const uint32_t *)j.B, j.ldb, j.beta, j.C, j.ldc, &so);
}

int prep_abi_batch(const ff_job *jobs, int njobs, const ff_opts &o, BatchPrep *B)
{
    if (njobs < 0 || (njobs > 0 && !jobs)) return fail(FF_EINVAL, "bad job list");
    std::vector<IJob> v;
    v.reserve(njobs);
    int path = o.path == FF_PATH_FP64 ? FF_PATH_FP64 : FF_PATH_INT8;
    int Smax = 1;
    int64_t big_m = 1, big_n = 1, big_k = 1;
    for (int i = 0; i < njobs; ++i) {
        IJob j;
        int rc = job_from_abi(jobs[i], o, &j);
        if (rc) return fail(rc, "job " + std::to_string(i) + ": " + ff_last_error());
        Smax = std::max(Smax, j.S);
        if (j.m * j.n * j.k > big_m * big_n * big_k) { big_m = j.m; big_n = j.n; big_k = j.k; }
        v.push_back(j);
    }
    int tile;
    if (path == FF_PATH_INT8) {
        tile = tuned_i8_tile(Smax, big_m, big_n, big_k);
        if (tile < 0) tile = i8_default_tile(Smax);
    } else {
        tile = choose_f64_tile();
    }
    return prep_batch(v, path, tile, B);
}

// ---------------------------------------------------------------------------
// HIP graph of a batch
// ---------------------------------------------------------------------------
struct BatchGraph {
    BatchPrep prep;
    char *ws = nullptr;
    unsigned *ctr = nullptr;
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

} // namespace ff

using namespace ff;

extern "C" {

int ff_fgemm_batched(const ff_job *jobs, int njobs, const ff_opts *opts)
{
    ff_opts o = opts ? *opts : default_opts();
    if (njobs == 0) return FF_OK;
    int rc = check_device();
    if (rc) return rc;
    BatchPrep B;
    if ((rc = prep_abi_batch(jobs, njobs, o, &B))) return rc;
    hipStream_t st = stream_of(&o);
    void *ws = nullptr;
    unsigned *ctr = nullptr;
    if ((rc = workspace(st, (size_t)std::max<int64_t>(B.ws_bytes, 256), &ws))) return rc;
    if ((rc = counter_buffer(st, &ctr))) return rc;
    if ((rc = upload_batch(B, (char *)ws, st, false))) return rc;
    if ((rc = launch_batch(B, ctr, st, 1))) return rc;
    for (const IJob &j : B.singles)
        if ((rc = run_single_job(j, o, st))) return rc;
    return FF_OK;
}

int ff_batch_graph_create(const ff_job *jobs, int njobs, const ff_opts *opts, void **graph)
{
    if (!graph) return fail(FF_EINVAL, "graph is null");
    ff_opts o = opts ? *opts : default_opts();
    int rc = check_device();
    if (rc) return rc;
    BatchGraph *g = new BatchGraph();
    auto cleanup = [&](int status) {
        if (g->exec) (void)hipGraphExecDestroy(g->exec);
        if (g->graph) (void)hipGraphDestroy(g->graph);
        if (g->cap) (void)hipStreamDestroy(g->cap);
        if (g->ws) (void)hipFree(g->ws);
        if (g->ctr) (void)hipFree(g->ctr);
        delete g;
        return status;
    };
    if ((rc = prep_abi_batch(jobs, njobs, o, &g->prep))) return cleanup(rc);
    if (!g->prep.singles.empty())
        return cleanup(fail(FF_EUNSUPPORTED, "a job exceeds the int32 K-block; "
                                             "graphs take single-pass jobs only"));
    if (hipMalloc(&g->ws, std::max<int64_t>(g->prep.ws_bytes, 256)) != hipSuccess ||
        hipMalloc(&g->ctr, 256) != hipSuccess)
        return cleanup(fail(FF_ENOMEM, "graph workspace allocation failed"));
    if (hipMemset(g->ctr, 0, 256) != hipSuccess) return cleanup(fail(FF_EHIP, "memset failed"));
    if ((rc = upload_batch(g->prep, g->ws, nullptr, true))) return cleanup(rc);
    if (hipStreamCreateWithFlags(&g->cap, hipStreamNonBlocking) != hipSuccess)
        return cleanup(fail(FF_EHIP, "stream creation failed"));
    if (hipStreamBeginCapture(g->cap, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return cleanup(fail(FF_EHIP, "begin capture failed"));
    rc = launch_batch(g->prep, g->ctr, g->cap, 1);
    hipGraph_t graph_tmp = nullptr;
    hipError_t e = hipStreamEndCapture(g->cap, &graph_tmp);
    g->graph = graph_tmp;
    if (rc) return cleanup(rc);
    if (e != hipSuccess) return cleanup(fail(FF_EHIP, std::string("end capture: ") + hipGetErrorString(e)));
    if (hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0) != hipSuccess)
        return cleanup(fail(FF_EHIP, "graph instantiation failed"));
    *graph = g;
    return FF_OK;
}

int ff_batch_graph_launch(void *graph, void *hip_stream)
{
    if (!graph) return fail(FF_EINVAL, "graph is null");
    BatchGraph *g = (BatchGraph *)graph;
    FF_HIP_CHECK(hipGraphLaunch(g->exec, (hipStream_t)hip_stream));
    return FF_OK;
}

int ff_batch_graph_destroy(void *graph)
{
    if (!graph) return fail(FF_EINVAL, "graph is null");
    BatchGraph *g = (BatchGraph *)graph;
    (void)hipDeviceSynchronize();
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    if (g->cap) (void)hipStreamDestroy(g->cap);
    if (g->ws) (void)hipFree(g->ws);
    if (g->ctr) (void)hipFree(g->ctr);
    delete g;
    return FF_OK;
}

} // extern "C"
