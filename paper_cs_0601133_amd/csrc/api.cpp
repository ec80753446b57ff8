// C ABI entry points: argument checks, quick returns, workspace, dispatch to
// the FP64 or INT8 path (with or without Winograd levels).
#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "ff_internal.h"
#include "ff_profile.h"
#include "ff_runtime.h"

namespace ff {

namespace {
thread_local std::string g_err;
thread_local hipStream_t g_stream = nullptr;
} // namespace

void set_error(const std::string &msg) { g_err = msg; }
int fail(int status, const std::string &msg)
{
    g_err = msg;
    return status;
}

// ---------------------------------------------------------------------------
// Per-device state
// ---------------------------------------------------------------------------
namespace {

struct Buffer {
    void *ptr = nullptr;
    size_t bytes = 0;
};

struct DevState {
    std::mutex mu;
    bool checked = false;
    bool ok = false;
    std::string arch;
    std::map<std::pair<hipStream_t, int>, Buffer> ws; // (stream, slot)
    std::map<hipStream_t, unsigned *> ctr;
    struct Staging {
        void *host = nullptr; // pinned
        size_t bytes = 0;
        hipEvent_t done = nullptr; // recorded after the last copy out of it
        bool pending = false;
    };
    std::map<hipStream_t, Staging> stage;
};

std::mutex g_mu;
std::map<int, DevState *> g_devs;

} // namespace


int check_device()
{
    int dev = 0;
    FF_HIP_CHECK(hipGetDevice(&dev));
    DevState *ds;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_devs.find(dev);
        if (it == g_devs.end()) it = g_devs.emplace(dev, new DevState()).first;
        ds = it->second;
    }
    std::lock_guard<std::mutex> lk(ds->mu);
    if (!ds->checked) {
        hipDeviceProp_t prop;
        FF_HIP_CHECK(hipGetDeviceProperties(&prop, dev));
        ds->arch = prop.gcnArchName;
        ds->ok = ds->arch.rfind("gfx950", 0) == 0;
        ds->checked = true;
    }
    if (!ds->ok)
        return fail(FF_EUNSUPPORTED, "device " + std::to_string(dev) + " is " + ds->arch +
                                         "; this library is built for gfx950 only");
    return FF_OK;
}

// Grow-only workspace per (device, stream).  Calls on one stream run in
// order, so reusing its workspace is safe; before a buffer is replaced the
// stream is drained.
int workspace(hipStream_t st, size_t bytes, void **out, int slot)
{
    int dev = 0;
    FF_HIP_CHECK(hipGetDevice(&dev));
    DevState *ds;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        ds = g_devs[dev];
    }
    std::lock_guard<std::mutex> lk(ds->mu);
    Buffer &b = ds->ws[{st, slot}];
    if (b.bytes < bytes) {
        if (b.ptr) {
            FF_HIP_CHECK(hipStreamSynchronize(st));
            FF_HIP_CHECK(hipFree(b.ptr));
            b.ptr = nullptr;
            b.bytes = 0;
        }
        size_t want = std::max<size_t>(bytes, size_t(1) << 20);
        if (hipMalloc(&b.ptr, want) != hipSuccess) {
            (void)hipGetLastError();
            b.ptr = nullptr;
            return fail(FF_ENOMEM, "workspace allocation of " + std::to_string(want) +
                                       " bytes failed");
        }
        b.bytes = want;
    }
    *out = b.ptr;
    return FF_OK;
}

int counter_buffer(hipStream_t st, unsigned **out)
{
    int dev = 0;
    FF_HIP_CHECK(hipGetDevice(&dev));
    DevState *ds;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        ds = g_devs[dev];
    }
    std::lock_guard<std::mutex> lk(ds->mu);
    unsigned *&c = ds->ctr[st];
    if (!c) {
        FF_HIP_CHECK(hipMalloc(&c, 256));
        FF_HIP_CHECK(hipMemset(c, 0, 256));
    }
    *out = c;
    return FF_OK;
}

// Host -> device copy through a pinned per-stream buffer, so that the
// caller's memory may be reused as soon as this returns and the copy stays
// asynchronous.  The buffer is reused once its previous copy has completed.
int upload_async(hipStream_t st, const void *src, size_t bytes, void *dst)
{
    int dev = 0;
    FF_HIP_CHECK(hipGetDevice(&dev));
    DevState *ds;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        ds = g_devs[dev];
    }
    std::lock_guard<std::mutex> lk(ds->mu);
    DevState::Staging &sg = ds->stage[st];
    if (!sg.done) FF_HIP_CHECK(hipEventCreateWithFlags(&sg.done, hipEventDisableTiming));
    if (sg.pending) {
        FF_HIP_CHECK(hipEventSynchronize(sg.done));
        sg.pending = false;
    }
    if (sg.bytes < bytes) {
        if (sg.host) FF_HIP_CHECK(hipHostFree(sg.host));
        sg.host = nullptr;
        sg.bytes = 0;
        const size_t want = std::max<size_t>(bytes, 64 << 10);
        FF_HIP_CHECK(hipHostMalloc(&sg.host, want, hipHostMallocDefault));
        sg.bytes = want;
    }
    std::memcpy(sg.host, src, bytes);
    FF_HIP_CHECK(hipMemcpyAsync(dst, sg.host, bytes, hipMemcpyHostToDevice, st));
    FF_HIP_CHECK(hipEventRecord(sg.done, st));
    sg.pending = true;
    return FF_OK;
}

int release_all()
{
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto &kv : g_devs) {
        DevState *ds = kv.second;
        std::lock_guard<std::mutex> lk2(ds->mu);
        for (auto &w : ds->ws) {
            if (w.second.ptr) {
                (void)hipStreamSynchronize(w.first.first);
                (void)hipFree(w.second.ptr);
            }
        }
        ds->ws.clear();
        for (auto &c : ds->ctr) {
            (void)hipStreamSynchronize(c.first);
            (void)hipFree(c.second);
        }
        ds->ctr.clear();
        for (auto &sg : ds->stage) {
            if (sg.second.done) {
                (void)hipEventSynchronize(sg.second.done);
                (void)hipEventDestroy(sg.second.done);
            }
            if (sg.second.host) (void)hipHostFree(sg.second.host);
        }
        ds->stage.clear();
    }
    return FF_OK;
}

hipStream_t stream_of(const ff_opts *o)
{
    if (o && o->stream) return (hipStream_t)o->stream;
    return g_stream;
}

void set_stream(hipStream_t s) { g_stream = s; }

ff_opts default_opts()
{
    ff_opts o;
    std::memset(&o, 0, sizeof(o));
    o.winograd_levels = -1;
    return o;
}

// ---------------------------------------------------------------------------
// Argument checks shared by the single and batched entry points
// ---------------------------------------------------------------------------
int check_args(uint32_t p, int transA, int transB, int64_t m, int64_t n, int64_t k,
               const uint32_t *A, int64_t lda, const uint32_t *B, int64_t ldb,
               const uint32_t *C, int64_t ldc)
{
    if (p < 2 || p > 0x7FFFFFFFu) return fail(FF_EINVAL, "p must satisfy 2 <= p < 2^31");
    if ((transA != 0 && transA != 1) || (transB != 0 && transB != 1))
        return fail(FF_EINVAL, "transA/transB must be FF_NOTRANS or FF_TRANS");
    if (m < 0 || n < 0 || k < 0) return fail(FF_EINVAL, "negative dimension");
    const int64_t DMAX = int64_t(1) << 30;
    if (m > DMAX || n > DMAX || k > DMAX) return fail(FF_EINVAL, "dimension exceeds 2^30");
    if (m == 0 || n == 0) return FF_OK;
    if (ldc < n) return fail(FF_EINVAL, "ldc < n");
    if (!C) return fail(FF_EINVAL, "C is null");
    if (k > 0) {
        if (lda < (transA ? m : k)) return fail(FF_EINVAL, "lda too small");
        if (ldb < (transB ? k : n)) return fail(FF_EINVAL, "ldb too small");
        if (!A || !B) return fail(FF_EINVAL, "A or B is null");
    }
    return FF_OK;
}

// alpha * R^t mod p, t = 0 .. 2S-2.
void digit_weights(uint32_t p, uint32_t alpha, int bits, int S, uint32_t *w)
{
    const uint64_t R = (uint64_t(1) << bits) % p;
    uint64_t x = alpha % p;
    for (int t = 0; t < 2 * S - 1; ++t) {
        w[t] = (uint32_t)x;
        x = (x * R) % p;
    }
}

int64_t round_up(int64_t x, int64_t q) { return (x + q - 1) / q * q; }

// Digit pairing (S >= 2): with D_i = A_i B_i and, for t = 1 .. 2S-3,
// K_t = sum over pairs i < j with i + j = t of (A_i + A_j)(B_i + B_j),
//     sum_t R^t E_t = sum_t R^t K_t + sum_i D_i (R^(2i) - sum_{j != i} R^(i+j)),
// because a_i b_j + a_j b_i = (a_i + a_j)(b_i + b_j) - a_i b_i - a_j b_j.
// The pairing kernel's accumulator sets are D_0 .. D_{S-1}, then K_1 ..
// K_{2S-3}; their weights (times alpha, mod p) follow.
static void pairing_weights(uint32_t p, const uint32_t *w, int S, uint32_t *out)
{
    for (int i = 0; i < S; ++i) {
        uint64_t x = w[2 * i];
        for (int j = 0; j < S; ++j)
            if (j != i) x += (uint64_t)(p - w[i + j]);
        out[i] = (uint32_t)(x % p);
    }
    for (int t = 1; t <= 2 * S - 3; ++t) out[S + t - 1] = w[t];
}

void i8_weights(I8Job &J, uint32_t alpha, int bits, int pairing)
{
    const int S = J.s;
    digit_weights(J.p, alpha, S == 1 ? 8 : bits, S, J.w);
    int nset = 2 * S - 1;
    if (pairing && S >= 2) {
        uint32_t pw[12];
        pairing_weights(J.p, J.w, S, pw);
        nset = 3 * S - 3;
        for (int t = 0; t < nset; ++t) J.w[t] = pw[t];
    }
    const double h = (double)(J.p / 2);
    for (int t = 0; t < nset; ++t)
        J.wc[t] = J.w[t] > J.p / 2 ? (double)J.w[t] - (double)J.p : (double)J.w[t];
    // every |E_t mod p| <= p/2 + 1 after the floating-point reduction
    const double bound = (double)nset * h * (h + 1.0) + (double)J.p;
    J.fp_epi = bound <= 9007199254740992.0 ? 1 : 0;
    // |E_t| <= S * KP * (R/2)^2 (balanced digits, R = 2^bits; the direct
    // plane's values are below 2^7); with pairing a set holds at most
    // pairing_max_pairs(S) products of digit sums, each <= R^2; |wc_t| <= p/2.
    // When the whole sum stays below 2^53 it is exact in binary64 and one
    // reduction suffices.
    const double dmax = S == 1 ? 128.0 : (double)(1 << (bits - 1));
    const double emax = pairing && S >= 2
                            ? (double)pairing_max_pairs(S) * (double)J.KP * 4.0 * dmax * dmax
                            : (double)S * (double)J.KP * dmax * dmax;
    J.epi_direct = J.fp_epi && (double)nset * h * emax + (double)J.p <= 9007199254740992.0;
}

// Packing task of one operand into centered doubles (row tile RT).
SliceJob pack_job(const void *X, int64_t ldx, int rows, int K, int trans, int in_mode,
                  uint32_t p, double *D, int RT, int KP)
{
    SliceJob s = slice_job(X, ldx, rows, K, trans, in_mode, p, 0, 0, (int8_t *)D, RT, KP);
    s.plane = (int64_t)s.rows_pad * KP * 8;
    return s;
}

// FP64 GEMM job on packed operands; kblock products fit between reductions.
F64Job f64_job(const double *Ad, const double *Bd, uint32_t *C, int64_t ldc, int64_t m,
               int64_t n, int KP, uint32_t p, uint32_t alpha, uint32_t beta, int64_t kblock,
               int tile)
{
    const F64Tile &t = f64_tile(tile);
    F64Job J;
    std::memset(&J, 0, sizeof(J));
    J.Ad = Ad; J.Bd = Bd; J.C = C; J.ldc = ldc;
    J.m = (int)m; J.n = (int)n; J.KP = KP;
    J.p = p; J.alpha = alpha; J.beta = beta;
    J.pd = (double)p; J.pinv = 1.0 / (double)p;
    // a stage adds F64_BK products to every partial sum
    J.fold_stages = (int)std::min<int64_t>(kblock / F64_BK, 0x3FFFFFFF);
    J.gm = t.GM;
    J.tiles_m = (int)((m + t.bm() - 1) / t.bm());
    J.tiles_n = (int)((n + t.bn() - 1) / t.bn());
    return J;
}

// ---------------------------------------------------------------------------
// Plain (no Winograd) paths
// ---------------------------------------------------------------------------
int run_f64_plain(uint32_t p, int transA, int transB, int64_t m, int64_t n, int64_t k,
                  uint32_t alpha, const void *A, int64_t lda, const void *B, int64_t ldb,
                  uint32_t beta, uint32_t *C, int64_t ldc, int in_mode, int64_t kblock,
                  int tile, void *ws, hipStream_t st)
{
    const F64Tile &t = f64_tile(tile);
    const int KP = (int)round_up(k, F64_BK);
    double *Ad = (double *)ws;
    double *Bd = Ad + round_up(m, t.bm()) * KP;
    // A: rows m, element (i, l) of op(A); B^T: rows n, element (j, l) = op(B)(l, j)
    SliceJob sa = pack_job(A, lda, (int)m, (int)k, transA, in_mode, p, Ad, t.bm(), KP);
    SliceJob sb = pack_job(B, ldb, (int)n, (int)k, transB ? 0 : 1, in_mode, p, Bd, t.bn(), KP);
    FF_HIP_CHECK(FF_TIMED(PROF_SLICE, st, launch_pack_f64_2(sa, sb, st)));
    F64Job J = f64_job(Ad, Bd, C, ldc, m, n, KP, p, alpha, beta, kblock, tile);
    int kts = 0;
    const int splits = f64_splits((int64_t)J.tiles_m * J.tiles_n, KP / F64_BK, &kts);
    if (splits > 1) {
        // partial products per K split, after the packed operands
        const int64_t packed = (round_up(m, t.bm()) + round_up(n, t.bn())) * KP * 8;
        J.kt_split = kts;
        J.part = (uint32_t *)((char *)ws + round_up(packed, 256));
    }
    FF_HIP_CHECK(FF_TIMED(PROF_GEMM, st, launch_f64(tile, J, st)));
    if (splits > 1)
        FF_HIP_CHECK(launch_split_reduce(J.part, splits, m, n, C, ldc, p, alpha, beta, st));
    return FF_OK;
}

// Describes the slicing of an operand into packed digit planes.
SliceJob slice_job(const void *X, int64_t ldx, int rows, int K, int trans, int in_mode,
                   uint32_t p, int S, int bits, int8_t *D, int RT, int KP)
{
    SliceJob s;
    std::memset(&s, 0, sizeof(s));
    s.X = X; s.ldx = ldx; s.rows = rows; s.K = K; s.trans = trans; s.in_mode = in_mode;
    s.p = p; s.S = S; s.bits = bits; s.D = D; s.RT = RT;
    s.rows_pad = (int)round_up(std::max(rows, 1), RT);
    s.KP = KP;
    s.plane = (int64_t)s.rows_pad * KP;
    return s;
}

int run_i8_plain(uint32_t p, int transA, int transB, int64_t m, int64_t n, int64_t k,
                 uint32_t alpha, const uint32_t *A, int64_t lda, const uint32_t *B,
                 int64_t ldb, uint32_t beta, uint32_t *C, int64_t ldc, const Plan &P,
                 void *ws, hipStream_t st)
{
    // tile shape: the plan's configuration, or the pairing kernel's
    const int bm = P.pairing ? i8p_bm(P.slices) : i8_tile(P.tile).bm();
    const int bn = P.pairing ? i8p_bn(P.slices) : i8_tile(P.tile).bn();
    const int gm = P.pairing ? 8 : i8_tile(P.tile).GM;
    // planes per operand: the digits, and with pairing the digit sums
    const int planes = P.pairing ? P.slices * (P.slices + 1) / 2 : P.slices;
    const int64_t kpass = std::min<int64_t>(k, P.kblock);
    const int KP = (int)round_up(kpass, I8_BK);
    const int mp = (int)round_up(m, bm), np = (int)round_up(n, bn);
    int8_t *Ad = (int8_t *)ws;
    int8_t *Bd = Ad + (int64_t)planes * mp * KP;
    for (int64_t k0 = 0; k0 < k; k0 += kpass) {
        const int kc = (int)std::min<int64_t>(kpass, k - k0);
        const int KPc = (int)round_up(kc, I8_BK);
        // A: rows m, element (i, l) of op(A)
        const uint32_t *Ak = transA ? A + k0 * lda : A + k0;
        SliceJob sa = slice_job(Ak, lda, (int)m, kc, transA, IN_RESIDUE, p, P.slices, P.bits,
                                Ad, bm, KPc);
        sa.pairs = P.pairing;
        // B^T: rows n, element (j, l) = op(B)(l, j)
        const uint32_t *Bk = transB ? B + k0 : B + k0 * ldb;
        SliceJob sb = slice_job(Bk, ldb, (int)n, kc, transB ? 0 : 1, IN_RESIDUE, p, P.slices,
                                P.bits, Bd, bn, KPc);
        sb.pairs = P.pairing;
        FF_HIP_CHECK(FF_TIMED(PROF_SLICE, st, launch_slice2(sa, sb, st)));
        I8Job J;
        std::memset(&J, 0, sizeof(J));
        J.Ad = Ad; J.Bd = Bd; J.a_plane = sa.plane; J.b_plane = sb.plane;
        J.C = C; J.ldc = ldc; J.m = (int)m; J.n = (int)n; J.KP = KPc; J.s = P.slices;
        J.p = p; J.beta = k0 == 0 ? beta : 1u;
        J.pd = (double)p; J.pinv = 1.0 / (double)p;
        i8_weights(J, alpha, P.bits, P.pairing);
        J.gm = gm;
        J.tiles_m = mp / bm; J.tiles_n = np / bn;
        if (P.pairing)
            FF_HIP_CHECK(FF_TIMED(PROF_GEMM, st, launch_i8_pair(J, st)));
        else
            FF_HIP_CHECK(FF_TIMED(PROF_GEMM, st, launch_i8(P.tile, J, st)));
    }
    return FF_OK;
}

// counter: device word for the count of bad entries, or null to allocate one
// for the call.
int validate_inputs(uint32_t p, int transA, int transB, int64_t m, int64_t n, int64_t k,
                    const uint32_t *A, int64_t lda, const uint32_t *B, int64_t ldb,
                    uint32_t beta, const uint32_t *C, int64_t ldc, hipStream_t st,
                    unsigned *counter)
{
    unsigned *bad = counter;
    if (!bad) FF_HIP_CHECK(hipMalloc(&bad, sizeof(unsigned)));
    unsigned h = 0;
    // zeroed by a kernel (C <- 0 * C on a 1 x 1 matrix), not a memset node
    hipError_t e = launch_scale(bad, 1, 1, 1, 2u, 0u, st);
    if (e == hipSuccess && k > 0) {
        e = launch_validate(A, lda, transA ? k : m, transA ? m : k, p, bad, st);
        if (e == hipSuccess) e = launch_validate(B, ldb, transB ? n : k, transB ? k : n, p, bad, st);
    }
    if (e == hipSuccess && beta) e = launch_validate(C, ldc, m, n, p, bad, st);
    if (e == hipSuccess) e = hipMemcpyAsync(&h, bad, sizeof(unsigned), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (!counter) (void)hipFree(bad);
    if (e != hipSuccess) return fail(FF_EHIP, std::string("validate: ") + hipGetErrorString(e));
    if (h) return fail(FF_EINVAL, std::to_string(h) + " input entries are not residues < p");
    return FF_OK;
}

} // namespace ff

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
using namespace ff;

namespace ff {

// Plan of one ff_fgemm_ex call.  The automatic path takes FP64 for a
// product small enough for the one-launch kernel (a single launch where the
// INT8 path slices and then multiplies), when no digit width is asked for
// and the FP64 K-block allows the modulus; otherwise the planner's choice.
static int plan_call(uint32_t p, int64_t m, int64_t n, int64_t k, const ff_opts &o, Plan *P)
{
    if (o.path == FF_PATH_AUTO && o.digit_bits == 0 && o.winograd_levels <= 0 &&
        !o.digit_pairing && f64_small(m, n, k)) {
        ff_opts fo = o;
        fo.path = FF_PATH_FP64;
        if (make_plan(p, m, n, k, fo, P) == FF_OK && P->small) return FF_OK;
    }
    return make_plan(p, m, n, k, o, P);
}

} // namespace ff

extern "C" {

int ff_init(void)
{
    int rc = check_device();
    if (rc == FF_OK) rc = noalloc_setup();
    return rc;
}

int ff_finalize(void) { return release_all(); }

int ff_set_stream(void *hip_stream)
{
    set_stream((hipStream_t)hip_stream);
    return FF_OK;
}

const char *ff_last_error(void) { return g_err.c_str(); }

int ff_plan_query(uint32_t p, int transA, int transB, int64_t m, int64_t n, int64_t k,
                  const ff_opts *opts, ff_plan_info *out)
{
    if (!out) return fail(FF_EINVAL, "out is null");
    if ((transA != 0 && transA != 1) || (transB != 0 && transB != 1))
        return fail(FF_EINVAL, "transA/transB must be FF_NOTRANS or FF_TRANS");
    if (m < 0 || n < 0 || k < 0) return fail(FF_EINVAL, "negative dimension");
    ff_opts o = opts ? *opts : default_opts();
    Plan P;
    int rc = plan_call(p, m, n, k, o, &P);
    if (rc) return rc;
    std::memset(out, 0, sizeof(*out));
    out->path = P.path;
    out->winograd_levels = P.levels;
    out->preadds_reduced = P.preadds_reduced;
    out->digit_bits = P.path == FF_PATH_INT8 ? P.bits : 0;
    out->slices = P.path == FF_PATH_INT8 ? P.slices : 0;
    out->operand_lo = P.lo;
    out->operand_hi = P.hi;
    out->max_abs_product = P.max_prod;
    out->kblock = P.kblock;
    out->workspace_bytes = P.ws_bytes;
    out->tile_config = P.tile;
    out->digit_products = P.path != FF_PATH_INT8 ? 0
                          : P.pairing ? P.slices * (P.slices + 1) / 2 : P.slices * P.slices;
    return FF_OK;
}

} // extern "C"

namespace ff {

int presliced_prepare(uint32_t p, int64_t m, int64_t n, int64_t k, const ff_opts &o,
                      hipStream_t st, PreSliced *ps)
{
    ps->ok = false;
    if (m <= 0 || n <= 0 || k <= 0 || o.validate) return FF_OK;
    Plan P;
    int rc = plan_call(p, m, n, k, o, &P);
    if (rc) return rc;
    if (P.levels > 0 || P.path != FF_PATH_INT8 || P.pairing || P.kblock < k) return FF_OK;
    const int bm = i8_tile(P.tile).bm(), bn = i8_tile(P.tile).bn();
    const int64_t KP = round_up(k, I8_BK), mp = round_up(m, bm), np = round_up(n, bn);
    void *ws = nullptr;
    if ((rc = workspace(st, (size_t)(P.slices * (mp + np) * KP), &ws))) return rc;
    ps->P = P;
    ps->Ad = (int8_t *)ws;
    ps->Bd = ps->Ad + P.slices * mp * KP;
    ps->plane_a = mp * KP;
    ps->plane_b = np * KP;
    ps->rta = bm;
    ps->rtb = bn;
    ps->KP = (int)KP;
    ps->ok = true;
    return FF_OK;
}

int presliced_run(const PreSliced &ps, uint32_t p, int64_t m, int64_t n, uint32_t alpha,
                  uint32_t beta, uint32_t *C, int64_t ldc, hipStream_t st)
{
    const Plan &P = ps.P;
    I8Job J;
    std::memset(&J, 0, sizeof(J));
    J.Ad = ps.Ad; J.Bd = ps.Bd; J.a_plane = ps.plane_a; J.b_plane = ps.plane_b;
    J.C = C; J.ldc = ldc; J.m = (int)m; J.n = (int)n; J.KP = ps.KP; J.s = P.slices;
    J.p = p; J.beta = beta % p;
    J.pd = (double)p; J.pinv = 1.0 / (double)p;
    i8_weights(J, alpha % p, P.bits, 0);
    J.gm = i8_tile(P.tile).GM;
    J.tiles_m = (int)(round_up(m, ps.rta) / ps.rta);
    J.tiles_n = (int)(round_up(n, ps.rtb) / ps.rtb);
    FF_HIP_CHECK(FF_TIMED(PROF_GEMM, st, launch_i8(P.tile, J, st)));
    return FF_OK;
}

int fgemm_call(uint32_t p, int transA, int transB, int64_t m, int64_t n, int64_t k,
               uint32_t alpha, const uint32_t *A, int64_t lda, const uint32_t *B,
               int64_t ldb, uint32_t beta, uint32_t *C, int64_t ldc, const ff_opts *opts,
               void *ws_fixed, size_t ws_fixed_bytes)
{
    int rc = check_args(p, transA, transB, m, n, k, A, lda, B, ldb, C, ldc);
    if (rc) return rc;
    if (m == 0 || n == 0) return FF_OK;
    ff_opts o = opts ? *opts : default_opts();
    if (ws_fixed) {
        // fixed scratch: plain products only (Winograd levels need temporaries)
        if (o.winograd_levels > 0)
            return fail(FF_EUNSUPPORTED, "Winograd levels need workspace; this entry point "
                                         "runs plain products only");
        o.winograd_levels = 0;
    }
    if ((rc = check_device())) return rc;
    hipStream_t st = stream_of(&o);
    alpha %= p;
    beta %= p;
    if (o.validate) {
        rc = validate_inputs(p, transA, transB, m, n, k, A, lda, B, ldb, beta, C, ldc, st,
                             (unsigned *)ws_fixed);
        if (rc) return rc;
    }
    if (k == 0 || alpha == 0) {
        if (beta == 1) return FF_OK;
        FF_HIP_CHECK(launch_scale(C, ldc, m, n, p, beta, st));
        return FF_OK;
    }
    Plan P;
    if ((rc = plan_call(p, m, n, k, o, &P))) return rc;
    if (P.levels > 0)
        return run_winograd(p, transA, transB, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc,
                            P, o, st);
    if (P.path == FF_PATH_FP64 && P.small) {
        F64Small J;
        std::memset(&J, 0, sizeof(J));
        J.A = A; J.B = B; J.lda = lda; J.ldb = ldb; J.ta = transA; J.tb = transB;
        J.C = C; J.ldc = ldc;
        J.m = (int)m; J.n = (int)n; J.k = (int)k;
        J.p = p; J.alpha = alpha; J.beta = beta;
        J.pd = (double)p; J.pinv = 1.0 / (double)p;
        J.fold_steps = (int)std::min<int64_t>(P.kblock / 4, 0x3FFFFFFF);
        FF_HIP_CHECK(FF_TIMED(PROF_GEMM, st, launch_f64_small(J, st)));
        return FF_OK;
    }
    void *ws = ws_fixed;
    if (ws_fixed) {
        if ((size_t)P.ws_bytes > ws_fixed_bytes)
            return fail(FF_EINVAL, "the product needs " + std::to_string(P.ws_bytes) +
                                       " bytes of scratch; the fixed scratch holds " +
                                       std::to_string(ws_fixed_bytes));
    } else if ((rc = workspace(st, (size_t)P.ws_bytes, &ws))) {
        return rc;
    }
    if (P.path == FF_PATH_FP64)
        return run_f64_plain(p, transA, transB, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc,
                             IN_RESIDUE, P.kblock, P.tile, ws, st);
    return run_i8_plain(p, transA, transB, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, P,
                        ws, st);
}

} // namespace ff

extern "C" {

int ff_fgemm_ex(uint32_t p, int transA, int transB, int64_t m, int64_t n, int64_t k,
                uint32_t alpha, const uint32_t *A, int64_t lda, const uint32_t *B,
                int64_t ldb, uint32_t beta, uint32_t *C, int64_t ldc, const ff_opts *opts)
{
    return fgemm_call(p, transA, transB, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, opts,
                      nullptr, 0);
}

int ff_fgemm(uint32_t p, int transA, int transB, int64_t m, int64_t n, int64_t k,
             uint32_t alpha, const uint32_t *A, int64_t lda, const uint32_t *B, int64_t ldb,
             uint32_t beta, uint32_t *C, int64_t ldc)
{
    return ff_fgemm_ex(p, transA, transB, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc,
                       nullptr);
}

} // extern "C"
