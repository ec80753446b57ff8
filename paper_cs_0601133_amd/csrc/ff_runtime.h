// Host-side helpers shared by the C ABI, the Winograd driver, the batched
// launcher and the server.  Not part of the C ABI.
#pragma once

#include "ff_internal.h"

namespace ff {

// ff_ftrsm_ex with one more choice: bt = 1 takes the m x n matrix B stored
// transposed (entry (i, j) at B[j * ldb + i], ldb >= m), which is how the
// LQUP recursion solves G T = X for G in place without transposing X.
int ftrsm_run(uint32_t p, int uplo, int transT, int diag, int64_t m, int64_t n, uint32_t alpha,
              const uint32_t *T, int64_t ldt, uint32_t *B, int64_t ldb, int bt,
              const ff_opts *opts);

int check_device();
// Per-(device, stream, slot) device buffer, grown on demand (growth waits
// for the stream).  Slot 0 serves fgemm; a routine that calls fgemm while
// holding data of its own (the triangular solve) uses slot 1.
int workspace(hipStream_t st, size_t bytes, void **out, int slot = 0);
// 256-byte zeroed counter block per (device, stream) for persistent kernels,
// which leave it zeroed.
int counter_buffer(hipStream_t st, unsigned **out);
// Asynchronous host -> device copy through pinned per-stream staging.
int upload_async(hipStream_t st, const void *src, size_t bytes, void *dst);
int release_all();
hipStream_t stream_of(const ff_opts *o);
void set_stream(hipStream_t s);
ff_opts default_opts();
int check_args(uint32_t p, int transA, int transB, int64_t m, int64_t n, int64_t k,
               const uint32_t *A, int64_t lda, const uint32_t *B, int64_t ldb,
               const uint32_t *C, int64_t ldc);
void digit_weights(uint32_t p, uint32_t alpha, int bits, int S, uint32_t *w);
int64_t round_up(int64_t x, int64_t q);
SliceJob slice_job(const void *X, int64_t ldx, int rows, int K, int trans, int in_mode,
                   uint32_t p, int S, int bits, int8_t *D, int RT, int KP);
int slice_blocks(const SliceJob &J);
SliceJob pack_job(const void *X, int64_t ldx, int rows, int K, int trans, int in_mode,
                  uint32_t p, double *D, int RT, int KP);
int pack_blocks(const SliceJob &J);
F64Job f64_job(const double *Ad, const double *Bd, uint32_t *C, int64_t ldc, int64_t m,
               int64_t n, int KP, uint32_t p, uint32_t alpha, uint32_t beta, int64_t kblock,
               int tile);
// ws: (round_up(m, bm) + round_up(n, bn)) * round_up(k, 16) doubles, then
// (256-aligned) the split-K partials when f64_splits splits the launch.
int run_f64_plain(uint32_t p, int transA, int transB, int64_t m, int64_t n, int64_t k,
                  uint32_t alpha, const void *A, int64_t lda, const void *B, int64_t ldb,
                  uint32_t beta, uint32_t *C, int64_t ldc, int in_mode, int64_t kblock,
                  int tile, void *ws, hipStream_t st);
int run_i8_plain(uint32_t p, int transA, int transB, int64_t m, int64_t n, int64_t k,
                 uint32_t alpha, const uint32_t *A, int64_t lda, const uint32_t *B,
                 int64_t ldb, uint32_t beta, uint32_t *C, int64_t ldc, const Plan &P,
                 void *ws, hipStream_t st);
// The whole ff_fgemm_ex call.  ws_fixed: device scratch of ws_fixed_bytes
// to use instead of the per-stream workspace (plain products only; a
// product that needs more is rejected), or null.
int fgemm_call(uint32_t p, int transA, int transB, int64_t m, int64_t n, int64_t k,
               uint32_t alpha, const uint32_t *A, int64_t lda, const uint32_t *B,
               int64_t ldb, uint32_t beta, uint32_t *C, int64_t ldc, const ff_opts *opts,
               void *ws_fixed, size_t ws_fixed_bytes);
// A product C <- alpha A B + beta C (A m x k, B k x n) whose operands a
// kernel of the caller writes as INT8 digit planes itself: presliced_prepare
// tells whether ff_fgemm_ex would run it as one plain INT8 launch (no
// Winograd level, no digit pairing, K in one pass, no validation) and, if
// so, takes the workspace for the planes (the stream's fgemm slot, valid
// until the next fgemm call on the stream) and fills *ps with their layout
// (the digit slicer's: A rows with row tile rta, B^T rows with row tile
// rtb, KP padded K, planes plane_a / plane_b bytes apart).  presliced_run
// then launches the INT8 GEMM on them, exactly as ff_fgemm_ex would after
// its slicing.
struct PreSliced {
    bool ok = false;
    Plan P;
    int8_t *Ad = nullptr, *Bd = nullptr;
    int64_t plane_a = 0, plane_b = 0;
    int rta = 0, rtb = 0, KP = 0;
};
int presliced_prepare(uint32_t p, int64_t m, int64_t n, int64_t k, const ff_opts &o,
                      hipStream_t st, PreSliced *ps);
int presliced_run(const PreSliced &ps, uint32_t p, int64_t m, int64_t n, uint32_t alpha,
                  uint32_t beta, uint32_t *C, int64_t ldc, hipStream_t st);
// Device address of the static scratch on the current device (noalloc.cpp);
// noalloc_setup() looks it up once per device.
int noalloc_setup();
// Winograd levels > 0 (winograd.cpp).
int run_winograd(uint32_t p, int transA, int transB, int64_t m, int64_t n, int64_t k,
                 uint32_t alpha, const uint32_t *A, int64_t lda, const uint32_t *B,
                 int64_t ldb, uint32_t beta, uint32_t *C, int64_t ldc, const Plan &P,
                 const ff_opts &o, hipStream_t st);

} // namespace ff
