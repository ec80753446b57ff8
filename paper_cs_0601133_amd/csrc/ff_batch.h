// Batch description shared by the batched entry points, the graph capture,
// the Winograd driver and the server.  Not part of the C ABI.
#pragma once

#include <vector>

#include "ff_runtime.h"

namespace ff {

// One fgemm of a batch, with the decisions of its plan.
struct IJob {
    uint32_t p = 0;
    int ta = 0, tb = 0;
    int64_t m = 0, n = 0, k = 0;
    uint32_t alpha = 0, beta = 0;
    const void *A = nullptr;
    int64_t lda = 0;
    const void *B = nullptr;
    int64_t ldb = 0;
    uint32_t *C = nullptr;
    int64_t ldc = 0;
    int in_mode = IN_RESIDUE; // residues, or centered int32 values
    int path = FF_PATH_INT8;
    int S = 0, bits = 0;      // INT8 digits
    int64_t kblock = 0;       // FP64 fold interval / INT8 int32 K-block
};

struct BatchPrep {
    int path = FF_PATH_INT8;
    int tile = -1;             // INT8 or FP64 tile configuration
    std::vector<SliceJob> sj;  // digit slicing (INT8) or packing (FP64) tasks
    std::vector<I8Job> ij;
    std::vector<F64Job> fj;    // jobs reduced per stage, then jobs reduced per step
    int fj_fine = 0;           // index of the first per-step job in fj
    int slice_blocks = 0, i8_tiles = 0, f64_tiles[2] = {0, 0};
    bool uniform_s = false;    // INT8: every job has the tile's digit count
    std::vector<IJob> scales;  // k == 0 or alpha == 0: C <- beta*C
    std::vector<IJob> singles; // longer than one int32 pass: run alone
    int64_t off_sj = 0, off_ij = 0, off_fj = 0;
    int64_t off_planes = 0, table_bytes = 0, ws_bytes = 0;
    std::vector<char> staging; // serialised tables bound to a workspace
    char *bound_ws = nullptr;
};

int prep_batch(const std::vector<IJob> &jobs, int path, int tile, BatchPrep *out);
int upload_batch(BatchPrep &B, char *ws, hipStream_t st, bool sync);
// slice = false: the digit planes or packed doubles are already written
// (fused Winograd pre-additions); only the GEMM launches run.
int launch_batch(BatchPrep &B, unsigned *ctr, hipStream_t st, int persistent, bool slice = true);
int job_from_abi(const ff_job &a, const ff_opts &o, IJob *out);
int run_single_job(const IJob &j, const ff_opts &o, hipStream_t st);
int prep_abi_batch(const ff_job *jobs, int njobs, const ff_opts &o, BatchPrep *B);

} // namespace ff
