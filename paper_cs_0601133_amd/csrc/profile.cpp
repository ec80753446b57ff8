// HIP event pairs around kernel launches, for measurement (ff_profile_*).
#include <mutex>
#include <vector>

#include "ff_profile.h"
#include "ff_runtime.h"

namespace ff {

namespace {
struct Pair {
    hipEvent_t a = nullptr, b = nullptr;
    int kind = 0;
};
std::mutex g_pmu;
int g_mask = 0;
std::vector<Pair> g_used, g_free;
} // namespace

bool profiling() { return g_mask != 0; }

void *prof_begin(int kind, hipStream_t st)
{
    if (!(g_mask & (kind == PROF_GEMM ? FF_PROFILE_GEMM : FF_PROFILE_PREP))) return nullptr;
    std::lock_guard<std::mutex> lk(g_pmu);
    Pair p;
    if (!g_free.empty()) {
        p = g_free.back();
        g_free.pop_back();
    } else {
        if (hipEventCreate(&p.a) != hipSuccess || hipEventCreate(&p.b) != hipSuccess)
            return nullptr;
    }
    p.kind = kind;
    if (hipEventRecord(p.a, st) != hipSuccess) {
        g_free.push_back(p);
        return nullptr;
    }
    g_used.push_back(p);
    return (void *)(uintptr_t)g_used.size(); // 1-based index
}

void prof_end(void *tok, hipStream_t st)
{
    if (!tok) return;
    std::lock_guard<std::mutex> lk(g_pmu);
    const size_t i = (size_t)(uintptr_t)tok - 1;
    if (i < g_used.size()) (void)hipEventRecord(g_used[i].b, st);
}

} // namespace ff

using namespace ff;

extern "C" {

int ff_profile_enable(int mask)
{
    std::lock_guard<std::mutex> lk(g_pmu);
    for (auto &p : g_used) g_free.push_back(p);
    g_used.clear();
    g_mask = mask & (FF_PROFILE_GEMM | FF_PROFILE_PREP);
    return FF_OK;
}

int ff_profile_read(double *gemm_ms, int64_t *gemm_launches, double *slice_ms,
                    int64_t *slice_launches)
{
    std::lock_guard<std::mutex> lk(g_pmu);
    double g = 0, s = 0;
    int64_t ng = 0, ns = 0;
    for (auto &p : g_used) {
        if (hipEventSynchronize(p.b) != hipSuccess) return fail(FF_EHIP, "event sync failed");
        float ms = 0;
        if (hipEventElapsedTime(&ms, p.a, p.b) != hipSuccess)
            return fail(FF_EHIP, "event elapsed time failed");
        if (p.kind == PROF_GEMM) { g += ms; ++ng; } else { s += ms; ++ns; }
        g_free.push_back(p);
    }
    g_used.clear();
    if (gemm_ms) *gemm_ms = g;
    if (gemm_launches) *gemm_launches = ng;
    if (slice_ms) *slice_ms = s;
    if (slice_launches) *slice_launches = ns;
    return FF_OK;
}

} // extern "C"
