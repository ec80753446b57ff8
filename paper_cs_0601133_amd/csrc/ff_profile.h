// Event-pair timing of kernel launches (enabled by ff_profile_enable).
#pragma once

#include <hip/hip_runtime.h>

namespace ff {

enum { PROF_GEMM = 0, PROF_SLICE = 1 };
bool profiling();
void *prof_begin(int kind, hipStream_t st);
void prof_end(void *tok, hipStream_t st);

// Brackets one launch expression.
#define FF_TIMED(kind, st, expr)                                              \
    ([&]() -> hipError_t {                                                    \
        void *tok_ = ::ff::prof_begin((kind), (st));                          \
        hipError_t e_ = (expr);                                               \
        ::ff::prof_end(tok_, (st));                                           \
        return e_;                                                            \
    }())

} // namespace ff
