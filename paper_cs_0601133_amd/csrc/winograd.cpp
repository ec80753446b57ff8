// Winograd's variant over Z/pZ (placeholder until the level driver lands).
#include "ff_runtime.h"

namespace ff {

int run_winograd(uint32_t, int, int, int64_t, int64_t, int64_t, uint32_t, const uint32_t *,
                 int64_t, const uint32_t *, int64_t, uint32_t, uint32_t *, int64_t,
                 const Plan &, const ff_opts &, hipStream_t)
{
    return fail(FF_EUNSUPPORTED, "Winograd levels are not available yet");
}

} // namespace ff
