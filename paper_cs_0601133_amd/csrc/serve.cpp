// Serving loop (placeholder until the server lands).
#include "ff_runtime.h"

using namespace ff;

extern "C" {
int ff_server_create(int64_t, const ff_opts *, void **) { return fail(FF_EUNSUPPORTED, "not available"); }
int ff_server_submit(void *, const ff_job *, uint64_t *) { return fail(FF_EUNSUPPORTED, "not available"); }
int ff_server_poll(void *, uint64_t, int *) { return fail(FF_EUNSUPPORTED, "not available"); }
int ff_server_wait(void *, uint64_t) { return fail(FF_EUNSUPPORTED, "not available"); }
int ff_server_stats(void *, double *, double *, double *, int64_t *, int64_t *)
{
    return fail(FF_EUNSUPPORTED, "not available");
}
int ff_server_destroy(void *) { return fail(FF_EUNSUPPORTED, "not available"); }
}
