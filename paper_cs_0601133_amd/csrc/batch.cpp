// Batched persistent launch (placeholder until the batch driver lands).
#include "ff_runtime.h"

using namespace ff;

extern "C" {
int ff_fgemm_batched(const ff_job *, int, const ff_opts *)
{
    return fail(FF_EUNSUPPORTED, "batched launches are not available yet");
}
int ff_batch_graph_create(const ff_job *, int, const ff_opts *, void **)
{
    return fail(FF_EUNSUPPORTED, "batch graphs are not available yet");
}
int ff_batch_graph_launch(void *, void *) { return fail(FF_EUNSUPPORTED, "not available"); }
int ff_batch_graph_destroy(void *) { return fail(FF_EUNSUPPORTED, "not available"); }
}
