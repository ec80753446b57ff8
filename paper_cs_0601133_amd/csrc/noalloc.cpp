// ff_fgemm_noalloc: the plain product of ff_fgemm_ex with its workspace (the
// digit planes of the INT8 path, the packed doubles and split-K partials of
// the FP64 path, the validation counter) in a static device array instead of
// memory the library allocates, for callers that cannot allocate.
//
// The array lives in this file's code object: each device that loads it holds
// its own copy, at its own address, until the process ends.  Host code never
// uses the array's name as a device address (on the host it names a stand-in
// object); the address comes from hipGetSymbolAddress, looked up once per
// device by noalloc_setup() (called by ff_init, else by the first call on the
// device) and passed to the kernels like any workspace pointer.
#include <mutex>
#include <string>

#include "ff_internal.h"
#include "ff_runtime.h"

static __device__ __align__(256) unsigned char scratch[FF_NOALLOC_SCRATCH_BYTES];

namespace ff {

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
void *g_ptr[MAX_DEVICES] = {};

int scratch_ptr(void **out)
{
    int dev = 0;
    FF_HIP_CHECK(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES)
        return fail(FF_EUNSUPPORTED, "device index " + std::to_string(dev) + " out of range");
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return fail(FF_EHIP, std::string("hipGetSymbolAddress(scratch): ") +
                                     hipGetErrorString(e));
        }
        g_ptr[dev] = ptr;
    }
    *out = g_ptr[dev];
    return FF_OK;
}

} // namespace

int noalloc_setup()
{
    void *ptr = nullptr;
    return scratch_ptr(&ptr);
}

} // namespace ff

using namespace ff;

extern "C" int ff_fgemm_noalloc(uint32_t p, int transA, int transB, int64_t m, int64_t n,
                                int64_t k, uint32_t alpha, const uint32_t *A, int64_t lda,
                                const uint32_t *B, int64_t ldb, uint32_t beta, uint32_t *C,
                                int64_t ldc, const ff_opts *opts)
{
    int rc = check_args(p, transA, transB, m, n, k, A, lda, B, ldb, C, ldc);
    if (rc) return rc;
    if (m == 0 || n == 0) return FF_OK;
    if ((rc = check_device())) return rc;
    void *ptr = nullptr;
    if ((rc = scratch_ptr(&ptr))) return rc;
    return fgemm_call(p, transA, transB, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, opts,
                      ptr, FF_NOALLOC_SCRATCH_BYTES);
}
