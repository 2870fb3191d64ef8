// noalloc.hip -- fglt_raw_noalloc: the single-graph transform on a workspace
// that lives in the library's own device memory, for callers that cannot
// allocate.  See include/fglt.h.
#include <mutex>

#include "raw.h"

using namespace fglt;

namespace {

// The workspace of fglt_raw_noalloc: one array per device, loaded with the
// library's code object and held until the process ends.  In host code its
// name is only a stand-in for the symbol: kernels and copies get its device
// address from hipGetSymbolAddress, taken once per device.
static __device__ __align__(256) unsigned char scratch[FGLT_NOALLOC_SCRATCH_BYTES];

constexpr int MAXDEV = 64;
std::mutex g_mu;
void* g_scratch[MAXDEV];  // device address of `scratch` on each device, once taken

hipError_t scratch_address(void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= MAXDEV) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        if ((e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch))) != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return hipSuccess;
}

}  // namespace

extern "C" int fglt_raw_noalloc(int64_t n, int64_t nnz, const int64_t* offsets, const int32_t* indices,
                                int64_t* out, unsigned flags, const fglt_raw_plan* plan, fglt_stats* stats,
                                void* stream) {
    // timing creates HIP events: not offered here
    if (flags & (FGLT_TIMING | FGLT_PROGRESS)) return FGLT_EINVAL;
    if (n < 0 || nnz < 0) return FGLT_EINVAL;
    if (n >= ((int64_t)1 << 31) || nnz >= ((int64_t)1 << 40)) return FGLT_EINVAL;
    if (fglt_raw_workspace(n, nnz) > (size_t)FGLT_NOALLOC_SCRATCH_BYTES) return FGLT_EWORKSPACE;
    void* ws = nullptr;
    if (n > 0) FGLT_HIP_TRY(scratch_address(&ws));
    // one stream: the transform's second stream would be created on first use
    // the status word lives in the array: the call waits and returns it
    return raw_run(n, nnz, offsets, indices, out, ws, (size_t)FGLT_NOALLOC_SCRATCH_BYTES, flags | FGLT_VALIDATE, plan,
                   stats, stream, true);
}
