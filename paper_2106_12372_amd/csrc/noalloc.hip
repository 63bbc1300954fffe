// A training step that allocates nothing, for callers that cannot allocate
// device memory (code under stream capture, tight serving loops).  Its scratch
// (the per-tile weight-gradient partials, loss partials and flags of one
// step) is a file-scope device array of a fixed size instead of a caller
// buffer; the step itself is the one nrc_train_step enqueues, on the same
// kernels.
//
// Each GPU the library runs on holds its own copy of the array until the
// process ends.  In host code the array's name is a host-side stand-in, so
// the array's device address is looked up once per device with
// hipGetSymbolAddress and only that address is handed to the kernels.  Every
// call on a GPU shares that GPU's array and leaves the last call's contents in
// it; the step writes every scratch byte it later reads, so nothing needs
// clearing between calls.  Calls that overlap on one GPU (two streams, two
// threads) race on the array.
#include <hip/hip_runtime.h>

#include <mutex>

#include "nrc_api_internal.h"
#include "nrc_internal.h"

namespace {

static __device__ __align__(256) unsigned char scratch[NRC_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};

// Device address of `scratch` on `dev` (looked up on the first call there,
// with `dev` current).  NULL and an error message when the lookup fails.
void* scratch_on(int dev) {
    std::lock_guard<std::mutex> lock(g_mu);
    if (g_scratch[dev]) return g_scratch[dev];
    int cur = 0;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) { nrc::device_fail(e, "hipGetDevice"); return nullptr; }
    if (cur != dev && (e = hipSetDevice(dev)) != hipSuccess) { nrc::device_fail(e, "hipSetDevice"); return nullptr; }
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != dev) (void)hipSetDevice(cur);
    if (e != hipSuccess || p == nullptr) {
        nrc::device_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "scratch symbol lookup");
        return nullptr;
    }
    g_scratch[dev] = p;
    return p;
}

}  // namespace

using namespace nrc;

extern "C" int nrc_train_step_noalloc(nrc_cache* cache, const void* enc, const float* target, int64_t n,
                                      float* loss_dev, int32_t* skipped_dev, void* stream) {
    if (!cache) return fail(NRC_EINVAL, "cache is NULL");
    if (n < 1) return fail(NRC_EINVAL, "a training batch needs n >= 1");
    if (n > ((int64_t)1 << 31)) return fail(NRC_EINVAL, "training batch too large");
    if (!enc || !target) return fail(NRC_EINVAL, "NULL buffer");
    if (!aligned16(enc) || ((uintptr_t)target & 3)) return fail(NRC_EINVAL, "misaligned buffer");
    if (((uintptr_t)loss_dev & 3) || ((uintptr_t)skipped_dev & 3)) return fail(NRC_EINVAL, "misaligned output");
    const size_t need = scratch_layout(cache->cfg, n).total;
    if (need > (size_t)NRC_NOALLOC_SCRATCH_BYTES)
        return fail(NRC_ENOMEM,
                    "a step over %lld records needs %zu bytes of scratch, more than the %zu bytes of the "
                    "library's fixed scratch array (use nrc_train_step with a caller buffer)",
                    (long long)n, need, (size_t)NRC_NOALLOC_SCRATCH_BYTES);
    if (cache->device < 0 || cache->device >= kMaxDevices) return fail(NRC_EINVAL, "device id out of range");
    char* sc = (char*)scratch_on(cache->device);
    if (!sc) return NRC_EDEVICE;
    const int rc = enqueue_train_step(cache, enc, target, nullptr, n, sc, loss_dev, skipped_dev,
                                      (hipStream_t)stream);
    return rc == NRC_OK ? ok() : rc;
}
