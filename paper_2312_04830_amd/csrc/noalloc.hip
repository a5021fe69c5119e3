// props_dnn_noalloc: the surrogate with PR fallback for callers that cannot allocate device
// memory (code under HIP graph capture, tight serving loops, harnesses that forbid
// hipMalloc).  The only device scratch of the surrogate call is its list of cells to
// recompute (a count and up to n indices); here it lives in a static device array of the
// library instead of a buffer of the network handle.
#include <mutex>

#include "props_internal.hpp"
#include "trace.hpp"

namespace {

// Word 0: the count; words 64..: the cell indices (the list starts 256 bytes in).  Each
// device the library runs on holds its own copy until the process ends.
constexpr int64_t kListOffset = 64;
__device__ __attribute__((aligned(256))) int scratch[kListOffset + PROPS_DNN_NOALLOC_MAX_CELLS];

// Device address of `scratch` on each device, taken once with that device current.  In host
// code the array's name is only a host-side stand-in; kernels get this address.
constexpr int kMaxDevices = 64;
std::mutex g_mu;
int *g_ptr[kMaxDevices] = {};

int scratch_on(int dev, int **out)
{
    if (dev < 0 || dev >= kMaxDevices) return props::fail(PROPS_EINVAL, "props_dnn_noalloc: device %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return props::fail(PROPS_EHIP, "props_dnn_noalloc: hipGetSymbolAddress(scratch) on device %d: %s", dev,
                               hipGetErrorString(e));
        g_ptr[dev] = static_cast<int *>(p);
    }
    *out = g_ptr[dev];
    return PROPS_OK;
}

}  // namespace

extern "C" int props_dnn_noalloc(props_dnn_t d, props_mech_t fb, const props_in *in, const props_out *out, int64_t n,
                                 uint8_t *status, void *hip_stream)
{
    props::ApiRange range_("props_dnn_noalloc");
    if (!d || !in || !out) return props::fail(PROPS_EINVAL, "props_dnn_noalloc: null network, input or output");
    if (n < 0) return props::fail(PROPS_EINVAL, "props_dnn_noalloc: n < 0");
    if (n > PROPS_DNN_NOALLOC_MAX_CELLS)
        return props::fail(PROPS_ETOOBIG, "props_dnn_noalloc: n = %lld exceeds the static fallback list of %d cells",
                           (long long)n, PROPS_DNN_NOALLOC_MAX_CELLS);
    if (n == 0) return PROPS_OK;
    int dev = -1;
    PROPS_HIP_TRY(hipGetDevice(&dev));
    if (dev != props::dnn_device(d) || (fb && fb->device != dev))
        return props::fail(PROPS_EINVAL, "props_dnn_noalloc: call with the device of the network (and mechanism) current");
    int *list = nullptr;
    if (fb) {
        const int rc = scratch_on(dev, &list);
        if (rc) return rc;
    }
    // dnn_eval resets the count with a kernel on hip_stream before the forward appends to it
    return props::dnn_eval(d, fb, in, out, n, n, status, fb ? list + kListOffset : nullptr, fb ? list : nullptr,
                           (hipStream_t)hip_stream);
}
