// Streaming copy: the measured HBM ceiling that the property kernels' traffic is compared
// with, beside the 8 TB/s specification.  One workgroup per 16 KB chunk (no grid-stride
// loop): each lane moves four 16-byte vectors, 4 KB apart, issued together, with
// non-temporal hints on both sides (the data is touched once).  Measured on MI355X over 1 GiB:
// 6.3 TB/s, against 4.2-5.2 TB/s for persistent grid-stride variants and 5.1 TB/s for a
// device-to-device hipMemcpy.

#include <hip/hip_runtime.h>

#include <cstdint>

#include "props_internal.hpp"

namespace props {

namespace {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
constexpr int kCopyThreads = 256;
constexpr int kCopyUnroll = 4;

__global__ __launch_bounds__(kCopyThreads) void stream_copy_kernel(const u32x4 *__restrict__ src,
                                                                   u32x4 *__restrict__ dst, int64_t nvec)
{
    const int64_t base = (int64_t)blockIdx.x * (kCopyThreads * kCopyUnroll) + threadIdx.x;
    u32x4 v[kCopyUnroll];
#pragma unroll
    for (int u = 0; u < kCopyUnroll; u++)
        if (base + u * kCopyThreads < nvec) v[u] = __builtin_nontemporal_load(src + base + u * kCopyThreads);
#pragma unroll
    for (int u = 0; u < kCopyUnroll; u++)
        if (base + u * kCopyThreads < nvec) __builtin_nontemporal_store(v[u], dst + base + u * kCopyThreads);
}

__global__ void stream_copy_bytes_kernel(const unsigned char *src, unsigned char *dst, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

}  // namespace

}  // namespace props

extern "C" int props_stream_copy(const void *src, void *dst, size_t bytes, void *hip_stream)
{
    using namespace props;
    if (bytes == 0) return PROPS_OK;
    if (!src || !dst) return fail(PROPS_EINVAL, "props_stream_copy: null pointer");
    if ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) & 15u)
        return fail(PROPS_EINVAL, "props_stream_copy: pointers must be 16-byte aligned");
    hipStream_t s = (hipStream_t)hip_stream;
    const int64_t nvec = (int64_t)(bytes / 16);
    if (nvec > 0) {
        const int64_t blocks = (nvec + kCopyThreads * kCopyUnroll - 1) / (kCopyThreads * kCopyUnroll);
        // a dispatch holds at most 2^32 - 1 work-items: 2^24 - 1 workgroups of 256
        if (blocks > 0xffffff) return fail(PROPS_ETOOBIG, "props_stream_copy: %zu bytes in one call", bytes);
        hipLaunchKernelGGL(stream_copy_kernel, dim3((unsigned)blocks), dim3(kCopyThreads), 0, s,
                           static_cast<const u32x4 *>(src), static_cast<u32x4 *>(dst), nvec);
    }
    const int64_t tail = (int64_t)(bytes - (size_t)nvec * 16);
    if (tail > 0)
        hipLaunchKernelGGL(stream_copy_bytes_kernel, dim3(1), dim3(64), 0, s,
                           static_cast<const unsigned char *>(src) + nvec * 16,
                           static_cast<unsigned char *>(dst) + nvec * 16, tail);
    PROPS_HIP_TRY(hipGetLastError());
    return PROPS_OK;
}
