// pb_stream.hip -- plain device copy used to measure the HBM bandwidth a
// streaming kernel attains on this GPU (the denominator the stencil kernels
// are compared with, next to the datasheet peak).
#include <algorithm>

#include "pb_common.h"

namespace pb {

// each thread moves one 16-byte word; consecutive lanes touch consecutive
// words (fully coalesced), one pass over the data (no grid-stride loop).
// Measured on MI355X against 2, 4 and 8 words per thread and grid-stride
// forms: the one-word form streams fastest (about 6.3-6.4 TB/s for 512 MiB
// each way, against 5.6-5.9 for four words per thread).
__global__ __launch_bounds__(256) void stream_copy_kernel(const double2 *__restrict__ src, double2 *__restrict__ dst,
                                                          long long n)
{
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i < n) {
        const double2 v = src[i];
        __builtin_nontemporal_store(v.x, &dst[i].x);
        __builtin_nontemporal_store(v.y, &dst[i].y);
    }
}

}  // namespace pb

extern "C" pb_status pb_stream_copy(const void *src, void *dst, size_t bytes, void *stream)
{
    PB_API_BEGIN
    if (!src || !dst || bytes == 0 || (bytes % 32) != 0 || ((uintptr_t)src % 32) || ((uintptr_t)dst % 32)) {
        pb::set_error("pb_stream_copy: src, dst non-NULL, 32-byte aligned; bytes a positive multiple of 32");
        return PB_EINVAL;
    }
    const long long n = (long long)(bytes / 16);
    const long long blocks = (n + 255) / 256;
    if (blocks > 0x7fffffffll) { pb::set_error("pb_stream_copy: too large"); return PB_EINVAL; }
    hipLaunchKernelGGL(pb::stream_copy_kernel, dim3((unsigned)blocks), dim3(256), 0, static_cast<hipStream_t>(stream),
                       static_cast<const double2 *>(src), static_cast<double2 *>(dst), n);
    PB_HIP(hipGetLastError());
    return PB_OK;
    PB_API_END
}
