// probe.hip -- a plain streaming copy, the practical HBM ceiling against
// which the stencil's achieved bandwidth is read, and the calibration
// kernel for the memory-traffic counters (its bytes are known exactly).

#include "hc_internal.hpp"

namespace hc {
namespace {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Each thread moves four 16-byte words per pass (four loads in flight before
// the first store); stores are non-temporal like the stencil's.
__global__ __launch_bounds__(256) void copy_probe_kernel(
    const u32x4 *__restrict__ src, u32x4 *__restrict__ dst, long long n16) {
    const long long stride = (long long)gridDim.x * 256;
    long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    for (; i + 3 * stride < n16; i += 4 * stride) {
        const u32x4 a = src[i];
        const u32x4 b = src[i + stride];
        const u32x4 c = src[i + 2 * stride];
        const u32x4 d = src[i + 3 * stride];
        __builtin_nontemporal_store(a, dst + i);
        __builtin_nontemporal_store(b, dst + i + stride);
        __builtin_nontemporal_store(c, dst + i + 2 * stride);
        __builtin_nontemporal_store(d, dst + i + 3 * stride);
    }
    for (; i < n16; i += stride) __builtin_nontemporal_store(src[i], dst + i);
}

}  // namespace

hipError_t launch_copy_probe(const void *src, void *dst, size_t bytes,
                             hipStream_t s) {
    const long long n16 = (long long)(bytes / 16);
    if (n16 == 0) return hipSuccess;
    long long nb = (n16 + 4 * 256 - 1) / (4 * 256);
    if (nb > 256 * 32) nb = 256 * 32;  // 32 blocks per CU, grid-stride beyond
    copy_probe_kernel<<<(unsigned)nb, 256, 0, s>>>(
        static_cast<const u32x4 *>(src), static_cast<u32x4 *>(dst), n16);
    return hipGetLastError();
}

}  // namespace hc
