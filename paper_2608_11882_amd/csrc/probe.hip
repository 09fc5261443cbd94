// probe.hip -- a plain streaming copy, the practical HBM ceiling against
// which the stencil's achieved bandwidth is read, and the calibration
// kernel for the memory-traffic counters (its bytes are known exactly).

#include "hc_internal.hpp"

namespace hc {
namespace {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// One 16-byte word per thread, consecutive threads on consecutive words and
// one block per 4 KiB: a grid of many short-lived blocks keeps every CU's
// load queue full without a grid-stride loop (which sends the loads of one
// thread to addresses megabytes apart).  Stores are non-temporal like the
// stencil's.  On MI355X this form measured fastest among contiguous and
// grid-stride copies of 1-16 words per thread, 256-1024 threads per block,
// with and without non-temporal loads.
__global__ __launch_bounds__(256) void copy_probe_kernel(
    const u32x4 *__restrict__ src, u32x4 *__restrict__ dst, long long n16) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i < n16) __builtin_nontemporal_store(src[i], dst + i);
}

}  // namespace

hipError_t launch_copy_probe(const void *src, void *dst, size_t bytes,
                             hipStream_t s) {
    const long long n16 = (long long)(bytes / 16);
    // a launch covers at most 2^32 - 256 work-items (the grid's x range)
    constexpr long long kMaxWords = (0xffffffffLL / 256) * 256;
    const u32x4 *a = static_cast<const u32x4 *>(src);
    u32x4 *b = static_cast<u32x4 *>(dst);
    for (long long w0 = 0; w0 < n16; w0 += kMaxWords) {
        const long long n = n16 - w0 < kMaxWords ? n16 - w0 : kMaxWords;
        copy_probe_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(a + w0, b + w0, n);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace hc
