// Benchmark support (not part of the method): a read pass over a buffer
// larger than the infinity cache, run before a timed kernel group in the
// "cold" timing mode so that the group's inputs are read from HBM.  Reading
// (rather than writing) leaves clean lines behind, so the timed group pays no
// write-backs for it.
#include "common.hpp"

namespace mecdf {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_flush_read(const u32x4 *__restrict__ a, int64_t n,
                                                    unsigned int *__restrict__ sink) {
    unsigned int acc = 0u;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * 256) {
        const u32x4 v = a[i];
        acc ^= v.x ^ v.y ^ v.z ^ v.w;
    }
    if (acc == 0x9e3779b9u)  // keeps the loads; almost never true
        sink[threadIdx.x] = acc;
}

int flush_read(const void *buf, size_t bytes, hipStream_t s) {
    const int64_t n = (int64_t)(bytes / 16) - 64;  // the last 1 KiB is the sink
    hipLaunchKernelGGL(k_flush_read, dim3(4096), dim3(256), 0, s, (const u32x4 *)buf, n,
                       (unsigned int *)((char *)buf + bytes - 1024));
    MECDF_LAUNCH_CHECK();
    return MECDF_OK;
}

}  // namespace mecdf
