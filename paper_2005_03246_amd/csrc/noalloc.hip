// Working memory of the entry points that allocate nothing: a fixed array in
// the library's device code object, one copy per device, kept until the
// process ends.
#include <mutex>
#include <vector>

#include "common.hpp"

namespace mecdf {

static __device__ __align__(256) unsigned char scratch[MECDF_NOALLOC_SCRATCH_BYTES];

namespace {
std::mutex g_scratch_mu;
std::vector<void *> g_scratch_ptr;  // per device: the array's address there
}  // namespace

// The array's device address on the current device, looked up once per
// device with that device current (each device holds its own copy).  The
// array's name in host code is only a handle for this lookup.
int noalloc_scratch(void **base, size_t *bytes) {
    int dev = 0;
    MECDF_TRY_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if ((int)g_scratch_ptr.size() <= dev)
        g_scratch_ptr.resize(dev + 1, nullptr);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || p == nullptr) {
            set_error(std::string("hipGetSymbolAddress of the scratch array failed: ") +
                      hipGetErrorString(e));
            return MECDF_EDEVICE;
        }
        g_scratch_ptr[dev] = p;
    }
    *base = g_scratch_ptr[dev];
    *bytes = MECDF_NOALLOC_SCRATCH_BYTES;
    return MECDF_OK;
}

}  // namespace mecdf
