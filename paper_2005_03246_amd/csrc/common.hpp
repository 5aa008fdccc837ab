// Shared helpers of libmecdf: status codes, per-device workspace, wave64
// primitives and small numeric types.  gfx950 only (64-lane wavefronts).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <type_traits>

#include "../../include/mecdf.h"

namespace mecdf {

// ------------------------------------------------------------------ errors
void set_error(const std::string &msg);
const char *last_error();

struct Status {
    int code = MECDF_OK;
};

#define MECDF_TRY_HIP(expr)                                                   \
    do {                                                                      \
        hipError_t _e = (expr);                                               \
        if (_e != hipSuccess) {                                               \
            ::mecdf::set_error(std::string(#expr) + ": " +                    \
                               hipGetErrorString(_e));                        \
            return MECDF_EDEVICE;                                             \
        }                                                                     \
    } while (0)

#define MECDF_TRY(expr)                                                       \
    do {                                                                      \
        int _rc = (expr);                                                     \
        if (_rc != MECDF_OK)                                                  \
            return _rc;                                                       \
    } while (0)

#define MECDF_LAUNCH_CHECK()                                                  \
    do {                                                                      \
        hipError_t _e = hipGetLastError();                                    \
        if (_e != hipSuccess) {                                               \
            ::mecdf::set_error(std::string("kernel launch: ") +               \
                               hipGetErrorString(_e));                        \
            return MECDF_EDEVICE;                                             \
        }                                                                     \
    } while (0)

// --------------------------------------------------------------- workspace
// One growing device buffer per device.  A call reserves its total need up
// front and carves it with an Arena.  Growing frees the old buffer, which
// synchronises the device, so buffers of earlier calls are never reused while
// in flight.
int workspace_reserve(size_t bytes, void **base);

// Streams of the current device that run work beside the caller's stream:
// side_streams makes each of them wait for the work enqueued on `caller` so
// far and returns them; side_streams_join makes `caller` wait for everything
// enqueued on them since.  Created on first use (default priority), kept
// until the workspace is released.  Work spread over them must use disjoint
// memory (FixedWorkspace regions).
constexpr int kSideStreams = 8;
int side_streams(hipStream_t caller, hipStream_t *streams);
int side_streams_join(hipStream_t caller);
void workspace_release_all();

// While set (for the calling thread), workspace_reserve hands out this fixed
// region instead of the growing buffer and fails with MECDF_EUNSUPPORTED when
// a call needs more, and upload_small copies straight from the caller's host
// array: nothing is allocated.  Used by the entry points that allocate
// nothing.
void set_fixed_workspace(void *base, size_t bytes);
struct FixedWorkspace {
    FixedWorkspace(void *base, size_t bytes) { set_fixed_workspace(base, bytes); }
    ~FixedWorkspace() { set_fixed_workspace(nullptr, 0); }
};
// The library's fixed device scratch array on the current device, for the
// entry points that allocate nothing.
int noalloc_scratch(void **base, size_t *bytes);

// Sizing: while set for the calling thread, workspace_reserve records the
// largest request in *bytes and returns kSizingOnly, which the drivers pass
// up before launching anything (every driver reserves before its first
// launch).  Never returned through the C ABI.
constexpr int kSizingOnly = 1;
void set_workspace_sizing(size_t *bytes);
int upload_small(const void *host, size_t bytes, void *dev_dst,
                 hipStream_t stream);

// ------------------------------------------------------- kernel profiling
// When enabled (mecdf_profile_enable), each ProfScope records a HIP event
// pair on its stream around the launches it encloses; mecdf_profile_collect
// sums the elapsed times per name.  Disabled, it costs one flag test.
bool profiling_enabled();
void profile_begin(const char *name, hipStream_t s, int *slot);
void profile_end(int slot, hipStream_t s);

struct ProfScope {
    int slot = -1;
    hipStream_t s;
    ProfScope(const char *name, hipStream_t st) : s(st) {
        if (profiling_enabled())
            profile_begin(name, s, &slot);
    }
    ~ProfScope() {
        if (slot >= 0)
            profile_end(slot, s);
    }
};

struct Arena {
    char *base = nullptr;
    size_t cap = 0;
    size_t used = 0;
    template <typename T> T *take(size_t count) {
        size_t off = (used + 255) & ~size_t(255);
        used = off + count * sizeof(T);
        return reinterpret_cast<T *>(base + off);
    }
};

// Sums the sizes the same sequence of take() calls will use.
struct ArenaPlan {
    size_t used = 0;
    template <typename T> void add(size_t count) {
        size_t off = (used + 255) & ~size_t(255);
        used = off + count * sizeof(T);
    }
};

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
__device__ __forceinline__ int64_t ceil_div_dev(int64_t a, int64_t b) {
    return (a + b - 1) / b;
}

inline int bits_for(uint64_t v) {  // number of bits to hold values 0..v
    int b = 0;
    while ((v >> b) != 0)
        ++b;
    return b;
}

// ------------------------------------------------------------- wave64 ops
constexpr int kWave = 64;

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

__device__ __forceinline__ uint64_t lanemask_lt() {
    int l = lane_id();
    return l == 0 ? 0ull : (~0ull >> (64 - l));
}

template <typename T> __device__ __forceinline__ T shfl_xor(T v, int m) {
    if constexpr (sizeof(T) == 8) {
        union {
            T t;
            int i[2];
        } u;
        u.t = v;
        u.i[0] = __shfl_xor(u.i[0], m, 64);
        u.i[1] = __shfl_xor(u.i[1], m, 64);
        return u.t;
    } else {
        union {
            T t;
            int i;
        } u;
        u.t = v;
        u.i = __shfl_xor(u.i, m, 64);
        return u.t;
    }
}

template <typename T> __device__ __forceinline__ T shfl_up(T v, int d) {
    if constexpr (sizeof(T) == 8) {
        union {
            T t;
            int i[2];
        } u;
        u.t = v;
        u.i[0] = __shfl_up(u.i[0], d, 64);
        u.i[1] = __shfl_up(u.i[1], d, 64);
        return u.t;
    } else {
        union {
            T t;
            int i;
        } u;
        u.t = v;
        u.i = __shfl_up(u.i, d, 64);
        return u.t;
    }
}

template <typename T> __device__ __forceinline__ T shfl_down(T v, int d) {
    if constexpr (sizeof(T) == 8) {
        union {
            T t;
            int i[2];
        } u;
        u.t = v;
        u.i[0] = __shfl_down(u.i[0], d, 64);
        u.i[1] = __shfl_down(u.i[1], d, 64);
        return u.t;
    } else {
        union {
            T t;
            int i;
        } u;
        u.t = v;
        u.i = __shfl_down(u.i, d, 64);
        return u.t;
    }
}

// Orders this wavefront's LDS accesses before and after the call (the
// compiler may not move them across it).
__device__ __forceinline__ void wave_lds_fence() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

template <typename T> __device__ __forceinline__ T shfl(T v, int src) {
    if constexpr (sizeof(T) == 8) {
        union {
            T t;
            int i[2];
        } u;
        u.t = v;
        u.i[0] = __shfl(u.i[0], src, 64);
        u.i[1] = __shfl(u.i[1], src, 64);
        return u.t;
    } else {
        union {
            T t;
            int i;
        } u;
        u.t = v;
        u.i = __shfl(u.i, src, 64);
        return u.t;
    }
}

// Inclusive scan across the 64 lanes in a fixed (Hillis-Steele) order, so the
// rounding of floating-point results depends only on the lane values.
template <typename T> __device__ __forceinline__ T wave_inclusive_scan(T v) {
    int l = lane_id();
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        T o = shfl_up(v, off);
        if (l >= off)
            v = v + o;
    }
    return v;
}

// Inclusive suffix scan (sum over lanes >= this lane).
template <typename T> __device__ __forceinline__ T wave_inclusive_suffix(T v) {
    int l = lane_id();
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        T o = shfl_down(v, off);
        if (l + off < 64)
            v = v + o;
    }
    return v;
}

// ------------------------------------------------------ compensated floats
// Kahan-Babuska-Neumaier accumulator used on the MECDF_F32C path.
struct KahanF {
    float s = 0.f, c = 0.f;
    __device__ __forceinline__ void add(float v) {
        float t = s + v;
        if (fabsf(s) >= fabsf(v))
            c += (s - t) + v;
        else
            c += (v - t) + s;
        s = t;
    }
    __device__ __forceinline__ float get() const { return s + c; }
};

}  // namespace mecdf
