// Host runtime of libmecdf: error strings, per-device workspace cache and a
// pinned staging buffer for small host-to-device uploads.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdlib>
#include <map>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "common.hpp"

namespace mecdf {

namespace {
thread_local std::string g_last_error;

struct DeviceState {
    void *ws = nullptr;
    size_t ws_bytes = 0;
    void *pinned = nullptr;
    size_t pinned_bytes = 0;
    hipEvent_t pinned_done = nullptr;
    bool pinned_pending = false;
    // streams beside the caller's (default priority) and their fork / join
    // events
    hipStream_t side[kSideStreams] = {};
    hipEvent_t fork = nullptr;
    hipEvent_t join[kSideStreams] = {};
};

std::mutex g_mu;
std::vector<DeviceState> g_dev;

DeviceState &state(int dev) {
    if ((int)g_dev.size() <= dev)
        g_dev.resize(dev + 1);
    return g_dev[dev];
}

size_t workspace_limit() {
    const char *e = std::getenv("MECDF_WORKSPACE_LIMIT");
    if (!e || !*e)
        return ~size_t(0);
    char *end = nullptr;
    unsigned long long v = std::strtoull(e, &end, 10);
    return (size_t)v;
}
}  // namespace

void set_error(const std::string &msg) { g_last_error = msg; }
const char *last_error() { return g_last_error.c_str(); }

namespace {
thread_local void *t_fixed_ws = nullptr;
thread_local size_t t_fixed_bytes = 0;
thread_local size_t *t_sizing = nullptr;
}  // namespace

void set_fixed_workspace(void *base, size_t bytes) {
    t_fixed_ws = base;
    t_fixed_bytes = bytes;
}

void set_workspace_sizing(size_t *bytes) { t_sizing = bytes; }

int workspace_reserve(size_t bytes, void **base) {
    if (t_sizing) {
        if (bytes > *t_sizing)
            *t_sizing = bytes;
        return kSizingOnly;
    }
    if (t_fixed_ws) {
        if (bytes > t_fixed_bytes) {
            set_error("this call needs " + std::to_string(bytes) +
                      " bytes of working memory; the fixed scratch array of the "
                      "no-allocation entry point holds " +
                      std::to_string(t_fixed_bytes));
            return MECDF_EUNSUPPORTED;
        }
        *base = t_fixed_ws;
        return MECDF_OK;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    int dev = 0;
    MECDF_TRY_HIP(hipGetDevice(&dev));
    DeviceState &st = state(dev);
    if (bytes == 0)
        bytes = 256;
    if (bytes > workspace_limit()) {
        set_error("workspace of " + std::to_string(bytes) +
                  " bytes exceeds MECDF_WORKSPACE_LIMIT");
        return MECDF_ENOMEM;
    }
    if (st.ws_bytes < bytes) {
        if (st.ws) {
            // hipFree waits for the device, so no in-flight call still uses it
            MECDF_TRY_HIP(hipFree(st.ws));
            st.ws = nullptr;
            st.ws_bytes = 0;
        }
        size_t want = bytes + bytes / 8;  // some headroom against regrowth
        if (want > workspace_limit())
            want = bytes;
        hipError_t e = hipMalloc(&st.ws, want);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            st.ws = nullptr;
            set_error("hipMalloc of " + std::to_string(want) +
                      " bytes failed: " + hipGetErrorString(e));
            return MECDF_ENOMEM;
        }
        st.ws_bytes = want;
    }
    *base = st.ws;
    return MECDF_OK;
}

int side_streams(hipStream_t caller, hipStream_t *streams) {
    std::lock_guard<std::mutex> lk(g_mu);
    int dev = 0;
    MECDF_TRY_HIP(hipGetDevice(&dev));
    DeviceState &st = state(dev);
    if (!st.fork) {
        MECDF_TRY_HIP(hipEventCreateWithFlags(&st.fork, hipEventDisableTiming));
        for (int k = 0; k < kSideStreams; ++k) {
            MECDF_TRY_HIP(hipStreamCreateWithFlags(&st.side[k], hipStreamNonBlocking));
            MECDF_TRY_HIP(hipEventCreateWithFlags(&st.join[k], hipEventDisableTiming));
        }
    }
    MECDF_TRY_HIP(hipEventRecord(st.fork, caller));
    for (int k = 0; k < kSideStreams; ++k) {
        MECDF_TRY_HIP(hipStreamWaitEvent(st.side[k], st.fork, 0));
        streams[k] = st.side[k];
    }
    return MECDF_OK;
}

int side_streams_join(hipStream_t caller) {
    std::lock_guard<std::mutex> lk(g_mu);
    int dev = 0;
    MECDF_TRY_HIP(hipGetDevice(&dev));
    DeviceState &st = state(dev);
    for (int k = 0; k < kSideStreams; ++k) {
        MECDF_TRY_HIP(hipEventRecord(st.join[k], st.side[k]));
        MECDF_TRY_HIP(hipStreamWaitEvent(caller, st.join[k], 0));
    }
    return MECDF_OK;
}

// Copies a small host array to device memory in stream order.  The host
// array may be freed as soon as this returns: it is first copied into a
// pinned staging buffer whose previous copy is waited for.
int upload_small(const void *host, size_t bytes, void *dev_dst,
                 hipStream_t stream) {
    if (bytes == 0)
        return MECDF_OK;
    if (t_fixed_ws) {
        // no staging buffer: HIP stages a copy from pageable memory itself
        // and has read the host array when the call returns
        MECDF_TRY_HIP(hipMemcpyAsync(dev_dst, host, bytes, hipMemcpyHostToDevice, stream));
        return MECDF_OK;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    int dev = 0;
    MECDF_TRY_HIP(hipGetDevice(&dev));
    DeviceState &st = state(dev);
    if (st.pinned_pending) {
        MECDF_TRY_HIP(hipEventSynchronize(st.pinned_done));
        st.pinned_pending = false;
    }
    if (st.pinned_bytes < bytes) {
        if (st.pinned)
            MECDF_TRY_HIP(hipHostFree(st.pinned));
        st.pinned = nullptr;
        st.pinned_bytes = 0;
        size_t want = bytes < (1u << 16) ? (1u << 16) : bytes;
        MECDF_TRY_HIP(hipHostMalloc(&st.pinned, want, hipHostMallocDefault));
        st.pinned_bytes = want;
    }
    if (!st.pinned_done)
        MECDF_TRY_HIP(hipEventCreateWithFlags(&st.pinned_done,
                                              hipEventDisableTiming));
    std::memcpy(st.pinned, host, bytes);
    MECDF_TRY_HIP(hipMemcpyAsync(dev_dst, st.pinned, bytes,
                                 hipMemcpyHostToDevice, stream));
    MECDF_TRY_HIP(hipEventRecord(st.pinned_done, stream));
    st.pinned_pending = true;
    return MECDF_OK;
}

// ------------------------------------------------------------- profiling
int flush_read(const void *buf, size_t bytes, hipStream_t s);  // profiling.hip

namespace {
struct ProfRec {
    std::string name;
    hipEvent_t a = nullptr, b = nullptr;
    int dev = 0;
};
std::atomic<bool> g_prof_on{false};
std::atomic<bool> g_prof_cold{false};
std::mutex g_prof_mu;
std::vector<ProfRec> g_prof;
size_t g_prof_used = 0;
// cold mode: a buffer larger than the 256 MB infinity cache, written before
// each timed group (outside its events) so that its inputs come from HBM
constexpr size_t kFlushBytes = size_t(1) << 30;
void *g_flush = nullptr;
int g_flush_dev = -1;
}  // namespace

bool profiling_enabled() { return g_prof_on.load(std::memory_order_relaxed); }

void profile_begin(const char *name, hipStream_t s, int *slot) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess)
        return;
    if (g_prof_used == g_prof.size())
        g_prof.emplace_back();
    ProfRec &r = g_prof[g_prof_used];
    if (r.a && r.dev != dev) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
        r.a = r.b = nullptr;
    }
    if (!r.a) {
        if (hipEventCreate(&r.a) != hipSuccess || hipEventCreate(&r.b) != hipSuccess)
            return;
        r.dev = dev;
    }
    r.name = name;
    if (g_prof_cold.load() && g_flush && g_flush_dev == dev)
        (void)flush_read(g_flush, kFlushBytes, s);
    if (hipEventRecord(r.a, s) != hipSuccess)
        return;
    *slot = (int)g_prof_used++;
}

void profile_end(int slot, hipStream_t s) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (slot < (int)g_prof.size())
        (void)hipEventRecord(g_prof[slot].b, s);
}

void workspace_release_all() {
    std::lock_guard<std::mutex> lk(g_mu);
    int cur = 0;
    (void)hipGetDevice(&cur);
    for (int dev = 0; dev < (int)g_dev.size(); ++dev) {
        DeviceState &st = g_dev[dev];
        if (!st.ws && !st.pinned && !st.pinned_done && !st.fork)
            continue;
        (void)hipSetDevice(dev);
        (void)hipDeviceSynchronize();
        if (st.ws)
            (void)hipFree(st.ws);
        if (st.pinned)
            (void)hipHostFree(st.pinned);
        if (st.pinned_done)
            (void)hipEventDestroy(st.pinned_done);
        if (st.fork) {
            (void)hipEventDestroy(st.fork);
            for (int k = 0; k < kSideStreams; ++k) {
                (void)hipStreamDestroy(st.side[k]);
                (void)hipEventDestroy(st.join[k]);
            }
        }
        st = DeviceState();
    }
    (void)hipSetDevice(cur);
}

}  // namespace mecdf

extern "C" {

int mecdf_profile_enable(int on) {
    std::lock_guard<std::mutex> lk(mecdf::g_prof_mu);
    if (on == 2) {
        int dev = 0;
        MECDF_TRY_HIP(hipGetDevice(&dev));
        if (mecdf::g_flush && mecdf::g_flush_dev != dev) {
            // the buffer of another device: freed with that device current
            int cur = dev;
            (void)hipSetDevice(mecdf::g_flush_dev);
            (void)hipFree(mecdf::g_flush);
            (void)hipSetDevice(cur);
            mecdf::g_flush = nullptr;
        }
        if (!mecdf::g_flush) {
            MECDF_TRY_HIP(hipMalloc(&mecdf::g_flush, mecdf::kFlushBytes));
            MECDF_TRY_HIP(hipMemset(mecdf::g_flush, 0, mecdf::kFlushBytes));
            mecdf::g_flush_dev = dev;
        }
    }
    mecdf::g_prof_cold.store(on == 2);
    mecdf::g_prof_on.store(on != 0);
    return MECDF_OK;
}

void mecdf_profile_reset(void) {
    std::lock_guard<std::mutex> lk(mecdf::g_prof_mu);
    mecdf::g_prof_used = 0;
}

int mecdf_profile_collect(int max, char *names, double *total_ms,
                          int64_t *launches) {
    std::lock_guard<std::mutex> lk(mecdf::g_prof_mu);
    std::map<std::string, std::pair<double, int64_t>> agg;
    std::vector<std::string> order;
    for (size_t i = 0; i < mecdf::g_prof_used; ++i) {
        mecdf::ProfRec &r = mecdf::g_prof[i];
        if (hipEventSynchronize(r.b) != hipSuccess)
            return MECDF_EDEVICE;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess)
            return MECDF_EDEVICE;
        auto it = agg.find(r.name);
        if (it == agg.end()) {
            order.push_back(r.name);
            agg[r.name] = {ms, 1};
        } else {
            it->second.first += ms;
            it->second.second += 1;
        }
    }
    int n = 0;
    for (const std::string &nm : order) {
        if (n >= max)
            break;
        std::snprintf(names + 64 * n, 64, "%s", nm.c_str());
        total_ms[n] = agg[nm].first;
        launches[n] = agg[nm].second;
        ++n;
    }
    return n;
}

}  // extern "C"
