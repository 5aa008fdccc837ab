// Stable least-significant-digit radix sort on integer keys with an optional
// payload, written for 64-lane wavefronts.
//
// One pass sorts by the digit (key >> shift) & (2^bits - 1), bits <= 9:
//   1. k_radix_hist    per-tile digit counts (tile = 4096 keys), tile-major
//   2. offsets         for every (tile, digit): the number of keys with a
//                      smaller digit plus the keys of that digit in earlier
//                      tiles (column sums over chunks of tiles, a scan of the
//                      chunk sums, then a rescan), written back tile-major
//   3. k_radix_scatter per-tile stable ranks (lanes of equal digit found
//                      through per-wave LDS masks), staging of the tile in LDS
//                      in digit order, then coalesced writes
// Stability (equal digits keep their input order) makes the result, and
// everything computed from it, deterministic.
#pragma once

#include "common.hpp"

namespace mecdf {

constexpr int kRadixThreads = 256;
constexpr int kRadixItems = 16;
constexpr int kRadixTile = kRadixThreads * kRadixItems;  // 4096 keys
constexpr int kRadixMaxBits = 9;
constexpr int kRadixMaxDigits = 1 << kRadixMaxBits;

struct NoPayload {};

template <typename K>
__global__ __launch_bounds__(256) void k_radix_hist(const K *__restrict__ keys,
                                                    int64_t n, int shift,
                                                    int bits,
                                                    uint32_t *__restrict__ hist,
                                                    int64_t ntiles) {
    __shared__ uint32_t h[kRadixMaxDigits];
    const int R = 1 << bits;
    for (int i = threadIdx.x; i < R; i += 256)
        h[i] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kRadixTile;
#pragma unroll 4
    for (int it = 0; it < kRadixItems; ++it) {
        int64_t p = base + (int64_t)it * 256 + threadIdx.x;
        if (p < n) {
            uint32_t dg = (uint32_t)(keys[p] >> shift) & (uint32_t)(R - 1);
            atomicAdd(&h[dg], 1u);
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < R; i += 256)
        hist[(int64_t)blockIdx.x * R + i] = h[i];
    (void)ntiles;
}

// ---- per-(tile, digit) offsets from the tile-major count table ------------
constexpr int kOffChunk = 64;  // tiles per chunk

// S[c*R + d] = sum of H[t*R + d] over the tiles t of chunk c
static __global__ __launch_bounds__(256) void k_off_chunks(const uint32_t *__restrict__ H,
                                                    int64_t ntiles, int R,
                                                    uint32_t *__restrict__ S) {
    int64_t nch = ceil_div_dev(ntiles, kOffChunk);
    int64_t id = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (id >= nch * R)
        return;
    int64_t c = id / R;
    int d = (int)(id - c * R);
    int64_t t0 = c * kOffChunk, t1 = t0 + kOffChunk < ntiles ? t0 + kOffChunk : ntiles;
    uint32_t s = 0;
#pragma unroll 16
    for (int64_t t = t0; t < t1; ++t)
        s += H[t * R + d];
    S[id] = s;
}

// Per digit: exclusive scan of the chunk sums (in place), and the digit
// bases B[d] = number of keys with a smaller digit.  One block of 512 threads;
// loads are issued 16 at a time so that they overlap.
template <typename T, int kW>
__device__ __forceinline__ T block_exclusive_scan(T v, T *wtot /*[kW]*/, T *total);

static __global__ __launch_bounds__(512) void k_off_scan(uint32_t *__restrict__ S,
                                                  int64_t nch, int R,
                                                  uint32_t *__restrict__ B) {
    __shared__ uint32_t wt[8];
    const int d = threadIdx.x;
    uint32_t run = 0;
    if (d < R) {
        for (int64_t c0 = 0; c0 < nch; c0 += 16) {
            uint32_t v[16];
#pragma unroll
            for (int u = 0; u < 16; ++u)
                v[u] = c0 + u < nch ? S[(c0 + u) * R + d] : 0u;
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                if (c0 + u < nch)
                    S[(c0 + u) * R + d] = run;
                run += v[u];
            }
        }
    }
    const uint32_t base = block_exclusive_scan<uint32_t, 8>(d < R ? run : 0u, wt, nullptr);
    if (d < R)
        B[d] = base;
}

// H[t*R + d] <- offset of digit d in tile t (in place)
static __global__ __launch_bounds__(256) void k_off_final(uint32_t *__restrict__ H,
                                                   int64_t ntiles, int R,
                                                   const uint32_t *__restrict__ S,
                                                   const uint32_t *__restrict__ B) {
    int64_t nch = ceil_div_dev(ntiles, kOffChunk);
    int64_t id = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (id >= nch * R)
        return;
    int64_t c = id / R;
    int d = (int)(id - c * R);
    int64_t t0 = c * kOffChunk, t1 = t0 + kOffChunk < ntiles ? t0 + kOffChunk : ntiles;
    uint32_t run = S[id] + B[d];
    for (int64_t t = t0; t < t1; t += 16) {
        uint32_t v[16];
#pragma unroll
        for (int u = 0; u < 16; ++u)
            v[u] = t + u < t1 ? H[(t + u) * R + d] : 0u;
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            if (t + u < t1)
                H[(t + u) * R + d] = run;
            run += v[u];
        }
    }
}

// ---- block-wide exclusive scan of the values of kW waves -------------------
template <typename T, int kW>
__device__ __forceinline__ T block_exclusive_scan(T v, T *wtot /*[kW]*/, T *total) {
    const int lane = lane_id();
    const int w = threadIdx.x >> 6;
    T inc = wave_inclusive_scan(v);
    if (lane == 63)
        wtot[w] = inc;
    __syncthreads();
    T off = T(0);
    for (int i = 0; i < w; ++i)
        off = off + wtot[i];
    if (total) {
        T t = T(0);
        for (int i = 0; i < kW; ++i)
            t = t + wtot[i];
        *total = t;
    }
    // exclusive value from the left neighbour (no subtraction: exact for
    // floating-point values too)
    T ex = shfl_up(inc, 1);
    T r = lane == 0 ? off : off + ex;
    __syncthreads();
    return r;
}

// ---- block-wide exclusive scan of 256 thread values (4 waves) -------------
template <typename T>
__device__ __forceinline__ T block_exclusive_scan256(T v, T *wtot /*[4]*/,
                                                    T *total) {
    const int lane = lane_id();
    const int w = threadIdx.x >> 6;
    T inc = wave_inclusive_scan(v);
    if (lane == 63)
        wtot[w] = inc;
    __syncthreads();
    T off = T(0);
    for (int i = 0; i < w; ++i)
        off = off + wtot[i];
    if (total)
        *total = wtot[0] + wtot[1] + wtot[2] + wtot[3];
    // exclusive value from the left neighbour (no subtraction: exact for
    // floating-point values too)
    T ex = shfl_up(inc, 1);
    T r = lane == 0 ? off : off + ex;
    __syncthreads();
    return r;
}

// ---- device-wide exclusive scan of uint32 (reduce, scan sums, apply) -----
constexpr int kScanItems = 8;
constexpr int kScanBlock = 256 * kScanItems;

static __global__ __launch_bounds__(256) void k_scan_reduce(const uint32_t *__restrict__ in,
                                                     int64_t n,
                                                     uint32_t *__restrict__ bsum) {
    __shared__ uint32_t wt[4];
    const int64_t base = (int64_t)blockIdx.x * kScanBlock;
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        int64_t p = base + (int64_t)i * 256 + threadIdx.x;
        if (p < n)
            s += in[p];
    }
    uint32_t tot;
    block_exclusive_scan256<uint32_t>(s, wt, &tot);
    if (threadIdx.x == 0)
        bsum[blockIdx.x] = tot;
}

static __global__ __launch_bounds__(256) void k_scan_sums(uint32_t *__restrict__ bsum,
                                                   int64_t nb) {
    __shared__ uint32_t wt[4];
    uint32_t carry = 0;
    for (int64_t c0 = 0; c0 < nb; c0 += 256) {
        int64_t p = c0 + threadIdx.x;
        uint32_t v = p < nb ? bsum[p] : 0u;
        uint32_t tot;
        uint32_t ex = block_exclusive_scan256<uint32_t>(v, wt, &tot);
        if (p < nb)
            bsum[p] = carry + ex;
        carry += tot;
    }
}

static __global__ __launch_bounds__(256) void k_scan_apply(const uint32_t *__restrict__ in,
                                                    uint32_t *__restrict__ out,
                                                    int64_t n,
                                                    const uint32_t *__restrict__ bsum) {
    __shared__ uint32_t wt[4];
    const int64_t base = (int64_t)blockIdx.x * kScanBlock;
    // blocked arrangement: thread t owns items [t*8, t*8+8)
    uint32_t v[kScanItems];
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        int64_t p = base + (int64_t)threadIdx.x * kScanItems + i;
        v[i] = p < n ? in[p] : 0u;
        s += v[i];
    }
    uint32_t ex = block_exclusive_scan256<uint32_t>(s, wt, nullptr) + bsum[blockIdx.x];
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        int64_t p = base + (int64_t)threadIdx.x * kScanItems + i;
        if (p < n)
            out[p] = ex;
        ex += v[i];
    }
}

inline int scan_exclusive_u32(const uint32_t *in, uint32_t *out, int64_t n,
                              uint32_t *bsum, hipStream_t s) {
    int64_t nb = ceil_div(n, kScanBlock);
    if (nb == 0)
        return MECDF_OK;
    ProfScope ps("scan_u32", s);
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(256), 0, s, in, n, bsum);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(256), 0, s, bsum, nb);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(256), 0, s, in, out, n, bsum);
    MECDF_LAUNCH_CHECK();
    return MECDF_OK;
}

inline size_t scan_bsum_count(int64_t n) { return (size_t)ceil_div(n, kScanBlock) + 1; }

// ---- scatter ---------------------------------------------------------------
constexpr int kScatWaves = 8;
constexpr int kScatThreads = kScatWaves * 64;
constexpr int kScatItems = kRadixTile / kScatThreads;  // 8 keys per thread
static_assert(kScatThreads >= kRadixMaxDigits, "one digit per thread");

// The tile that workgroup b of a launch of nt workgroups works on.  The
// dispatcher hands workgroups to the eight XCDs in turn (b mod 8); here each
// XCD takes a contiguous range of tiles, in order, so that what neighbouring
// tiles write next to each other (the runs of one digit in the radix scatter,
// the row ends of neighbouring column blocks in the axis scans) goes through
// one L2, which merges the cache lines they share instead of sending two
// partial lines to memory.  A bijection of [0, nt) for any nt.  Not for work
// of uneven size (the grid lines): one XCD would get a whole region of long
// lines.
constexpr int kXcds = 8;
__device__ __forceinline__ int64_t xcd_tile(int64_t b, int64_t nt) {
    const int64_t q = nt / kXcds, r = nt % kXcds;
    const int64_t x = b % kXcds, k = b / kXcds;
    return x * q + (x < r ? x : r) + k;
}

template <typename K, typename P>
__global__ __launch_bounds__(kScatThreads) void k_radix_scatter(
    const K *__restrict__ kin, const P *__restrict__ pin, K *__restrict__ kout,
    P *__restrict__ pout, const uint32_t *__restrict__ offs, int64_t n,
    int shift, int bits, int64_t ntiles) {
    constexpr bool kPay = !std::is_same<P, NoPayload>::value;
    constexpr int kPaySize = kPay ? (int)sizeof(P) : 1;
    constexpr int kStage0 = (int)sizeof(K) > kPaySize ? (int)sizeof(K) : kPaySize;
    constexpr int kStage = kStage0 > 8 ? kStage0 : 8;
    __shared__ uint32_t wcnt[kScatWaves][kRadixMaxDigits];
    __shared__ uint32_t loff[kRadixMaxDigits];
    __shared__ uint32_t gbase[kRadixMaxDigits];
    __shared__ uint32_t wt[kScatWaves];
    // one staging buffer: the per-wave peer masks while ranking, then the
    // keys, then the payloads
    __shared__ __attribute__((aligned(16))) char s_stage[kRadixTile * kStage];
    static_assert(kRadixTile * kStage >= kScatWaves * kRadixMaxDigits * 8, "mask space");
    K *s_key = reinterpret_cast<K *>(s_stage);
    P *s_pay = reinterpret_cast<P *>(s_stage);

    const int R = 1 << bits;
    const uint32_t mask = (uint32_t)(R - 1);
    const int tid = threadIdx.x;
    const int w = tid >> 6;
    const int lane = tid & 63;
    const int64_t tile = xcd_tile(blockIdx.x, ntiles);
    const int64_t base = tile * kRadixTile;

    // all global loads first, so that they are in flight together;
    // wave w owns the contiguous run [w*8*64, (w+1)*8*64) of the tile
    K key[kScatItems];
    P pay[kScatItems];
#pragma unroll
    for (int r = 0; r < kScatItems; ++r) {
        int64_t p = base + ((int64_t)(w * kScatItems + r) << 6) + lane;
        bool valid = p < n;
        key[r] = valid ? __builtin_nontemporal_load(kin + p) : K(0);
        if constexpr (kPay)
            pay[r] = valid ? __builtin_nontemporal_load(pin + p) : P();
    }
    if (tid < R) {
#pragma unroll
        for (int q = 0; q < kScatWaves; ++q)
            wcnt[q][tid] = 0;
        gbase[tid] = offs[tile * R + tid];
    }
    __syncthreads();

    // stable rank of each key among the equal digits of its wave, and the
    // per-wave digit counts.  The lanes holding the same digit are found
    // through a per-wave LDS word per digit: cleared by its lanes, then each
    // lane ORs in its own bit, which gives the same mask whatever the order of
    // the ORs.
    uint64_t *wmask = reinterpret_cast<uint64_t *>(s_stage) + (size_t)w * kRadixMaxDigits;
    uint32_t slot[kScatItems];
    const uint64_t lt = lanemask_lt();
#pragma unroll
    for (int r = 0; r < kScatItems; ++r) {
        int64_t p = base + ((int64_t)(w * kScatItems + r) << 6) + lane;
        bool valid = p < n;
        uint32_t dg = (uint32_t)(key[r] >> shift) & mask;
        if (valid)
            wmask[dg] = 0ull;
        wave_lds_fence();
        if (valid)
            atomicOr(reinterpret_cast<unsigned long long *>(wmask + dg), 1ull << lane);
        wave_lds_fence();
        const uint64_t peers = valid ? wmask[dg] : 0ull;
        uint32_t before = valid ? wcnt[w][dg] : 0u;
        uint32_t rk = (uint32_t)__popcll(peers & lt);
        wave_lds_fence();
        if (valid && rk == 0)
            wcnt[w][dg] = before + (uint32_t)__popcll(peers);
        wave_lds_fence();
        slot[r] = valid ? before + rk : 0xffffffffu;
    }
    __syncthreads();

    // per digit (one per thread): offsets of each wave inside the digit's
    // run, then the digits' offsets inside the tile
    uint32_t td = 0;
    if (tid < R) {
#pragma unroll
        for (int q = 0; q < kScatWaves; ++q) {
            uint32_t t = wcnt[q][tid];
            wcnt[q][tid] = td;
            td += t;
        }
    }
    uint32_t tot;
    uint32_t ex = block_exclusive_scan<uint32_t, kScatWaves>(td, wt, &tot);
    if (tid < R)
        loff[tid] = ex;
    __syncthreads();

    // keys to their place in the tile (digit order, stable)
#pragma unroll
    for (int r = 0; r < kScatItems; ++r) {
        if (slot[r] != 0xffffffffu) {
            uint32_t dg = (uint32_t)(key[r] >> shift) & mask;
            slot[r] += loff[dg] + wcnt[w][dg];
            s_key[slot[r]] = key[r];
        }
    }
    __syncthreads();

    // coalesced runs out; remember each destination for the payloads
    uint32_t dst[kScatItems];
#pragma unroll
    for (int i = 0; i < kScatItems; ++i) {
        uint32_t q = (uint32_t)(tid + kScatThreads * i);
        dst[i] = 0xffffffffu;
        if (q < tot) {
            K kk = s_key[q];
            uint32_t dg = (uint32_t)(kk >> shift) & mask;
            dst[i] = gbase[dg] + (q - loff[dg]);
            kout[dst[i]] = kk;
        }
    }
    if constexpr (kPay) {
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kScatItems; ++r)
            if (slot[r] != 0xffffffffu)
                s_pay[slot[r]] = pay[r];
        __syncthreads();
#pragma unroll
        for (int i = 0; i < kScatItems; ++i) {
            uint32_t q = (uint32_t)(tid + kScatThreads * i);
            if (q < tot)
                pout[dst[i]] = s_pay[q];
        }
    }
}

// All per-(tile, digit) offsets in one workgroup, for at most kOffSmall
// tiles: thread d walks digit d's column of the tile-major count table
// (exclusive running sum), the digit totals are scanned across the
// workgroup, and the digit bases are added in a second walk.
constexpr int kOffSmall = 64;
static __global__ __launch_bounds__(512) void k_off_small(uint32_t *__restrict__ H, int64_t nt,
                                                          int R) {
    __shared__ uint32_t wt[8];
    const int d = threadIdx.x;
    uint32_t run = 0;
    if (d < R) {
        for (int64_t t0 = 0; t0 < nt; t0 += 16) {
            uint32_t v[16];
#pragma unroll
            for (int u = 0; u < 16; ++u)
                v[u] = t0 + u < nt ? H[(t0 + u) * R + d] : 0u;
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                if (t0 + u < nt)
                    H[(t0 + u) * R + d] = run;
                run += v[u];
            }
        }
    }
    const uint32_t base = block_exclusive_scan<uint32_t, 8>(d < R ? run : 0u, wt, nullptr);
    if (d < R)
        for (int64_t t = 0; t < nt; ++t)
            H[t * R + d] += base;
}

// Workspace needed by radix_sort for n keys.
inline size_t radix_bsum_count(int64_t n) {
    int64_t nt = ceil_div(n, kRadixTile);
    return (size_t)(ceil_div(nt, kOffChunk) * kRadixMaxDigits) +
           scan_bsum_count(nt * kRadixMaxDigits);
}

inline void radix_plan(ArenaPlan &pl, int64_t n) {
    int64_t nt = ceil_div(n, kRadixTile);
    pl.add<uint32_t>((size_t)(nt * kRadixMaxDigits));
    pl.add<uint32_t>(radix_bsum_count(n));
}

struct RadixScratch {
    uint32_t *hist = nullptr;
    uint32_t *bsum = nullptr;
};

inline RadixScratch radix_take(Arena &a, int64_t n) {
    int64_t nt = ceil_div(n, kRadixTile);
    RadixScratch r;
    r.hist = a.take<uint32_t>((size_t)(nt * kRadixMaxDigits));
    r.bsum = a.take<uint32_t>(radix_bsum_count(n));
    return r;
}

// One stable pass from (kin, pin) to (kout, pout).
// hist_ready: the producer of kin already wrote the per-tile digit counts of
// this pass into rs.hist (tile-major, 1 << bits entries per tile).
template <typename K, typename P>
int radix_pass(const K *kin, const P *pin, K *kout, P *pout, int64_t n,
               int shift, int bits, const RadixScratch &rs, hipStream_t s,
               bool hist_ready = false) {
    if (n <= 0)
        return MECDF_OK;
    int64_t nt = ceil_div(n, kRadixTile);
    int R = 1 << bits;
    if (!hist_ready) {
        ProfScope ps("radix_hist", s);
        hipLaunchKernelGGL(k_radix_hist<K>, dim3((unsigned)nt), dim3(256), 0, s,
                           kin, n, shift, bits, rs.hist, nt);
    }
    if (nt <= kOffSmall) {
        ProfScope ps("radix_offsets", s);
        hipLaunchKernelGGL(k_off_small, dim3(1), dim3(512), 0, s, rs.hist, nt, R);
    } else {
        ProfScope ps("radix_offsets", s);
        int64_t nch = ceil_div(nt, kOffChunk);
        unsigned nb = (unsigned)ceil_div(nch * R, 256);
        hipLaunchKernelGGL(k_off_chunks, dim3(nb), dim3(256), 0, s, rs.hist, nt, R,
                           rs.bsum);
        uint32_t *B = rs.bsum + nch * R;
        hipLaunchKernelGGL(k_off_scan, dim3(1), dim3(512), 0, s, rs.bsum, nch, R, B);
        hipLaunchKernelGGL(k_off_final, dim3(nb), dim3(256), 0, s, rs.hist, nt, R,
                           rs.bsum, B);
    }
    {
        ProfScope ps("radix_scatter", s);
        hipLaunchKernelGGL((k_radix_scatter<K, P>), dim3((unsigned)nt), dim3(kScatThreads), 0,
                           s, kin, pin, kout, pout, rs.hist, n, shift, bits, nt);
    }
    MECDF_LAUNCH_CHECK();
    return MECDF_OK;
}

// Stable sort by key bits [lo, hi).  Data start in (k0, p0) (which may be a
// read-only input when it is not one of the ping-pong buffers: pass
// inputs_readonly = true) and ping-pong between (k1, p1) and (k2, p2).  On
// return *which is 0, 1 or 2: the buffer pair holding the sorted result.
template <typename K, typename P>
int radix_sort_bits(const K *k0, const P *p0, K *k1, P *p1, K *k2, P *p2,
                    int64_t n, int lo, int hi, const RadixScratch &rs,
                    hipStream_t s, int *which, bool first_hist_ready = false) {
    const K *ck = k0;
    const P *cp = p0;
    int cur = 0;
    for (int b = lo; b < hi; b += kRadixMaxBits) {
        int bits = hi - b < kRadixMaxBits ? hi - b : kRadixMaxBits;
        K *nk = (cur == 1) ? k2 : k1;
        P *np = (cur == 1) ? p2 : p1;
        MECDF_TRY((radix_pass<K, P>(ck, cp, nk, np, n, b, bits, rs, s,
                                    first_hist_ready && b == lo)));
        cur = (cur == 1) ? 2 : 1;
        ck = nk;
        cp = np;
    }
    *which = cur;
    return MECDF_OK;
}

}  // namespace mecdf
