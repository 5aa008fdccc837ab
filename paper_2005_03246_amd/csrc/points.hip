// Points path: generalized ECDF / ESF at the sample points themselves
// (Section 2.2 of Langrene & Warin, arXiv 2005.03246).
//
// The paper's divide-and-conquer (after Bentley) halves the points along one
// coordinate, recurses on both halves, and merges the cross pairs one
// coordinate lower; it excludes the point itself and uses strict
// inequalities, and it is exact only for tie-free data.  Here the result is
// eq. (ECDF) / eq. (ESF) exactly, ties included:
//
//   ranks      per coordinate, order-preserving 64-bit keys of the doubles
//              (-0 == +0) are radix-sorted and turned into dense integer
//              ranks r, equal values sharing a rank; a point with a NaN
//              coordinate is dropped (it dominates nothing and its result is 0).
//   items      every point is a data item (weight y_i) and a query item.
//              ECDF: data and query coordinates are r (<= in every axis).
//              ESF:  x_i > x_j  <=>  r_i >= r_j + 1, so with reversed ranks
//              a = U-1-r (data) and b = U-2-r (query) it becomes a <= b.
//              The count for query q is the weight of the data items i with
//              a_i <= b_q on every axis.
//   order      items sorted by (coordinate 0, type) with data before queries,
//              so "i before q" encodes coordinate 0 (ties included).
//   recursion  level-synchronous, one coordinate per depth m = 1..d-1:
//              * below the last coordinate, pairs inside blocks of kBlockT
//                items are counted by brute force in LDS, which also sorts
//                each block by coordinate m; then sorted blocks of size
//                h = kBlockT, 2 kBlockT, ... are merged pairwise by
//                coordinate m, and each merged block becomes a sub-problem
//                of depth m+1, with a bit recording whether the item came
//                from the left or right half;
//              * at the last coordinate every merge level counts, for each
//                query of the right half, the weight of the left-half data at
//                or below it (a prefix sum carried over the merged runs):
//                levels up to kBlockT in LDS, the others one per launch; the
//                count travels with the item and reaches the result once.
//              A pair is counted at one depth only, by the items being
//              data-left / query-right at every enclosing split.
// Counts are exact int64; weighted sums accumulate in float64 in a fixed
// order, so results are deterministic.
#include <cstdlib>

#include "common.hpp"
#include "radix.hpp"

namespace mecdf {

constexpr int kBlockT = 512;   // items per LDS brute-force block
constexpr int kIdShift = 5;    // idt = id << 5 | side bits (1..4) | type (bit 0)

template <int NC> struct Item {
    uint32_t c[NC];  // coordinates 1..d-1 (ranks, possibly reversed / shifted)
    uint32_t idt;
};

__device__ __forceinline__ uint64_t order_key(double v) {
    if (v == 0.0)
        v = 0.0;  // -0 -> +0
    uint64_t b = (uint64_t)__double_as_longlong(v);
    if (v != v)
        b = 0x7ff8000000000000ull;
    return (b & 0x8000000000000000ull) ? ~b : (b | 0x8000000000000000ull);
}

__global__ __launch_bounds__(256) void k_fp_keys(const double *__restrict__ x,
                                                 int64_t n, int k,
                                                 uint64_t *__restrict__ keys,
                                                 uint32_t *__restrict__ idx,
                                                 uint32_t *__restrict__ drop) {
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n)
        return;
    double v = x[(int64_t)k * n + i];
    keys[i] = order_key(v);
    idx[i] = (uint32_t)i;
    uint32_t nan = (v != v) ? 1u : 0u;
    drop[i] = (k == 0) ? nan : (drop[i] | nan);
}

__global__ __launch_bounds__(256) void k_rank_flags(const uint64_t *__restrict__ keys,
                                                    int64_t n,
                                                    uint32_t *__restrict__ flags) {
    int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= n)
        return;
    flags[p] = (p > 0 && keys[p] != keys[p - 1]) ? 1u : 0u;
}

// dense rank of sorted position p = (number of value changes up to p)
__global__ __launch_bounds__(256) void k_rank_scatter(const uint32_t *__restrict__ flags,
                                                      const uint32_t *__restrict__ excl,
                                                      const uint32_t *__restrict__ idx,
                                                      int64_t n,
                                                      uint32_t *__restrict__ rank,
                                                      uint32_t *__restrict__ U) {
    int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= n)
        return;
    uint32_t r = excl[p] + flags[p];
    rank[idx[p]] = r;
    if (p == n - 1)
        *U = r + 1;
}

// Two item slots per point: 2i data, 2i+1 query.  Inert slots (see below)
// get the largest top key so they sort last.
template <int NC, typename YT>
__global__ __launch_bounds__(256) void k_make_items(
    const uint32_t *__restrict__ rank /*[d][N]*/, const uint32_t *__restrict__ U,
    const uint32_t *__restrict__ drop, const YT *__restrict__ y, int64_t N, int d,
    int survival, uint64_t invalid_key, uint64_t *__restrict__ topkey,
    uint32_t *__restrict__ slot, Item<NC> *__restrict__ items,
    double *__restrict__ W) {
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= N)
        return;
    bool ok = drop[i] == 0u;
    Item<NC> di, qi;
    int64_t a0 = 0, b0 = 0;
    bool qok = ok;
    for (int k = 0; k < d; ++k) {
        int64_t r = rank[(int64_t)k * N + i];
        int64_t a, b;
        if (survival) {
            a = (int64_t)U[k] - 1 - r;
            b = (int64_t)U[k] - 2 - r;
        } else {
            a = r;
            b = r;
        }
        if (b < 0)
            qok = false;
        if (k == 0) {
            a0 = a;
            b0 = b;
        } else if (k - 1 < NC) {
            di.c[k - 1] = (uint32_t)a;
            qi.c[k - 1] = (uint32_t)(b < 0 ? 0 : b);
        }
    }
    for (int k = d - 1; k < NC; ++k) {
        di.c[k] = 0u;
        qi.c[k] = 0u;
    }
    // A point with a NaN coordinate counts for no query: its data item is
    // made a query (it only receives), and its results are discarded in
    // k_points_out, like those of a survival query below every point.  Such
    // items sort after all others (invalid_key) and run through the
    // recursion, so the number of items is 2N whatever the data.
    di.idt = ((uint32_t)i << kIdShift) | (ok ? 0u : 1u);
    qi.idt = ((uint32_t)i << kIdShift) | 1u;
    topkey[2 * i] = ok ? (((uint64_t)a0 << 1) | 0ull) : invalid_key;
    topkey[2 * i + 1] = qok ? (((uint64_t)(b0 < 0 ? 0 : b0) << 1) | 1ull) : invalid_key;
    slot[2 * i] = (uint32_t)(2 * i);
    slot[2 * i + 1] = (uint32_t)(2 * i + 1);
    items[2 * i] = di;
    items[2 * i + 1] = qi;
    if (W) {
        double w = 1.0;
        if constexpr (!std::is_same<YT, NoPayload>::value)
            w = (double)y[i];
        W[2 * i] = ok ? w : 0.0;
        W[2 * i + 1] = 0.0;
    }
}

// ---- queries at arbitrary points (eq. (ECDFdelta)) -----------------------
// The distinct values of axis k in increasing key order: uv[r] = the key of
// dense rank r.
__global__ __launch_bounds__(256) void k_rank_values(const uint32_t *__restrict__ flags,
                                                     const uint32_t *__restrict__ excl,
                                                     const uint64_t *__restrict__ keys,
                                                     int64_t n, uint64_t *__restrict__ uv) {
    int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= n)
        return;
    if (p == 0 || flags[p])
        uv[excl[p] + flags[p]] = keys[p];
}

// The rank a query takes on axis k: data of rank a count for it exactly when
// a <= b, so b = (number of distinct data values <= z, or < z on an axis
// where the query's delta bit asks for the strict inequality) - 1.  A query
// below every data value on some axis (b < 0) or with a NaN coordinate
// counts nothing: it is inert and its result is 0.
__global__ __launch_bounds__(256) void k_query_ranks(const double *__restrict__ z, int64_t Q,
                                                     int d, const uint8_t *__restrict__ delta,
                                                     const uint64_t *__restrict__ uv, int64_t N,
                                                     const uint32_t *__restrict__ U,
                                                     uint32_t *__restrict__ qrank,
                                                     uint8_t *__restrict__ qinert) {
    int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= Q)
        return;
    bool inert = false;
    const uint32_t dl = delta ? delta[q] : 0u;
    for (int k = 0; k < d; ++k) {
        const double v = z[(int64_t)k * Q + q];
        int64_t lo = 0;
        if (v != v) {
            inert = true;
        } else {
            const uint64_t key = order_key(v);
            const bool strict = ((dl >> k) & 1u) != 0u;
            const uint64_t *u = uv + (int64_t)k * N;
            int64_t hi = U[k];
            while (lo < hi) {
                const int64_t mid = (lo + hi) >> 1;
                if (strict ? u[mid] < key : u[mid] <= key)
                    lo = mid + 1;
                else
                    hi = mid;
            }
            if (lo == 0)
                inert = true;
        }
        qrank[(int64_t)k * Q + q] = lo > 0 ? (uint32_t)(lo - 1) : 0u;
    }
    qinert[q] = inert ? 1 : 0;
}

// The double whose order key is k (the inverse of order_key; -0 comes back
// as +0 and every NaN as the one NaN the keys keep).
__device__ __forceinline__ double key_value(uint64_t k) {
    const uint64_t b = (k & 0x8000000000000000ull) ? (k & 0x7fffffffffffffffull) : ~k;
    return __longlong_as_double((long long)b);
}

// Queries at the 2^d corners x_i + delta h of the data points themselves
// (coordinates x_{k,i} + h_k and x_{k,i} - h_k, rounded once): the corner's
// rank on axis k depends only on the dense rank r of x_{k,i}, so it is found
// once per distinct value, by the rule of k_query_ranks (<= for + h, the
// strict < for - h): tab[r] for + h, tab[N + r] for - h, 0xffffffff where no
// data value counts (the query is inert).  Rounding is monotone, so the
// searches of neighbouring values hit neighbouring entries.
constexpr uint32_t kNoRank = 0xffffffffu;
__global__ __launch_bounds__(256) void k_shift_table(const uint64_t *__restrict__ uv,
                                                     const uint32_t *__restrict__ U, int64_t N,
                                                     double h, uint32_t *__restrict__ tab) {
    const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t nu = *U;
    if (r >= nu)
        return;
    const double v = key_value(uv[r]);
#pragma unroll
    for (int side = 0; side < 2; ++side) {
        const double e = side ? v - h : v + h;
        uint32_t out = kNoRank;
        if (e == e) {
            const uint64_t key = order_key(e);
            int64_t lo = 0, hi = nu;
            while (lo < hi) {
                const int64_t mid = (lo + hi) >> 1;
                if (side ? uv[mid] < key : uv[mid] <= key)
                    lo = mid + 1;
                else
                    hi = mid;
            }
            if (lo > 0)
                out = (uint32_t)(lo - 1);
        }
        tab[(int64_t)side * N + r] = out;
    }
}

// Corner t = c N + i of data point i (bit k of c set: x_{k,i} - h_k, the
// strict inequality): its ranks from the tables; a point with a NaN
// coordinate gives inert corners, as a NaN query coordinate does.
__global__ __launch_bounds__(256) void k_query_ranks_shift(const uint32_t *__restrict__ rank,
                                                           const uint32_t *__restrict__ drop,
                                                           int64_t N, int d,
                                                           const uint32_t *__restrict__ tab,
                                                           int64_t Q,
                                                           uint32_t *__restrict__ qrank,
                                                           uint8_t *__restrict__ qinert) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= Q)
        return;
    const int64_t c = t / N, i = t - c * N;
    bool inert = drop[i] != 0u;
    for (int k = 0; k < d; ++k) {
        const uint32_t r = rank[(int64_t)k * N + i];
        const uint32_t e = tab[(int64_t)(2 * k + ((c >> k) & 1)) * N + r];
        inert = inert || e == kNoRank;
        qrank[(int64_t)k * Q + t] = e == kNoRank ? 0u : e;
    }
    qinert[t] = inert ? 1 : 0;
}

// Items of the data (slots 0..N-1) and of the queries (slots N..N+Q-1).  A
// data point with a NaN coordinate and an inert query get the largest top
// key, so they sort after every other item (the data before the queries) and
// no live query counts them.  Data items never write a result, so their id
// field is left 0.
template <int NC, typename YT>
__global__ __launch_bounds__(256) void k_make_items_ext(
    const uint32_t *__restrict__ rank /*[d][N]*/, const uint32_t *__restrict__ drop,
    const YT *__restrict__ y, int64_t N, const uint32_t *__restrict__ qrank /*[d][Q]*/,
    const uint8_t *__restrict__ qinert, int64_t Q, int d, uint64_t invalid_key,
    uint64_t *__restrict__ topkey, uint32_t *__restrict__ slot, Item<NC> *__restrict__ items,
    double *__restrict__ W) {
    int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= N + Q)
        return;
    Item<NC> it;
    const bool data = t < N;
    const int64_t i = data ? t : t - N;
    const uint32_t *r = data ? rank : qrank;
    const int64_t n = data ? N : Q;
    for (int k = 1; k < d && k - 1 < NC; ++k)
        it.c[k - 1] = r[(int64_t)k * n + i];
    for (int k = d - 1; k < NC; ++k)
        it.c[k] = 0u;
    bool ok;
    if (data) {
        ok = drop[i] == 0u;
        it.idt = 0u;
    } else {
        ok = qinert[i] == 0;
        it.idt = ((uint32_t)i << kIdShift) | 1u;
    }
    topkey[t] = ok ? (((uint64_t)r[i] << 1) | (data ? 0ull : 1ull)) : invalid_key;
    slot[t] = (uint32_t)t;
    items[t] = it;
    if (W) {
        double w = 1.0;
        if constexpr (!std::is_same<YT, NoPayload>::value)
            if (data)
                w = (double)y[i];
        W[t] = (data && ok) ? w : 0.0;
    }
}

template <int NC>
__global__ __launch_bounds__(256) void k_gather_items(const uint32_t *__restrict__ perm,
                                                      int64_t n,
                                                      const Item<NC> *__restrict__ in,
                                                      const double *__restrict__ win,
                                                      Item<NC> *__restrict__ out,
                                                      double *__restrict__ wout) {
    int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= n)
        return;
    uint32_t s = perm[p];
    out[p] = in[s];
    if (win)
        wout[p] = win[s];
}

template <int NC>
__device__ __forceinline__ uint64_t item_key(const Item<NC> &it, int m) {
    return ((uint64_t)it.c[m - 1] << 1) | (uint64_t)(it.idt & 1u);
}

// active predicates at depth m: enclosing side bits 1..m-1 all 0 (data) or
// all 1 (query)
__device__ __forceinline__ bool active_data(uint32_t idt, uint32_t mask) {
    return (idt & 1u) == 0u && (idt & mask) == 0u;
}
__device__ __forceinline__ bool active_query(uint32_t idt, uint32_t mask) {
    return (idt & 1u) == 1u && (idt & mask) == mask;
}
inline uint32_t side_mask(int m) { return ((1u << (m - 1)) - 1u) << 1; }

// Pairs inside each block of kBlockT items at depth m: every active query
// adds the weight of the active data placed before it whose coordinates
// m..d-1 are all <= its own (the active data items and weights are first
// compacted in LDS, in block order, so each query scans only them, and the
// number of them before a query is its compaction offset).  The block is then sorted by
// (coordinate m, type, position) with a bitonic network in LDS and written
// back.  (The last coordinate has its own kernel, k_block_count.)
template <int NC, bool kW>
__global__ __launch_bounds__(256) void k_block_brute(Item<NC> *__restrict__ S,
                                                     double *__restrict__ W,
                                                     void *__restrict__ acc_raw, int64_t n,
                                                     int m, uint32_t mask) {
    using AccT = typename std::conditional<kW, double, int64_t>::type;
    constexpr int T = kBlockT;
    static_assert(T == 512, "two items per thread");
    __shared__ Item<NC> sI[T];
    __shared__ double sW[kW ? T : 1];
    __shared__ uint64_t sk[T];
    __shared__ Item<NC> dI[T];
    __shared__ double dW[kW ? T : 1];
    __shared__ uint32_t wt[4];
    const int tid = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * T;
    const int cnt = (int)((n - base) < T ? (n - base) : T);
    for (int t = tid; t < cnt; t += 256) {
        sI[t] = S[base + t];
        if constexpr (kW)
            sW[t] = W[base + t];
    }
    __syncthreads();
    // compact the active data (blocked: thread t owns local items 2t, 2t+1)
    bool fd[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        int li = 2 * tid + u;
        fd[u] = li < cnt && active_data(sI[li].idt, mask);
    }
    const uint32_t off = block_exclusive_scan256<uint32_t>((uint32_t)fd[0] + (uint32_t)fd[1],
                                                           wt, nullptr);
    const uint32_t nbefore[2] = {off, off + (uint32_t)fd[0]};
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        if (fd[u]) {
            dI[nbefore[u]] = sI[2 * tid + u];
            if constexpr (kW)
                dW[nbefore[u]] = sW[2 * tid + u];
        }
    }
    __syncthreads();
    // active queries scan the active data before them
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        int li = 2 * tid + u;
        if (li >= cnt || !active_query(sI[li].idt, mask))
            continue;
        const Item<NC> me = sI[li];
        const uint32_t nb = nbefore[u];
        auto dom = [&](const Item<NC> &J) {
            bool r = true;
#pragma unroll
            for (int q = 0; q < NC; ++q)
                if (q >= m - 1)
                    r = r && (J.c[q] <= me.c[q]);
            return r;
        };
        auto wgt = [&](uint32_t k) -> AccT {
            if constexpr (kW)
                return dW[k];
            else
                return AccT(1);
        };
        AccT sum = AccT(0);
        uint32_t k = 0;
        for (; k + 4 <= nb; k += 4) {
            Item<NC> J[4];
#pragma unroll
            for (int v = 0; v < 4; ++v)
                J[v] = dI[k + v];
#pragma unroll
            for (int v = 0; v < 4; ++v)
                if (dom(J[v]))
                    sum += wgt(k + v);
        }
        for (; k < nb; ++k)
            if (dom(dI[k]))
                sum += wgt(k);
        if (sum != AccT(0))
            reinterpret_cast<AccT *>(acc_raw)[me.idt >> kIdShift] += sum;
    }
    // bitonic sort of (key, local index)
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        int li = tid + u * 256;
        sk[li] = li < cnt ? ((item_key(sI[li], m) << 10) | (uint64_t)li) : ~0ull;
    }
    __syncthreads();
    for (int k = 2; k <= T; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                int i = tid + u * 256;
                int pr = i ^ j;
                if (pr > i) {
                    uint64_t a = sk[i], b = sk[pr];
                    bool asc = (i & k) == 0;
                    if (asc ? (a > b) : (a < b)) {
                        sk[i] = b;
                        sk[pr] = a;
                    }
                }
            }
            __syncthreads();
        }
    }
    // write back in sorted order
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        int r = 2 * tid + u;
        if (r < cnt) {
            int li = (int)(sk[r] & 1023ull);
            S[base + r] = sI[li];
            if constexpr (kW)
                W[base + r] = sW[li];
        }
    }
}

// Merge of aligned sorted blocks of size h into blocks of size 2h by the
// depth-m key (A = left block first on equal keys).  The side bit of depth m
// is set on every output and a copy is written for depth m + 1 (with only the
// last coordinate when NCC == 1).  Each workgroup produces kMpT consecutive
// outputs of one merged block (h >= kMpT / 2).  Two searches on the merge
// diagonal give the A and B ranges feeding the tile, which are staged in LDS;
// each thread finds its own diagonal in LDS and merges four outputs,
// recording where each output comes from; the workgroup then writes the tile
// with coalesced stores.
constexpr int kMpT = 1024;

template <int NC>
__device__ __forceinline__ uint64_t item_key_sel(const Item<NC> &it, int m) {
    // the coordinate m - 1 by bit masks (a chain of selects between the
    // item's fields would be turned into an indexed load from scratch memory)
    uint32_t c = it.c[0];
#pragma unroll
    for (int k = 1; k < NC; ++k) {
        const uint32_t sel = (k == m - 1) ? ~0u : 0u;
        c = (it.c[k] & sel) | (c & ~sel);
    }
    return ((uint64_t)c << 1) | (uint64_t)(it.idt & 1u);
}

// Wave 0 of a merge workgroup: lanes 0..31 search diagonal k0 and lanes
// 32..63 diagonal k1 of the merge of A[0, ha) and B[0, hb), each for the
// smallest i with A[i] ordered after B[k - i - 1] (32 probes per step); the
// A index of each split goes to split[0] / split[1].
template <int NC>
__device__ __forceinline__ void merge_split(const Item<NC> *A, const Item<NC> *B,
                                            int64_t ha, int64_t hb, int64_t k0, int64_t k1,
                                            int m, int64_t *split) {
    const int lane = threadIdx.x & 63;
    const int half = lane >> 5, l = lane & 31;
    const int64_t k = half ? k1 : k0;
    int64_t lo = k - hb > 0 ? k - hb : 0;
    int64_t hi = k < ha ? k : ha;
    const uint64_t hmask = half ? 0xffffffff00000000ull : 0x00000000ffffffffull;
    for (;;) {
        const int64_t span = hi - lo;
        const bool go = span > 0;  // uniform over the half wave
        int64_t step = (span + 31) / 32;
        int64_t q = lo + (int64_t)(l + 1) * step - 1;
        const bool probe = go && q < hi;
        bool after = false;
        if (probe)
            after = item_key_sel(A[q], m) > item_key_sel(B[k - q - 1], m);
        const uint64_t bal = __ballot(probe && after) & hmask;
        const uint64_t any = __ballot(go) & hmask;
        if (any == 0ull)
            break;
        if (go) {
            if (bal) {
                const int f = (__ffsll((unsigned long long)bal) - 1) & 31;
                const int64_t qf = lo + (int64_t)(f + 1) * step - 1;
                hi = qf;
                lo = f == 0 ? lo : lo + (int64_t)f * step;
            } else {
                // every probe below hi said "before": past the last one
                const int64_t nvalid = span / step < 32 ? span / step : 32;
                lo += nvalid * step;
            }
        }
    }
    if (l == 0)
        split[half] = lo;
}

// Each thread merges outputs 4t .. 4t+3 of the tile from the staged keys
// (sk[0, na) the A range, sk[na, na + nb) the B range); src[q] receives the
// staging slot of output q.
__device__ __forceinline__ void merge_local(const uint32_t *sk, int na, int nb,
                                            uint16_t *src) {
    const int tot = na + nb;
    const int dl = 4 * (int)threadIdx.x;
    if (dl >= tot)
        return;
    const uint32_t *ska = sk;
    const uint32_t *skb = sk + na;
    int lo = dl - nb > 0 ? dl - nb : 0;
    int hi = dl < na ? dl : na;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (ska[mid] <= skb[dl - mid - 1])
            lo = mid + 1;
        else
            hi = mid;
    }
    int i = lo, j = dl - lo;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        if (dl + u >= tot)
            break;
        const bool takeA = (j >= nb) || (i < na && ska[i] <= skb[j]);
        src[dl + u] = (uint16_t)(takeA ? i : na + j);
        if (takeA)
            ++i;
        else
            ++j;
    }
}

template <int NC, bool kW, int NCC = NC>
__global__ __launch_bounds__(256) void k_merge_path(
    const Item<NC> *__restrict__ in, const double *__restrict__ win,
    Item<NC> *__restrict__ out, double *__restrict__ wout,
    Item<NCC> *__restrict__ copy, double *__restrict__ wcopy, int64_t n, int64_t h,
    int m) {
    constexpr int kWn = kW ? kMpT : 1;
    __shared__ Item<NC> sI[kMpT];     // A range, then B range
    __shared__ uint32_t sk[kMpT];     // their keys (ranks < 2^31)
    __shared__ double sW[kWn];        // their weights
    __shared__ uint16_t sSrc[kMpT];   // per output: source slot in sI
    __shared__ int64_t sspl[2];
    const int tid = threadIdx.x;
    // consecutive output tiles on one XCD: neighbouring tiles read the ends
    // of each other's input ranges and search near the same diagonals
    const int64_t o0 = xcd_tile(blockIdx.x, gridDim.x) * kMpT;
    const int64_t s = (o0 / (2 * h)) * (2 * h);
    const int64_t ha = (n - s) < h ? (n - s) : h;
    const int64_t hb = (n - s - ha) < h ? (n - s - ha) : h;
    const int64_t k0 = o0 - s;
    const int64_t k1 = k0 + kMpT < ha + hb ? k0 + kMpT : ha + hb;
    if (tid < 64)
        merge_split<NC>(in + s, in + s + ha, ha, hb, k0, k1, m, sspl);
    __syncthreads();
    const int64_t ia0 = sspl[0], ia1 = sspl[1];
    const int64_t jb0 = k0 - ia0, jb1 = k1 - ia1;
    const int na = (int)(ia1 - ia0), nb = (int)(jb1 - jb0);
    const int tot = na + nb;
    for (int t = tid; t < tot; t += 256) {
        const int64_t g = t < na ? s + ia0 + t : s + ha + jb0 + (t - na);
        const Item<NC> it = in[g];
        sI[t] = it;
        sk[t] = (uint32_t)item_key_sel(it, m);
        if constexpr (kW)
            sW[t] = win[g];
    }
    __syncthreads();
    merge_local(sk, na, nb, sSrc);
    __syncthreads();
    const uint32_t bit = 1u << m;
    for (int q = tid; q < tot; q += 256) {
        const int src = sSrc[q];
        const int64_t o = o0 + q;
        Item<NC> it = sI[src];
        it.idt = src < na ? (it.idt & ~bit) : (it.idt | bit);
        if constexpr (NCC == NC) {
            copy[o] = it;
        } else {
            static_assert(NCC == 1, "compact copies keep the last coordinate");
            Item<1> c1;
            c1.c[0] = it.c[NC - 1];
            c1.idt = it.idt;
            copy[o] = c1;
        }
        out[o] = it;
        if constexpr (kW) {
            wout[o] = sW[src];
            wcopy[o] = sW[src];
        }
    }
}

// ---- the last coordinate --------------------------------------------------
// Per item, in merged order: p, the prefix of active data weight up to and
// including the item in its merged block, and c, the weight counted so far
// for the item as an active query.  c travels with the item through the
// merges and is added to the result once, at the last merge (ids are below
// 2^26, so counts fit 32 bits).
template <bool kW> struct PCnt;
template <> struct PCnt<false> {
    uint32_t p, c;
};
template <> struct PCnt<true> {
    double p, c;
};
template <bool kW> using PVal = typename std::conditional<kW, double, uint32_t>::type;
template <bool kW> using AccOf = typename std::conditional<kW, double, int64_t>::type;

// The merge levels of runs of 1, 2, ..., kBlockT/2 items inside each block of
// kBlockT items, in LDS.  Each item finds its rank in the other run by binary
// search (left run first on equal keys); an active query of a right run adds
// the left run's active data weight at or below its key, which is the left
// run's prefix at that rank; every item's prefix grows by the other run's
// prefix at its rank.  The sorted block is written back with its p and c
// (kFlush: the block is the whole sub-problem, and c goes to the result).
template <bool kW, bool kFlush>
__global__ __launch_bounds__(256) void k_block_count(Item<1> *__restrict__ S,
                                                     const double *__restrict__ W,
                                                     PCnt<kW> *__restrict__ PC,
                                                     AccOf<kW> *__restrict__ acc, int64_t n,
                                                     uint32_t mask) {
    using PV = PVal<kW>;
    constexpr int T = kBlockT;
    static_assert(T == 512, "two items per thread");
    __shared__ Item<1> sI[T];
    __shared__ uint32_t sk[2][T];   // keys in run order
    __shared__ uint16_t sx[2][T];   // item slot of each run position
    __shared__ PV sp[2][T];         // prefix of active data weight in the run
    __shared__ PV sc[T];            // count per item slot
    const int tid = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * T;
    const int cnt = (int)((n - base) < T ? (n - base) : T);
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        const int t = tid + u * 256;
        uint32_t key = 0xffffffffu;  // padding sorts last (keys are below 2^28)
        PV w = PV(0);
        if (t < cnt) {
            const Item<1> it = S[base + t];
            sI[t] = it;
            key = (it.c[0] << 1) | (it.idt & 1u);
            if (active_data(it.idt, mask)) {
                if constexpr (kW)
                    w = W[base + t];
                else
                    w = 1u;
            }
        }
        sk[0][t] = key;
        sx[0][t] = (uint16_t)t;
        sp[0][t] = w;
        sc[t] = PV(0);
    }
    __syncthreads();
    int cur = 0;
    // the levels unrolled, so that each search has a fixed number of steps
    // and the two items' searches interleave
#pragma unroll
    for (int len = 1; len < T; len <<= 1) {
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int r = tid + u * 256;
            const int b0 = r & ~(2 * len - 1);
            const bool inA = (r & len) == 0;
            const int ob = inA ? b0 + len : b0;
            const uint32_t key = sk[cur][r];
            // A items count B keys below theirs, B items A keys at or below:
            // the number of keys of the other run (sorted, len of them) that
            // satisfy the test, by halving steps over its first len - 1 and a
            // last look at the key it stops at
            const uint32_t *o = sk[cur] + ob;
            int lo = 0;
#pragma unroll
            for (int step = len >> 1; step > 0; step >>= 1) {
                const uint32_t k2 = o[lo + step - 1];
                if (inA ? (k2 < key) : (k2 <= key))
                    lo += step;
            }
            {
                const uint32_t k2 = o[lo];
                if (inA ? (k2 < key) : (k2 <= key))
                    lo += 1;
            }
            const int slot = sx[cur][r];
            const PV other = lo > 0 ? sp[cur][ob + lo - 1] : PV(0);
            if (!inA && slot < cnt && active_query(sI[slot].idt, mask))
                sc[slot] += other;
            const int dst = b0 + (r & (len - 1)) + lo;
            sk[cur ^ 1][dst] = key;
            sx[cur ^ 1][dst] = (uint16_t)slot;
            sp[cur ^ 1][dst] = sp[cur][r] + other;
        }
        // up to runs of 32, the next level's blocks of 64 items lie in one
        // wavefront's ranges (items w*64.. and 256 + w*64..), which only it
        // reads and writes: its own LDS accesses are ordered, no barrier
        if (len <= 16) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        } else {
            __syncthreads();
        }
        cur ^= 1;
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        const int r = tid + u * 256;
        if (r >= cnt)
            continue;
        if constexpr (kFlush) {
            if (sc[r] != PV(0))
                acc[sI[r].idt >> kIdShift] += (AccOf<kW>)sc[r];
        } else {
            const int slot = sx[cur][r];
            S[base + r] = sI[slot];
            PCnt<kW> v;
            v.p = sp[cur][r];
            v.c = sc[slot];
            PC[base + r] = v;
        }
    }
}

// A merge level of the last coordinate above the LDS blocks (h >= kBlockT):
// the merge of k_merge_path on compact items, carrying p and c.  An output
// from one side has, before it in the merged block, the items of the other
// side up to its tile position minus its index in its range; the other
// side's prefix there is added to its p, and to its c when it is an active
// query from the right side.  kFlush (the last level of the sub-problem):
// nothing is written back and every nonzero c goes to the result.
template <bool kW, bool kFlush>
__global__ __launch_bounds__(256) void k_merge_count(
    const Item<1> *__restrict__ in, const PCnt<kW> *__restrict__ pcin,
    Item<1> *__restrict__ out, PCnt<kW> *__restrict__ pcout, AccOf<kW> *__restrict__ acc,
    int64_t n, int64_t h, uint32_t mask) {
    using PV = PVal<kW>;
    __shared__ Item<1> sI[kMpT];      // A range, then B range
    __shared__ uint32_t sk[kMpT];     // their keys
    __shared__ PCnt<kW> sPC[kMpT];    // their p and c
    __shared__ uint16_t sSrc[kMpT];   // per output: source slot
    __shared__ int64_t sspl[2];
    __shared__ PV sPrev[2];           // p just before the A and the B range
    const int tid = threadIdx.x;
    // consecutive output tiles on one XCD: neighbouring tiles read the ends
    // of each other's input ranges and search near the same diagonals
    const int64_t o0 = xcd_tile(blockIdx.x, gridDim.x) * kMpT;
    const int64_t s = (o0 / (2 * h)) * (2 * h);
    const int64_t ha = (n - s) < h ? (n - s) : h;
    const int64_t hb = (n - s - ha) < h ? (n - s - ha) : h;
    const int64_t k0 = o0 - s;
    const int64_t k1 = k0 + kMpT < ha + hb ? k0 + kMpT : ha + hb;
    if (tid < 64)
        merge_split<1>(in + s, in + s + ha, ha, hb, k0, k1, 1, sspl);
    __syncthreads();
    const int64_t ia0 = sspl[0], ia1 = sspl[1];
    const int64_t jb0 = k0 - ia0, jb1 = k1 - ia1;
    const int na = (int)(ia1 - ia0), nb = (int)(jb1 - jb0);
    const int tot = na + nb;
    for (int t = tid; t < tot; t += 256) {
        const int64_t g = t < na ? s + ia0 + t : s + ha + jb0 + (t - na);
        const Item<1> it = in[g];
        sI[t] = it;
        sk[t] = (it.c[0] << 1) | (it.idt & 1u);
        sPC[t] = pcin[g];
    }
    if (tid == 0)
        sPrev[0] = ia0 > 0 ? pcin[s + ia0 - 1].p : PV(0);
    if (tid == 1)
        sPrev[1] = jb0 > 0 ? pcin[s + ha + jb0 - 1].p : PV(0);
    __syncthreads();
    merge_local(sk, na, nb, sSrc);
    __syncthreads();
    for (int q = tid; q < tot; q += 256) {
        const int src = sSrc[q];
        const Item<1> it = sI[src];
        PCnt<kW> v = sPC[src];
        PV other;
        if (src < na) {
            const int jb = q - src;  // B items before it: jb0 + jb
            other = jb > 0 ? sPC[na + jb - 1].p : sPrev[1];
        } else {
            const int ia = q - (src - na);  // A items before it: ia0 + ia
            other = ia > 0 ? sPC[ia - 1].p : sPrev[0];
            if (active_query(it.idt, mask))
                v.c += other;
        }
        if constexpr (kFlush) {
            if (v.c != PV(0))
                acc[it.idt >> kIdShift] += (AccOf<kW>)v.c;
        } else {
            v.p += other;
            out[o0 + q] = it;
            pcout[o0 + q] = v;
        }
    }
}

// ---- segmented inclusive prefix of active-data weight ---------------------
// Segments are the aligned blocks of size h (a power of two >= kBlockT).
constexpr int kSegItems = 8;
constexpr int kSegTile = 256 * kSegItems;

template <int NC, bool kW, typename T>
__device__ __forceinline__ T seg_value(const Item<NC> *S, const double *W, int64_t p,
                                       int64_t n, uint32_t mask) {
    if (p >= n)
        return T(0);
    if (!active_data(S[p].idt, mask))
        return T(0);
    if constexpr (kW)
        return (T)W[p];
    else
        return T(1);
}

// per tile: sum of the values after the last segment head in the tile, and
// whether the tile holds a head
template <int NC, bool kW, typename T>
__global__ __launch_bounds__(256) void k_seg_tiles(const Item<NC> *__restrict__ S,
                                                   const double *__restrict__ W,
                                                   int64_t n, int64_t h, uint32_t mask,
                                                   T *__restrict__ tagg,
                                                   uint32_t *__restrict__ thead) {
    __shared__ T ws[4];
    __shared__ uint32_t wf[4];
    const int64_t base = (int64_t)blockIdx.x * kSegTile + (int64_t)threadIdx.x * kSegItems;
    T v = T(0);
    uint32_t f = 0;
#pragma unroll
    for (int u = 0; u < kSegItems; ++u) {
        int64_t p = base + u;
        if (p < n && (p % h) == 0) {
            v = T(0);
            f = 1;
        }
        v = v + seg_value<NC, kW, T>(S, W, p, n, mask);
    }
    // segmented reduction across threads: combine (a,fa) then (b,fb)
    const int lane = lane_id();
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        T ov = shfl_up(v, off);
        uint32_t of = (uint32_t)__shfl_up((int)f, off, 64);
        if (lane >= off && !f) {
            v = ov + v;
            f = of;
        } else if (lane >= off) {
            f = f | of;
        }
    }
    const int w = threadIdx.x >> 6;
    if (lane == 63) {
        ws[w] = v;
        wf[w] = f;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        T a = ws[0];
        uint32_t fa = wf[0];
        for (int q = 1; q < 4; ++q) {
            if (wf[q]) {
                a = ws[q];
                fa = 1;
            } else {
                a = a + ws[q];
            }
        }
        tagg[blockIdx.x] = a;
        thead[blockIdx.x] = fa;
    }
}

// carry-in of every tile (exclusive segmented scan over the tiles): one block
// of 1024 threads, each owning a contiguous chunk of tiles
template <typename T>
__global__ __launch_bounds__(1024) void k_seg_carry(T *__restrict__ tagg,
                                                    const uint32_t *__restrict__ thead,
                                                    int64_t nt) {
    __shared__ T ws[16];
    __shared__ uint32_t wf[16];
    const int64_t ch = ceil_div_dev(nt, 1024);
    const int64_t t0 = (int64_t)threadIdx.x * ch;
    const int64_t t1 = t0 + ch < nt ? t0 + ch : nt;
    T v = T(0);
    uint32_t f = 0;
    for (int64_t t = t0; t < t1; ++t) {
        if (thead[t]) {
            v = tagg[t];
            f = 1;
        } else {
            v = v + tagg[t];
        }
    }
    const int lane = lane_id();
    T inc = v;
    uint32_t finc = f;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        T ov = shfl_up(inc, off);
        uint32_t of = (uint32_t)__shfl_up((int)finc, off, 64);
        if (lane >= off) {
            if (!finc)
                inc = ov + inc;
            finc = finc | of;
        }
    }
    const int w = threadIdx.x >> 6;
    if (lane == 63) {
        ws[w] = inc;
        wf[w] = finc;
    }
    __syncthreads();
    T pre = T(0);
    for (int q = 0; q < w; ++q)
        pre = wf[q] ? ws[q] : pre + ws[q];
    T ex = shfl_up(inc, 1);
    uint32_t exf = (uint32_t)__shfl_up((int)finc, 1, 64);
    if (lane == 0)
        ex = pre;
    else if (!exf)
        ex = pre + ex;
    T carry = ex;
    for (int64_t t = t0; t < t1; ++t) {
        T a = tagg[t];
        uint32_t h = thead[t];
        tagg[t] = carry;
        carry = h ? a : carry + a;
    }
}

template <int NC, bool kW, typename T>
__global__ __launch_bounds__(256) void k_seg_apply(const Item<NC> *__restrict__ S,
                                                   const double *__restrict__ W,
                                                   int64_t n, int64_t h, uint32_t mask,
                                                   const T *__restrict__ carry,
                                                   T *__restrict__ P) {
    __shared__ T ws[4];
    __shared__ uint32_t wf[4];
    const int64_t base = (int64_t)blockIdx.x * kSegTile + (int64_t)threadIdx.x * kSegItems;
    T vals[kSegItems];
    T v = T(0);
    uint32_t f = 0;
#pragma unroll
    for (int u = 0; u < kSegItems; ++u) {
        int64_t p = base + u;
        if (p < n && (p % h) == 0) {
            v = T(0);
            f = 1;
        }
        vals[u] = seg_value<NC, kW, T>(S, W, p, n, mask);
        v = v + vals[u];
    }
    // exclusive segmented scan across the block of thread aggregates
    const int lane = lane_id();
    T inc = v;
    uint32_t finc = f;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        T ov = shfl_up(inc, off);
        uint32_t of = (uint32_t)__shfl_up((int)finc, off, 64);
        if (lane >= off) {
            if (!finc)
                inc = ov + inc;
            finc = finc | of;
        }
    }
    const int w = threadIdx.x >> 6;
    if (lane == 63) {
        ws[w] = inc;
        wf[w] = finc;
    }
    __syncthreads();
    // prefix from earlier waves and the tile carry
    T pre = carry[blockIdx.x];
    uint32_t pf = 0;
    for (int q = 0; q < w; ++q) {
        if (wf[q]) {
            pre = ws[q];
            pf = 1;
        } else {
            pre = pre + ws[q];
        }
    }
    T ex = shfl_up(inc, 1);
    uint32_t exf = (uint32_t)__shfl_up((int)finc, 1, 64);
    if (lane == 0) {
        ex = pre;
    } else if (!exf) {
        ex = pre + ex;
    }
    T run = ex;
#pragma unroll
    for (int u = 0; u < kSegItems; ++u) {
        int64_t p = base + u;
        if (p < n) {
            if ((p % h) == 0)
                run = T(0);
            run = run + vals[u];
            P[p] = run;
        }
    }
    (void)pf;
}

// d == 1: the count of query q is the data weight up to its position
template <bool kW, typename T>
__global__ __launch_bounds__(256) void k_d1_collect(const Item<1> *__restrict__ S,
                                                    const T *__restrict__ P, int64_t n,
                                                    void *__restrict__ acc_raw) {
    int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= n)
        return;
    uint32_t idt = S[p].idt;
    if ((idt & 1u) == 1u)
        reinterpret_cast<T *>(acc_raw)[idt >> kIdShift] = P[p];
}

// The result of point i, 0 for a point with a NaN coordinate and, for the
// survival function, for a point at the largest rank of some coordinate (no
// point is strictly above it there).
template <typename OutT, typename AccT>
__global__ __launch_bounds__(256) void k_points_out(const AccT *__restrict__ acc,
                                                    int64_t N, int scale,
                                                    const uint32_t *__restrict__ drop,
                                                    const uint32_t *__restrict__ rank,
                                                    const uint32_t *__restrict__ U, int d,
                                                    int survival, OutT *__restrict__ F) {
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= N)
        return;
    bool zero = drop[i] != 0u;
    if (survival)
        for (int k = 0; k < d; ++k)
            zero = zero || rank[(int64_t)k * N + i] + 1u == U[k];
    if (zero)
        F[i] = (OutT)0;
    else if constexpr (std::is_same<AccT, int64_t>::value)
        F[i] = (OutT)acc[i];
    else
        F[i] = scale ? (OutT)(acc[i] / (double)N) : (OutT)acc[i];
}

// The result of query q (0 for an inert query).
template <typename OutT, typename AccT>
__global__ __launch_bounds__(256) void k_query_out(const AccT *__restrict__ acc, int64_t Q,
                                                   int64_t N, int scale,
                                                   const uint8_t *__restrict__ qinert,
                                                   OutT *__restrict__ F) {
    int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= Q)
        return;
    if (qinert[q])
        F[q] = (OutT)0;
    else if constexpr (std::is_same<AccT, int64_t>::value)
        F[q] = (OutT)acc[q];
    else
        F[q] = scale ? (OutT)(acc[q] / (double)N) : (OutT)acc[q];
}

__global__ void k_zero_u32(uint32_t *a, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n)
        a[i] = 0u;
}
__global__ void k_zero_f64(double *a, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n)
        a[i] = 0.0;
}

// ----------------------------------------------------------- host driver
template <int NC, bool kW> struct Dnc {
    using AccT = AccOf<kW>;
    int d;
    int64_t n;
    hipStream_t s;
    Item<NC> *S[MECDF_MAX_DIM];
    Item<NC> *T[MECDF_MAX_DIM];
    double *SW[MECDF_MAX_DIM];
    double *TW[MECDF_MAX_DIM];
    AccT *acc;
    AccT *P;
    PCnt<kW> *PCa;
    PCnt<kW> *PCb;
    AccT *tagg;
    uint32_t *thead;

    int prefix(int depth, int64_t h, uint32_t mask) {
        Item<NC> *cur = S[depth];
        double *cw = SW[depth];
        int64_t nt = ceil_div(n, kSegTile);
        hipLaunchKernelGGL((k_seg_tiles<NC, kW, AccT>), dim3((unsigned)nt), dim3(256), 0,
                           s, cur, cw, n, h, mask, tagg, thead);
        hipLaunchKernelGGL((k_seg_carry<AccT>), dim3(1), dim3(1024), 0, s, tagg, thead, nt);
        hipLaunchKernelGGL((k_seg_apply<NC, kW, AccT>), dim3((unsigned)nt), dim3(256), 0,
                           s, cur, cw, n, h, mask, tagg, P);
        MECDF_LAUNCH_CHECK();
        return MECDF_OK;
    }

    // The last depth works on compact items (its coordinate and the id/side
    // word) when NC > 1: SL / TL with the weights of SW at that depth.
    Item<1> *SL = nullptr, *TL = nullptr;

    // solves depth `depth` inside aligned blocks of size H of S[depth]
    int solve(int depth, int64_t H) {
        if (depth == d - 1)
            return solve_last(depth, H);
        const uint32_t mask = side_mask(depth);
        static_assert(2 * kBlockT >= kMpT, "every merge uses the merge-path kernel");
        const unsigned nbp = (unsigned)ceil_div(n, kMpT);
        {
            ProfScope prof("points_block_brute", s);
            hipLaunchKernelGGL((k_block_brute<NC, kW>), dim3((unsigned)ceil_div(n, kBlockT)),
                               dim3(256), 0, s, S[depth], SW[depth], (void *)acc, n, depth,
                               mask);
        }
        MECDF_LAUNCH_CHECK();
        for (int64_t h = kBlockT; h < H; h *= 2) {
            if (depth + 1 == d - 1 && NC > 1) {
                ProfScope prof("points_merge", s);
                hipLaunchKernelGGL((k_merge_path<NC, kW, 1>), dim3(nbp), dim3(256), 0, s,
                                   S[depth], SW[depth], T[depth], TW[depth], SL, SW[depth + 1],
                                   n, h, depth);
            } else {
                ProfScope prof("points_merge", s);
                hipLaunchKernelGGL((k_merge_path<NC, kW>), dim3(nbp), dim3(256), 0, s,
                                   S[depth], SW[depth], T[depth], TW[depth], S[depth + 1],
                                   SW[depth + 1], n, h, depth);
            }
            MECDF_LAUNCH_CHECK();
            std::swap(S[depth], T[depth]);
            std::swap(SW[depth], TW[depth]);
            MECDF_TRY(solve(depth + 1, 2 * h));
        }
        return MECDF_OK;
    }

    // the last depth on Item<1> (the compact items, or the items themselves
    // when NC == 1): LDS merges up to kBlockT, then one merge level per launch;
    // the counts reach the result at the last level
    int solve_last(int depth, int64_t H) {
        const uint32_t mask = side_mask(depth);
        Item<1> **L, **Lt;
        if constexpr (NC > 1) {
            L = &SL;
            Lt = &TL;
        } else {
            L = &S[depth];
            Lt = &T[depth];
        }
        const unsigned nbb = (unsigned)ceil_div(n, kBlockT);
        const unsigned nbp = (unsigned)ceil_div(n, kMpT);
        if (H <= kBlockT) {
            ProfScope prof("points_block_count", s);
            hipLaunchKernelGGL((k_block_count<kW, true>), dim3(nbb), dim3(256), 0, s, *L,
                               SW[depth], PCa, acc, n, mask);
            MECDF_LAUNCH_CHECK();
            return MECDF_OK;
        }
        {
            ProfScope prof("points_block_count", s);
            hipLaunchKernelGGL((k_block_count<kW, false>), dim3(nbb), dim3(256), 0, s, *L,
                               SW[depth], PCa, acc, n, mask);
        }
        MECDF_LAUNCH_CHECK();
        for (int64_t h = kBlockT; h < H; h *= 2) {
            if (2 * h >= H) {
                ProfScope prof("points_merge_flush", s);
                hipLaunchKernelGGL((k_merge_count<kW, true>), dim3(nbp), dim3(256), 0, s, *L,
                                   PCa, (Item<1> *)nullptr, (PCnt<kW> *)nullptr, acc, n, h,
                                   mask);
            } else {
                ProfScope prof("points_merge_count", s);
                hipLaunchKernelGGL((k_merge_count<kW, false>), dim3(nbp), dim3(256), 0, s, *L,
                                   PCa, *Lt, PCb, acc, n, h, mask);
                std::swap(*L, *Lt);
                std::swap(PCa, PCb);
            }
            MECDF_LAUNCH_CHECK();
        }
        return MECDF_OK;
    }
};

// Queries at Q arbitrary points (eq. (ECDFdelta)) instead of at the sample
// points: coordinates z[k*Q + q] and per-query delta bit masks (device).
struct ExtQueries {
    int64_t Q;
    const double *z;
    const uint8_t *delta;  // NULL: <= on every axis
    // corners of the data points instead of z and delta: Q = 2^d N queries,
    // corner c of point i at slot c N + i, x_{k,i} - h_k and < where bit k of
    // c is set, x_{k,i} + h_k and <= elsewhere
    bool corners;
    double h[MECDF_MAX_DIM];
};

template <int NC, bool kW, typename YT, typename OutT>
static int points_run_t(int d, int64_t N, const double *x, const YT *y, OutT *F,
                        int survival, const ExtQueries *ext, hipStream_t s) {
    using AccT = AccOf<kW>;
    const int64_t nq = ext ? ext->Q : N;    // result slots
    const int64_t n2 = ext ? N + nq : 2 * N;
    const int depths = d > 1 ? d - 1 : 1;
    ArenaPlan pl;
    pl.add<uint64_t>((size_t)N);           // keys
    pl.add<uint64_t>((size_t)N);
    pl.add<uint64_t>((size_t)N);
    pl.add<uint32_t>((size_t)N);           // idx
    pl.add<uint32_t>((size_t)N);
    pl.add<uint32_t>((size_t)N);
    pl.add<uint32_t>((size_t)N);           // flags
    pl.add<uint32_t>((size_t)N);           // excl
    pl.add<uint32_t>((size_t)N * d);       // ranks
    pl.add<uint32_t>((size_t)N);           // drop
    pl.add<uint32_t>(8);                   // U
    if (ext) {
        pl.add<uint64_t>((size_t)N * d);   // distinct values per axis
        pl.add<uint32_t>((size_t)nq * d);  // query ranks
        pl.add<uint8_t>((size_t)nq);       // inert queries
        if (ext->corners)
            pl.add<uint32_t>((size_t)N * 2 * d);  // corner rank tables
    }
    pl.add<uint64_t>((size_t)n2);          // topkey x3
    pl.add<uint64_t>((size_t)n2);
    pl.add<uint64_t>((size_t)n2);
    pl.add<uint32_t>((size_t)n2);          // slot x3
    pl.add<uint32_t>((size_t)n2);
    pl.add<uint32_t>((size_t)n2);
    pl.add<Item<NC>>((size_t)n2);          // items (slot order)
    if (kW)
        pl.add<double>((size_t)n2);
    for (int q = 0; q < depths; ++q) {
        if (NC > 1 && q + 1 == d - 1) {  // compact items at the last depth
            pl.add<Item<1>>((size_t)n2);
            pl.add<Item<1>>((size_t)n2);
        } else {
            pl.add<Item<NC>>((size_t)n2);
            pl.add<Item<NC>>((size_t)n2);
        }
        if (kW) {
            pl.add<double>((size_t)n2);
            pl.add<double>((size_t)n2);
        }
    }
    pl.add<AccT>((size_t)nq);              // acc
    pl.add<AccT>((size_t)n2);              // P
    pl.add<PCnt<kW>>((size_t)n2);          // p and c at the last depth, x2
    pl.add<PCnt<kW>>((size_t)n2);
    pl.add<AccT>((size_t)ceil_div(n2, kSegTile) + 1);
    pl.add<uint32_t>((size_t)ceil_div(n2, kSegTile) + 1);
    radix_plan(pl, n2);
    void *wsb = nullptr;
    MECDF_TRY(workspace_reserve(pl.used, &wsb));
    Arena a;
    a.base = (char *)wsb;
    uint64_t *k0 = a.take<uint64_t>((size_t)N), *k1 = a.take<uint64_t>((size_t)N),
             *k2 = a.take<uint64_t>((size_t)N);
    uint32_t *i0 = a.take<uint32_t>((size_t)N), *i1 = a.take<uint32_t>((size_t)N),
             *i2 = a.take<uint32_t>((size_t)N);
    uint32_t *flags = a.take<uint32_t>((size_t)N);
    uint32_t *excl = a.take<uint32_t>((size_t)N);
    uint32_t *rank = a.take<uint32_t>((size_t)N * d);
    uint32_t *drop = a.take<uint32_t>((size_t)N);
    uint32_t *U = a.take<uint32_t>(8);
    uint64_t *uv = ext ? a.take<uint64_t>((size_t)N * d) : nullptr;
    uint32_t *qrank = ext ? a.take<uint32_t>((size_t)nq * d) : nullptr;
    uint8_t *qinert = ext ? a.take<uint8_t>((size_t)nq) : nullptr;
    uint32_t *ctab = (ext && ext->corners) ? a.take<uint32_t>((size_t)N * 2 * d) : nullptr;
    uint64_t *tk0 = a.take<uint64_t>((size_t)n2), *tk1 = a.take<uint64_t>((size_t)n2),
             *tk2 = a.take<uint64_t>((size_t)n2);
    uint32_t *sl0 = a.take<uint32_t>((size_t)n2), *sl1 = a.take<uint32_t>((size_t)n2),
             *sl2 = a.take<uint32_t>((size_t)n2);
    Item<NC> *items = a.take<Item<NC>>((size_t)n2);
    double *Wslot = kW ? a.take<double>((size_t)n2) : nullptr;
    Dnc<NC, kW> dnc{};
    dnc.d = d;
    dnc.s = s;
    for (int q = 0; q < depths; ++q) {
        const bool compact = NC > 1 && q + 1 == d - 1;
        if (compact) {
            dnc.SL = a.take<Item<1>>((size_t)n2);
            dnc.TL = a.take<Item<1>>((size_t)n2);
        } else {
            dnc.S[q + 1] = a.take<Item<NC>>((size_t)n2);
            dnc.T[q + 1] = a.take<Item<NC>>((size_t)n2);
        }
        dnc.SW[q + 1] = kW ? a.take<double>((size_t)n2) : nullptr;
        dnc.TW[q + 1] = kW ? a.take<double>((size_t)n2) : nullptr;
    }
    dnc.acc = a.take<AccT>((size_t)nq);
    dnc.P = a.take<AccT>((size_t)n2);
    dnc.PCa = a.take<PCnt<kW>>((size_t)n2);
    dnc.PCb = a.take<PCnt<kW>>((size_t)n2);
    dnc.tagg = a.take<AccT>((size_t)ceil_div(n2, kSegTile) + 1);
    dnc.thead = a.take<uint32_t>((size_t)ceil_div(n2, kSegTile) + 1);
    RadixScratch rs = radix_take(a, n2);

    const unsigned nbN = (unsigned)ceil_div(N, 256);
    // ---- dense ranks per coordinate
    {
        ProfScope prof("points_ranks", s);
        for (int k = 0; k < d; ++k) {
            hipLaunchKernelGGL(k_fp_keys, dim3(nbN), dim3(256), 0, s, x, N, k, k0, i0, drop);
            int which = 0;
            MECDF_TRY((radix_sort_bits<uint64_t, uint32_t>(k0, i0, k1, i1, k2, i2, N, 0, 64,
                                                           rs, s, &which)));
            uint64_t *ks = which == 1 ? k1 : (which == 2 ? k2 : k0);
            uint32_t *is = which == 1 ? i1 : (which == 2 ? i2 : i0);
            hipLaunchKernelGGL(k_rank_flags, dim3(nbN), dim3(256), 0, s, ks, N, flags);
            MECDF_TRY(scan_exclusive_u32(flags, excl, N, rs.bsum, s));
            hipLaunchKernelGGL(k_rank_scatter, dim3(nbN), dim3(256), 0, s, flags, excl, is, N,
                               rank + (size_t)k * N, U + k);
            if (ext)
                hipLaunchKernelGGL(k_rank_values, dim3(nbN), dim3(256), 0, s, flags, excl, ks,
                                   N, uv + (size_t)k * N);
        }
        if (ext && nq > 0 && ext->corners) {
            for (int k = 0; k < d; ++k)
                hipLaunchKernelGGL(k_shift_table, dim3(nbN), dim3(256), 0, s, uv + (size_t)k * N,
                                   U + k, N, ext->h[k], ctab + (size_t)k * 2 * N);
            hipLaunchKernelGGL(k_query_ranks_shift, dim3((unsigned)ceil_div(nq, 256)), dim3(256),
                               0, s, rank, drop, N, d, ctab, nq, qrank, qinert);
        } else if (ext && nq > 0) {
            hipLaunchKernelGGL(k_query_ranks, dim3((unsigned)ceil_div(nq, 256)), dim3(256), 0, s,
                               ext->z, nq, d, ext->delta, uv, N, U, qrank, qinert);
        }
        MECDF_LAUNCH_CHECK();
    }
    // ---- items, sorted by (coordinate 0, type)
    const int kb = bits_for((uint64_t)N) + 1;
    const uint64_t invalid_key = (kb >= 63) ? ~0ull : ((1ull << (kb + 1)) - 1ull);
    if (ext)
        hipLaunchKernelGGL((k_make_items_ext<NC, YT>), dim3((unsigned)ceil_div(n2, 256)),
                           dim3(256), 0, s, rank, drop, y, N, qrank, qinert, nq, d, invalid_key,
                           tk0, sl0, items, Wslot);
    else
        hipLaunchKernelGGL((k_make_items<NC, YT>), dim3(nbN), dim3(256), 0, s, rank, U, drop, y,
                           N, d, survival, invalid_key, tk0, sl0, items, Wslot);
    MECDF_LAUNCH_CHECK();
    int which = 0;
    {
        ProfScope prof("points_topsort", s);
        MECDF_TRY((radix_sort_bits<uint64_t, uint32_t>(tk0, sl0, tk1, sl1, tk2, sl2, n2, 0,
                                                       kb + 1, rs, s, &which)));
    }
    uint32_t *perm = which == 1 ? sl1 : (which == 2 ? sl2 : sl0);
    const int64_t n = n2;  // every item, the inert ones last
    dnc.n = n;
    hipLaunchKernelGGL((k_gather_items<NC>), dim3((unsigned)ceil_div(n > 0 ? n : 1, 256)),
                       dim3(256), 0, s, perm, n, items, Wslot, dnc.S[1], dnc.SW[1]);
    // int64 and double zeros share their bits
    if (nq > 0)
        hipLaunchKernelGGL(k_zero_f64, dim3((unsigned)ceil_div(nq, 256)), dim3(256), 0, s,
                           (double *)dnc.acc, nq);
    MECDF_LAUNCH_CHECK();

    if (n > 0) {
        if (d == 1) {
            // prefix of data weight in (coordinate 0, type) order
            MECDF_TRY(dnc.prefix(1, (int64_t)1 << 62, 0u));
            hipLaunchKernelGGL((k_d1_collect<kW, AccT>), dim3((unsigned)ceil_div(n, 256)),
                               dim3(256), 0, s, (const Item<1> *)dnc.S[1], dnc.P, n,
                               (void *)dnc.acc);
            MECDF_LAUNCH_CHECK();
        } else {
            int64_t H = 1;
            while (H < n)
                H *= 2;
            MECDF_TRY(dnc.solve(1, H));
        }
    }
    if (ext) {
        if (nq > 0)
            hipLaunchKernelGGL((k_query_out<OutT, AccT>), dim3((unsigned)ceil_div(nq, 256)),
                               dim3(256), 0, s, dnc.acc, nq, N, kW ? 1 : 0, qinert, F);
    } else {
        hipLaunchKernelGGL((k_points_out<OutT, AccT>), dim3(nbN), dim3(256), 0, s, dnc.acc, N,
                           kW ? 1 : 0, drop, rank, U, d, survival, F);
    }
    MECDF_LAUNCH_CHECK();
    return MECDF_OK;
}

// ---- direct evaluation for small samples --------------------------------
// eq. (ECDF) / (ESF) as written: every (query, point) pair.  16 queries per
// block; the points are cut into 64 slices, and lane l of wave w takes query
// l mod 16 over slice 4 w + l / 16, 16 points at a time through the wave's
// LDS (each group of 16 lanes reads one address).  The 64 partial results of
// a query are then combined in slice order.  Counts are exact; float64
// weights are summed with Neumaier compensation and float32 weights with
// Kahan compensation, in a fixed order.
constexpr int kDirectWaves = 16;
constexpr int kDirectQ = 16;                      // queries per block
constexpr int kDirectSlices = kDirectWaves * 4;   // point slices per block

template <typename P> struct DirectAcc;
template <> struct DirectAcc<NoPayload> {
    int64_t v = 0;
    __device__ __forceinline__ void add(NoPayload) { ++v; }
    __device__ __forceinline__ void merge(const DirectAcc &o) { v += o.v; }
};
template <> struct DirectAcc<double> {
    double s = 0.0, c = 0.0;
    __device__ __forceinline__ void add(double a) {
        double t = s + a;
        c += fabs(s) >= fabs(a) ? (s - t) + a : (a - t) + s;
        s = t;
    }
    __device__ __forceinline__ void merge(const DirectAcc &o) {
        add(o.s);
        c += o.c;
    }
};
template <> struct DirectAcc<float> {
    KahanF k;
    __device__ __forceinline__ void add(float a) { k.add(a); }
    __device__ __forceinline__ void merge(const DirectAcc &o) {
        k.add(o.k.s);
        k.c += o.k.c;
    }
};

template <int D, typename P, typename OutT>
__global__ __launch_bounds__(kDirectWaves * 64) void k_points_direct(
    const double *__restrict__ x, int64_t n, const P *__restrict__ y,
    OutT *__restrict__ F, int survival) {
    constexpr bool kW = !std::is_same<P, NoPayload>::value;
    __shared__ double sx[kDirectWaves][D][64];
    __shared__ typename std::conditional<kW, P, int>::type sy[kDirectWaves][64];
    __shared__ __attribute__((aligned(16))) char
        part_raw[sizeof(DirectAcc<P>) * kDirectSlices * kDirectQ];
    DirectAcc<P> *part = reinterpret_cast<DirectAcc<P> *>(part_raw);
    const int w = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int qi = lane & (kDirectQ - 1);
    const int sl = lane >> 4;                 // this lane's slice within the wave
    const int g = w * 4 + sl;                 // slice index 0..63
    const int64_t i = (int64_t)blockIdx.x * kDirectQ + qi;
    double q[D];
#pragma unroll
    for (int k = 0; k < D; ++k)
        q[k] = i < n ? x[(int64_t)k * n + i] : 0.0;
    const int64_t per = (n + kDirectSlices - 1) / kDirectSlices;
    const int64_t j0 = (int64_t)g * per < n ? (int64_t)g * per : n;
    const int64_t j1 = j0 + per < n ? j0 + per : n;
    // the four slices of a wave have the same length except at the end
    const int64_t len = j1 - j0;
    DirectAcc<P> acc;
    // the next 16 points of the slice are loaded while the current ones are
    // compared
    double nx[D];
    typename std::conditional<kW, P, int>::type ny{};
    auto load = [&](int64_t t0) {
        const bool v = t0 + qi < len;
        const int64_t j = j0 + t0 + qi;
#pragma unroll
        for (int k = 0; k < D; ++k)
            nx[k] = v ? x[(int64_t)k * n + j] : 0.0;
        if constexpr (kW)
            ny = v ? y[j] : P(0);
    };
    load(0);
    for (int64_t t0 = 0; t0 < per; t0 += 16) {  // uniform over the wave
#pragma unroll
        for (int k = 0; k < D; ++k)
            sx[w][k][lane] = nx[k];
        if constexpr (kW)
            sy[w][lane] = ny;
        wave_lds_fence();
        if (t0 + 16 < per)
            load(t0 + 16);
        const int64_t rem = len - t0;
        const int cnt = rem <= 0 ? 0 : (rem < 16 ? (int)rem : 16);
        const int b = sl * 16;
#pragma unroll
        for (int t = 0; t < 16; ++t) {
            if (t < cnt) {
                bool dom = true;
#pragma unroll
                for (int k = 0; k < D; ++k)
                    dom = dom && (survival ? (sx[w][k][b + t] > q[k]) : (sx[w][k][b + t] <= q[k]));
                if (dom) {
                    if constexpr (kW)
                        acc.add(sy[w][b + t]);
                    else
                        acc.add(NoPayload{});
                }
            }
        }
        wave_lds_fence();
    }
    part[g * kDirectQ + qi] = acc;
    __syncthreads();
    if (threadIdx.x >= kDirectQ || i >= n)
        return;
    DirectAcc<P> r = part[qi];
    for (int q2 = 1; q2 < kDirectSlices; ++q2)
        r.merge(part[q2 * kDirectQ + qi]);
    if constexpr (kW) {
        if constexpr (std::is_same<P, double>::value)
            F[i] = (OutT)((r.s + r.c) / (double)n);
        else
            F[i] = (OutT)((double)r.k.get() / (double)n);
    } else {
        F[i] = (OutT)r.v;
    }
}

template <int D>
static int points_direct_d(int64_t N, const double *x, const void *y, void *F, int survival,
                           int prec, hipStream_t s) {
    const unsigned nb = (unsigned)ceil_div(N, kDirectQ);
    ProfScope prof("points_direct", s);
    if (y == nullptr)
        hipLaunchKernelGGL((k_points_direct<D, NoPayload, int64_t>), dim3(nb),
                           dim3(kDirectWaves * 64), 0, s, x, N, (const NoPayload *)nullptr,
                           (int64_t *)F, survival);
    else if (prec == MECDF_F64)
        hipLaunchKernelGGL((k_points_direct<D, double, double>), dim3(nb),
                           dim3(kDirectWaves * 64), 0, s, x, N, (const double *)y,
                           (double *)F, survival);
    else
        hipLaunchKernelGGL((k_points_direct<D, float, float>), dim3(nb),
                           dim3(kDirectWaves * 64), 0, s, x, N, (const float *)y,
                           (float *)F, survival);
    MECDF_LAUNCH_CHECK();
    return MECDF_OK;
}

// Samples up to this size use the direct evaluation (cost N^2 d); the
// environment variable MECDF_POINTS_DIRECT_MAX overrides it (0: never).  The
// sizes per d are where the two paths took the same time on one MI355X
// (weighted and count calls; the recursion's cost grows with d as
// N log^(d-1) N, the direct one as d N^2).
static int64_t points_direct_max(int d) {
    const char *e = std::getenv("MECDF_POINTS_DIRECT_MAX");
    if (e && *e)
        return (int64_t)std::strtoll(e, nullptr, 10);
    static const int64_t kMax[MECDF_MAX_DIM] = {20000, 24000, 32000, 46000, 80000, 150000};
    return kMax[(d < 1 ? 1 : (d > MECDF_MAX_DIM ? MECDF_MAX_DIM : d)) - 1];
}

template <int NC>
static int points_dispatch(int d, int64_t N, const double *x, const void *y, void *F,
                           int survival, int prec, const ExtQueries *ext, hipStream_t s) {
    if (y == nullptr)
        return points_run_t<NC, false, NoPayload, int64_t>(d, N, x, nullptr, (int64_t *)F,
                                                           survival, ext, s);
    if (prec == MECDF_F64)
        return points_run_t<NC, true, double, double>(d, N, x, (const double *)y,
                                                      (double *)F, survival, ext, s);
    return points_run_t<NC, true, float, float>(d, N, x, (const float *)y, (float *)F,
                                                survival, ext, s);
}

static int points_dispatch_d(int d, int64_t N, const double *x, const void *y, void *F,
                             int survival, int prec, const ExtQueries *ext, hipStream_t s) {
    switch (d) {
    case 1:
    case 2:
        return points_dispatch<1>(d, N, x, y, F, survival, prec, ext, s);
    case 3:
        return points_dispatch<2>(d, N, x, y, F, survival, prec, ext, s);
    case 4:
        return points_dispatch<3>(d, N, x, y, F, survival, prec, ext, s);
    case 5:
        return points_dispatch<4>(d, N, x, y, F, survival, prec, ext, s);
    default:
        return points_dispatch<5>(d, N, x, y, F, survival, prec, ext, s);
    }
}

int points_run(int d, int64_t N, const double *x, const void *y, void *F,
               int survival, int prec, hipStream_t s) {
    if (N > (int64_t(1) << 26)) {
        set_error("the points path supports N <= 2^26");
        return MECDF_EUNSUPPORTED;
    }
    if (N > 0 && N <= points_direct_max(d)) {
        switch (d) {
        case 1: return points_direct_d<1>(N, x, y, F, survival, prec, s);
        case 2: return points_direct_d<2>(N, x, y, F, survival, prec, s);
        case 3: return points_direct_d<3>(N, x, y, F, survival, prec, s);
        case 4: return points_direct_d<4>(N, x, y, F, survival, prec, s);
        case 5: return points_direct_d<5>(N, x, y, F, survival, prec, s);
        default: return points_direct_d<6>(N, x, y, F, survival, prec, s);
        }
    }
    return points_dispatch_d(d, N, x, y, F, survival, prec, nullptr, s);
}

int points_delta_run(int d, int64_t N, const double *x, const void *y, int64_t Q,
                     const double *z, const uint8_t *delta, void *F, int prec, hipStream_t s) {
    if (N > (int64_t(1) << 26) || Q > (int64_t(1) << 26)) {
        set_error("queries at arbitrary points support N <= 2^26 and Q <= 2^26");
        return MECDF_EUNSUPPORTED;
    }
    ExtQueries ext{};
    ext.Q = Q;
    ext.z = z;
    ext.delta = delta;
    return points_dispatch_d(d, N, x, y, F, 0, prec, &ext, s);
}

// eq. (ECDFdelta) at the 2^d corners x_i + delta h of every data point (the
// corner queries of the uniform kernel at the sample points), F[c N + i].
int points_corners_run(int d, int64_t N, const double *x, const void *y, const double *h,
                       void *F, int prec, hipStream_t s) {
    const int64_t Q = N << d;
    if (N > (int64_t(1) << 26) || Q > (int64_t(1) << 26)) {
        set_error("queries at the corners of the points support 2^d N <= 2^26");
        return MECDF_EUNSUPPORTED;
    }
    ExtQueries ext{};
    ext.Q = Q;
    ext.corners = true;
    for (int k = 0; k < d; ++k)
        ext.h[k] = h[k];
    return points_dispatch_d(d, N, x, y, F, 0, prec, &ext, s);
}

}  // namespace mecdf
