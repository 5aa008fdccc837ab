// Kernel path: Laplacian kernel density estimation and Nadaraya-Watson
// regression at the sample points, with leave-one-out CV scores (Section 3.1
// and Appendix D of Langrene & Warin, arXiv 2005.03246).
//
// eq. (Laplacian_decomposition_nD) writes the kernel sum at z as 2^d
// generalized ECDFs, one per sign orthant delta, with weights
// w_i exp(sum_k delta_k x_{k,i} / h_k) and a factor exp(-sum_k delta_k z_k / h_k).
// Appendix D evaluates all orthants in one divide-and-conquer over the points.
// The GPU version keeps that structure, one split coordinate per depth:
//
//   * points sorted by x1 once; blocks of 64 consecutive points (one
//     wavefront) are sorted by the next coordinate in registers; pairs inside
//     a block are summed directly;
//   * merge levels h = 64, 128, ...: sorted blocks A (left in x1) and B are
//     merged by the next coordinate.  For a pair (i in A, j in B),
//     x1_i <= c <= x1_j with c the first x1 of B, so the x1 factor splits as
//     exp(-(c - x1_i)/h1) * exp(-(x1_j - c)/h1), both <= 1.
//   * d = 2: along the merged x2 order the x2 factor is a product of the
//     decays exp(-(x2_p - x2_{p-1})/h2) between neighbours.  A forward scan
//     (orthants with delta_2 = +1) and a backward scan (delta_2 = -1) of the
//     decayed sums, per side, give every item its kernel sum over the other
//     side: B items collect the delta_1 = +1 orthants from A, A items the
//     delta_1 = -1 orthants from B.
//   * d = 3: each merged block of the x1 levels (items tagged A or B, sorted
//     by x2) is itself split the same way on x2 (inner levels, split point c2,
//     64-blocks sorted by x3, merges by x3), and the scans run over x3 with
//     four running sums, one per (x1 side, x2 side); an item collects the sums
//     whose sides differ from its own in both coordinates.  Pairs in the same
//     inner 64-block are summed directly when their x1 sides differ.
//   Every factor is at most 1, so the exponential weights of the decomposition
//   never overflow (their orthant shifts are the local split points), and each
//   unordered pair is counted exactly once, where it splits.
//   * the merge structure does not depend on h: it is built once per call and
//     stored; each batch of bandwidths only runs the scans, adding level
//     contributions into an accumulator kept in the level's order and moved
//     down level by level through the stored merge maps (monotone streams).
//
// d = 1 is the same scan over the sorted sample (the two-sided recursion of
// the 1-D decomposition).  The sums exclude the point itself (leave-one-out);
// the full estimate adds w_j K(0).
#include <vector>

#include "common.hpp"
#include "lse.hpp"
#include "radix.hpp"

namespace mecdf {

constexpr int kKB = 4;     // bandwidths per batch
constexpr int kKT = 64;    // bottom block: one wavefront
constexpr int kKItems = 4;
constexpr int kKTile = 256 * kKItems;
constexpr int64_t kKdeDirectMaxN = int64_t(1) << 20;  // d >= 4: O(N^2) direct sums

__device__ __forceinline__ uint64_t order_key_kde(double v) {
    if (v == 0.0)
        v = 0.0;
    uint64_t b = (uint64_t)__double_as_longlong(v);
    return (b & 0x8000000000000000ull) ? ~b : (b | 0x8000000000000000ull);
}

template <typename T> __device__ __forceinline__ T kexp(T v);
template <> __device__ __forceinline__ double kexp<double>(double v) { return exp(v); }
template <> __device__ __forceinline__ float kexp<float>(float v) { return expf(v); }

struct KBatch {
    double ih[kKB][3];  // 1/h_k per bandwidth and coordinate
    double norm_full[kKB];
    double norm_loo[kKB];
    int nb;             // bandwidths used in this batch (<= kKB)
};

// Structure-of-arrays state of the sample in some order.
struct KState {
    double *x[3];
    double *w0, *w1;
    uint8_t *bits;   // bit 0: x1 side (A = 0, B = 1); bit 1: x2 side (d = 3)
    uint32_t *map;   // position of each item in the next (merged or block-sorted) state
};

// ----------------------------------------------------------- build kernels
__global__ __launch_bounds__(256) void k_kx_keys(const double *__restrict__ x0, int64_t n,
                                                 uint64_t *__restrict__ keys,
                                                 uint32_t *__restrict__ idx) {
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n)
        return;
    keys[i] = order_key_kde(x0[i]);
    idx[i] = (uint32_t)i;
}

template <typename WT>
__global__ __launch_bounds__(256) void k_kgather0(const uint32_t *__restrict__ idx, int64_t n,
                                                  int d, const double *__restrict__ x,
                                                  const WT *__restrict__ w0in,
                                                  const WT *__restrict__ w1in, KState o,
                                                  uint32_t *__restrict__ id) {
    int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= n)
        return;
    uint32_t i = idx[p];
    for (int k = 0; k < 3; ++k)
        o.x[k][p] = k < d ? x[(int64_t)k * n + i] : 0.0;
    o.w0[p] = w0in ? (double)w0in[i] : 1.0;
    o.w1[p] = w1in ? (double)w1in[i] : 0.0;
    o.bits[p] = 0;
    id[p] = i;
}

// One wavefront per block of 64 items: bitonic sort by coordinate `key` in
// registers.  Writes the block sorted into `o`, map[p] = new position.
__global__ __launch_bounds__(256) void k_kblocksort(KState in, int key, int64_t n, KState o,
                                                    uint32_t *__restrict__ map) {
    const int lane = threadIdx.x & 63;
    const int64_t blk = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int64_t p = blk * 64 + lane;
    if (blk * 64 >= n)
        return;
    bool v = p < n;
    uint64_t kk = v ? order_key_kde(in.x[key][p]) : ~0ull;
    int src = lane;
#pragma unroll
    for (int k = 2; k <= 64; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            uint64_t ok = shfl_xor(kk, j);
            int os = __shfl_xor(src, j, 64);
            bool up = (lane & k) == 0;
            bool lower = (lane & j) == 0;
            bool less = (ok < kk) || (ok == kk && os < src);
            bool greater = (ok > kk) || (ok == kk && os > src);
            bool take = (lower == up) ? less : greater;
            if (take) {
                kk = ok;
                src = os;
            }
        }
    }
    int64_t q = blk * 64 + src;
    int64_t dst = blk * 64 + lane;
    if (q < n) {
        for (int c = 0; c < 3; ++c)
            o.x[c][dst] = in.x[c][q];
        o.w0[dst] = in.w0[q];
        o.w1[dst] = in.w1[q];
        o.bits[dst] = in.bits[q];
        map[q] = (uint32_t)dst;
    }
}

// Merge of aligned blocks of size h (a power of two) sorted by coordinate
// `key` (A then B) into 2h, one thread per item; sets bit `sbit` to the item's
// side and records in.map[p] = new position.
__global__ __launch_bounds__(256) void k_kmerge(KState in, int key, int64_t n, int64_t h,
                                                int sbit, KState o) {
    int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= n)
        return;
    int64_t s = p & ~(2 * h - 1);
    int64_t ha = (n - s) < h ? (n - s) : h;
    int64_t hb = (n - s - ha) < h ? (n - s - ha) : h;
    const double *K = in.x[key];
    double kv = K[p];
    bool inA = (p - s) < ha;
    int64_t pos;
    if (inA) {
        const double *B = K + s + ha;
        int64_t lo = 0, hi = hb;
        while (lo < hi) {
            int64_t mid = (lo + hi) >> 1;
            if (B[mid] < kv)
                lo = mid + 1;
            else
                hi = mid;
        }
        pos = p + lo;
    } else {
        const double *A = K + s;
        int64_t lo = 0, hi = ha;
        while (lo < hi) {
            int64_t mid = (lo + hi) >> 1;
            if (A[mid] <= kv)
                lo = mid + 1;
            else
                hi = mid;
        }
        pos = s + (p - s - ha) + lo;
    }
    for (int c = 0; c < 3; ++c)
        o.x[c][pos] = in.x[c][p];
    o.w0[pos] = in.w0[p];
    o.w1[pos] = in.w1[p];
    uint8_t b = in.bits[p];
    b = inA ? (uint8_t)(b & ~(1u << sbit)) : (uint8_t)(b | (1u << sbit));
    o.bits[pos] = b;
    in.map[p] = (uint32_t)pos;
}

// ----------------------------------------------------------- scan kernels
// Per item p of a level (merged order, segments of 2 hin items):
//   alpha_p = exp(-(xs_p - xs_{p-1}) / h_s)   (0 at a segment start)
//   beta_p  = exp(-(xs_{p+1} - xs_p) / h_s)   (0 before a segment start)
//   f_p     = exp(-sum over split coordinates k of |x_k - c_k| / h_k)
//   own_p   = f_p w_p on the item's side combination
// Forward state F_p = alpha_p F_{p-1} + own_p, backward B_p = beta_p B_{p+1} + own_p
// (one value per side combination and channel).  Item p receives
//   f_p * (alpha_p F_{p-1} + beta_p B_{p+1})   of the opposite combination,
// its kernel sum over the items on the other side of every split.  In the
// 1-D case (oneside) there is one side and f = 1.  Both recurrences are affine
// scans, state -> m * state + l, evaluated as tile aggregates, tile carries
// and a final pass, with fixed-order tree scans inside each tile.
//
// The decay m of a run of items is the product of their decays,
// exp(-(x_last - x_before) / h).  It is formed from those two coordinates
// each time it is used, never multiplied out: a product of k rounded factors
// carries k roundings (for float32 factors over 2^20 sorted normal points at
// h = 1 that is a relative error of 2.5e-4), while each weight then passes
// through O(log N) compositions.  A map stores lo, the scanned coordinate
// before its run (-inf when a segment starts inside the run, so m = 0), and
// hi, the coordinate of its last item; maps of the backward scan store both
// negated, so that one rule serves both directions.  lo = NaN marks the
// identity.
//
// Inside a tile of kKTile items float64 decays are also carried multiplied
// out (m): at most kKTile roundings, a relative error below 1.2e-13, for one
// multiplication per composition instead of an exponential.  Float32 decays
// are always formed from the coordinates, and across tiles both are.
template <typename T> constexpr bool tile_products() { return std::is_same<T, double>::value; }

template <typename T, int CH, int NSD> struct Aff {
    double lo, hi;
    T m[kKB];  // the decay multiplied out (used when tile_products<T>())
    T l[kKB][NSD][CH];
};

template <typename T, int CH, int NSD>
__device__ __forceinline__ void aff_identity(Aff<T, CH, NSD> &a) {
    a.lo = a.hi = __builtin_nan("");
#pragma unroll
    for (int b = 0; b < kKB; ++b) {
        a.m[b] = T(1);
#pragma unroll
        for (int s = 0; s < NSD; ++s)
#pragma unroll
            for (int c = 0; c < CH; ++c)
                a.l[b][s][c] = T(0);
    }
}

// The decay of map a for bandwidth b (ih: 1/h of the scanned coordinate),
// from the coordinates (A) or as carried.
template <bool A, typename T, int CH, int NSD>
__device__ __forceinline__ T aff_m(const Aff<T, CH, NSD> &a, const double (&ih)[kKB], int b) {
    if constexpr (!A)
        return a.m[b];
    return (a.lo != a.lo) ? T(1) : kexp<T>((T)(-(a.hi - a.lo) * ih[b]));
}

// first `x`, then `y` (y's run follows x's): state -> y.m (x.m state + x.l) + y.l
template <bool A, typename T, int CH, int NSD>
__device__ __forceinline__ Aff<T, CH, NSD> aff_then(const Aff<T, CH, NSD> &x,
                                                    const Aff<T, CH, NSD> &y,
                                                    const double (&ih)[kKB]) {
    Aff<T, CH, NSD> r;
    if constexpr (A) {
        const bool xid = x.lo != x.lo, yid = y.lo != y.lo;
        r.lo = xid ? y.lo : (y.lo == -INFINITY ? -INFINITY : x.lo);
        r.hi = yid ? x.hi : y.hi;
    } else {
        // the identity needs no special case here (m = 1, l = 0); the
        // coordinates of a tile's total are set from the tile itself
        r.lo = r.hi = 0.0;
    }
#pragma unroll
    for (int b = 0; b < kKB; ++b) {
        const T my = aff_m<A>(y, ih, b);
        if constexpr (!A)
            r.m[b] = x.m[b] * my;
#pragma unroll
        for (int s = 0; s < NSD; ++s)
#pragma unroll
            for (int c = 0; c < CH; ++c)
                r.l[b][s][c] = my * x.l[b][s][c] + y.l[b][s][c];
    }
    return r;
}

// 1/h of the scanned coordinate for each bandwidth of the batch
__device__ __forceinline__ void scan_ih(const KBatch &kb, int sc, double (&ih)[kKB]) {
#pragma unroll
    for (int b = 0; b < kKB; ++b)
        ih[b] = kb.ih[b][sc];
}

template <typename T, int CH, int NSD> struct KTileAgg {
    Aff<T, CH, NSD> fwd;  // items in ascending order
    Aff<T, CH, NSD> bwd;  // items in descending order
};
template <typename T, int CH, int NSD> struct KCarry {
    T F[kKB][NSD][CH];  // forward state after all earlier tiles
    T B[kKB][NSD][CH];  // backward state after all later tiles
};

struct KLevelArgs {
    const double *xs;       // scanned coordinate
    int sc;                 // its index (for the bandwidth)
    const double *xa;       // first split coordinate (x1)
    const double *ca;       // split points source for xa (x1-sorted sample)
    int64_t ha;             // half size of the xa split blocks (ha, hb, hin: powers of two)
    const double *xb;       // second split coordinate (x2, d = 3) or nullptr
    const double *cb;       // split points source for xb
    int64_t hb;
    const double *w0, *w1;
    const uint8_t *bits;
    int64_t n, hin;         // scan segments are 2 hin
    int oneside;
};

// The split point of the block of 2h items holding p (h a power of two).
__device__ __forceinline__ double split_point(const double *src, int64_t p, int64_t h,
                                              int64_t n) {
    const int64_t s = p & ~(2 * h - 1);
    return (s + h < n) ? src[s + h] : src[n - 1];
}

// Item p's decays and weights from its loaded values: x, the scanned
// coordinate of it (xp, xn: of its neighbours), da / db its distances to the
// split points of the split coordinates, side bits sb, weights w0v, w1v.
template <typename T, int CH, int NSD>
__device__ __forceinline__ void kitem(const KLevelArgs &L, const KBatch &kb, int64_t p,
                                      double x, double xp, double xn, double da, double db,
                                      uint32_t sb, double w0v, double w1v, T alpha[kKB],
                                      T *beta, T f[kKB], int &sd, T wv[CH]) {
    const int64_t seg = 2 * L.hin;  // a power of two
    const int64_t s = p & ~(seg - 1);
    const bool start = (p == s);
    const bool last = (p + 1 >= L.n) || (p + 1 == s + seg);
    sd = L.oneside ? 0 : (int)(sb & (NSD - 1));
    wv[0] = (T)w0v;
    if (CH > 1)
        wv[CH - 1] = (T)w1v;
#pragma unroll
    for (int b = 0; b < kKB; ++b) {
        double ihs = kb.ih[b][L.sc];
        alpha[b] = start ? T(0) : kexp<T>((T)(-(x - xp) * ihs));
        if (beta)
            beta[b] = last ? T(0) : kexp<T>((T)(-(xn - x) * ihs));
        f[b] = L.oneside ? T(1) : kexp<T>((T)(-(da * kb.ih[b][0] + db * kb.ih[b][1])));
    }
}

// the kKItems (= 4) doubles at q (32-byte aligned) as two 16-byte loads
__device__ __forceinline__ void load4(const double *q, double v[4]) {
    const double2 a = reinterpret_cast<const double2 *>(q)[0];
    const double2 b = reinterpret_cast<const double2 *>(q)[1];
    v[0] = a.x;
    v[1] = a.y;
    v[2] = b.x;
    v[3] = b.y;
}

// Side-indexed access to small per-thread arrays with the side as a select
// over all sides, so that the arrays stay in registers (a runtime index
// would place them in scratch memory).
template <typename T, int CH, int NSD>
__device__ __forceinline__ void add_side(T (&l)[NSD][CH], int sd, const T (&v)[CH]) {
#pragma unroll
    for (int s = 0; s < NSD; ++s)
#pragma unroll
        for (int c = 0; c < CH; ++c)
            l[s][c] += (s == sd) ? v[c] : T(0);
}
// a or b by an integer mask on the bits (the compiler keeps this a register
// operation; a select between array elements can become an indexed load
// from scratch memory)
__device__ __forceinline__ double mask_pick(bool take_b, double a, double b) {
    const uint64_t m = take_b ? ~0ull : 0ull;
    const uint64_t r = ((uint64_t)__double_as_longlong(a) & ~m) |
                       ((uint64_t)__double_as_longlong(b) & m);
    return __longlong_as_double((long long)r);
}
__device__ __forceinline__ float mask_pick(bool take_b, float a, float b) {
    const uint32_t m = take_b ? ~0u : 0u;
    return __uint_as_float((__float_as_uint(a) & ~m) | (__float_as_uint(b) & m));
}

template <typename T, int CH, int NSD>
__device__ __forceinline__ T get_side(const T (&l)[NSD][CH], int sd, int c) {
    T r = l[0][c];
#pragma unroll
    for (int s = 1; s < NSD; ++s)
        r = mask_pick(s == sd, r, l[s][c]);
    return r;
}

// Where the thread's items sit on the scanned coordinate: the first and the
// last valid item's value, the values just before and after the items, and
// which items start or end a segment (bit u).  Kept as scalars: selecting
// among array elements by a runtime condition can place the array in memory.
struct ItemPos {
    double xfirst, xlast;
    double xprev, xnext;
    uint32_t starts, lasts, vmask;
};

// The maps of the thread's items composed in order: forward (dir = 0, items
// ascending) or backward (dir = 1, descending).
template <typename T, int CH, int NSD>
__device__ __forceinline__ Aff<T, CH, NSD> thread_aff(const T alpha[kKItems + 1][kKB],
                                                      const T f[kKItems][kKB],
                                                      const int sd[kKItems],
                                                      const T wv[kKItems][CH],
                                                      const bool val[kKItems],
                                                      const ItemPos &ps, int dir) {
    Aff<T, CH, NSD> a;
    aff_identity(a);
    if (!tile_products<T>() && ps.vmask) {
        if (dir == 0) {
            a.lo = (ps.starts & ps.vmask) ? -INFINITY : ps.xprev;
            a.hi = ps.xlast;
        } else {
            a.lo = (ps.lasts & ps.vmask) ? -INFINITY : -ps.xnext;
            a.hi = -ps.xfirst;
        }
    }
#pragma unroll
    for (int k = 0; k < kKItems; ++k) {
        const int u = dir ? kKItems - 1 - k : k;
        if (!val[u])
            continue;
#pragma unroll
        for (int b = 0; b < kKB; ++b) {
            const T dec = dir ? alpha[u + 1][b] : alpha[u][b];
            if constexpr (tile_products<T>())
                a.m[b] *= dec;
#pragma unroll
            for (int s = 0; s < NSD; ++s)
#pragma unroll
                for (int c = 0; c < CH; ++c)
                    a.l[b][s][c] *= dec;
            T add[CH];
#pragma unroll
            for (int c = 0; c < CH; ++c)
                add[c] = f[u][b] * wv[u][c];
            add_side<T, CH, NSD>(a.l[b], sd[u], add);
        }
    }
    return a;
}

// alpha[u] for the thread's items u; alpha[kKItems] is the last item's beta.
// The beta of item u < kKItems - 1 is alpha[u + 1]: both are the decay across
// the same pair of neighbours (0 at a segment boundary or past the end).  The
// items' arrays are read as whole records: base is a multiple of kKItems and
// every array starts 256-byte aligned.
template <typename T, int CH, int NSD>
__device__ __forceinline__ void load_items(const KLevelArgs &L, const KBatch &kb,
                                           int64_t base, T alpha[kKItems + 1][kKB],
                                           T f[kKItems][kKB], int sd[kKItems],
                                           T wv[kKItems][CH], bool val[kKItems],
                                           ItemPos &ps) {
    static_assert(kKItems == 4, "items read as two 16-byte loads per array");
    double xs[4], xa[4] = {0.0, 0.0, 0.0, 0.0}, xb[4] = {0.0, 0.0, 0.0, 0.0};
    double w0[4], w1[4] = {0.0, 0.0, 0.0, 0.0};
    uint32_t bits4 = 0u;
    if (base + 4 <= L.n) {
        load4(L.xs + base, xs);
        load4(L.w0 + base, w0);
        if (CH > 1)
            load4(L.w1 + base, w1);
        if (!L.oneside) {
            load4(L.xa + base, xa);
            if (NSD == 4)
                load4(L.xb + base, xb);
            bits4 = *reinterpret_cast<const uint32_t *>(L.bits + base);
        }
    } else {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t p = base + u;
            const bool v = p < L.n;
            xs[u] = v ? L.xs[p] : 0.0;
            w0[u] = v ? L.w0[p] : 0.0;
            if (CH > 1)
                w1[u] = v ? L.w1[p] : 0.0;
            if (!L.oneside && v) {
                xa[u] = L.xa[p];
                if (NSD == 4)
                    xb[u] = L.xb[p];
                bits4 |= (uint32_t)L.bits[p] << (8 * u);
            }
        }
    }
    const double xprev = base > 0 && base - 1 < L.n ? L.xs[base - 1] : 0.0;
    const double xnext = base + 4 < L.n ? L.xs[base + 4] : 0.0;
    ps.xprev = xprev;
    ps.xnext = xnext;
    ps.xfirst = xs[0];
    ps.xlast = xs[0];
    ps.starts = ps.lasts = ps.vmask = 0u;
    {
        const int64_t seg = 2 * L.hin;  // a power of two
#pragma unroll
        for (int u = 0; u < kKItems; ++u) {
            const int64_t p = base + u;
            if (p < L.n) {
                ps.vmask |= 1u << u;
                ps.xlast = xs[u];
            }
            const int64_t s0 = p & ~(seg - 1);
            if (p == s0)
                ps.starts |= 1u << u;
            if (p + 1 >= L.n || p + 1 == s0 + seg)
                ps.lasts |= 1u << u;
        }
    }
#pragma unroll
    for (int b = 0; b < kKB; ++b)
        alpha[kKItems][b] = T(0);
#pragma unroll
    for (int u = 0; u < kKItems; ++u) {
        int64_t p = base + u;
        val[u] = p < L.n;
        if (val[u]) {
            double da = 0.0, db = 0.0;
            if (!L.oneside) {
                da = fabs(xa[u] - split_point(L.ca, p, L.ha, L.n));
                if (NSD == 4)
                    db = fabs(xb[u] - split_point(L.cb, p, L.hb, L.n));
            }
            kitem<T, CH, NSD>(L, kb, p, xs[u], u > 0 ? xs[u - 1] : xprev,
                              u < kKItems - 1 ? xs[u + 1] : xnext, da, db, bits4 >> (8 * u),
                              w0[u], w1[u], alpha[u],
                              u == kKItems - 1 ? alpha[kKItems] : nullptr, f[u], sd[u], wv[u]);
        } else {
            sd[u] = 0;
#pragma unroll
            for (int b = 0; b < kKB; ++b)
                alpha[u][b] = f[u][b] = T(0);
#pragma unroll
            for (int c = 0; c < CH; ++c)
                wv[u][c] = T(0);
        }
    }
}

// The 256 thread maps sit in LDS field by field (element f of thread t at
// f * 256 + t), so that a wavefront's accesses to one field are consecutive.
// (A: the map's coordinates are moved, else its multiplied-out decays)
template <bool A, typename T, int CH, int NSD>
__device__ __forceinline__ void aff_put(Aff<T, CH, NSD> *buf, int t,
                                        const Aff<T, CH, NSD> &a) {
    double *qd = reinterpret_cast<double *>(buf);
    if constexpr (A) {
        qd[t] = a.lo;
        qd[256 + t] = a.hi;
    }
    T *q = reinterpret_cast<T *>(qd + 512);
#pragma unroll
    for (int b = 0; b < kKB; ++b) {
        if constexpr (!A)
            q[b * 256 + t] = a.m[b];
#pragma unroll
        for (int s = 0; s < NSD; ++s)
#pragma unroll
            for (int c = 0; c < CH; ++c)
                q[(kKB + (b * NSD + s) * CH + c) * 256 + t] = a.l[b][s][c];
    }
}
template <bool A, typename T, int CH, int NSD>
__device__ __forceinline__ Aff<T, CH, NSD> aff_get(const Aff<T, CH, NSD> *buf, int t) {
    const double *qd = reinterpret_cast<const double *>(buf);
    Aff<T, CH, NSD> a;
    a.lo = A ? qd[t] : 0.0;
    a.hi = A ? qd[256 + t] : 0.0;
    const T *q = reinterpret_cast<const T *>(qd + 512);
#pragma unroll
    for (int b = 0; b < kKB; ++b) {
        a.m[b] = A ? T(1) : q[b * 256 + t];
#pragma unroll
        for (int s = 0; s < NSD; ++s)
#pragma unroll
            for (int c = 0; c < CH; ++c)
                a.l[b][s][c] = q[(kKB + (b * NSD + s) * CH + c) * 256 + t];
    }
    return a;
}

// Inclusive tree scan of the 256 thread maps in LDS: forward (dir = 0, thread
// t composes threads 0..t) or backward (dir = 1, threads 255..t).
template <bool A, typename T, int CH, int NSD>
__device__ __forceinline__ Aff<T, CH, NSD> block_aff_scan(Aff<T, CH, NSD> v,
                                                          Aff<T, CH, NSD> *buf, int dir,
                                                          const double (&ih)[kKB]) {
    const int t = threadIdx.x;
    aff_put<A>(buf, t, v);
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        Aff<T, CH, NSD> r = v;
        if (dir == 0 && t >= off)
            r = aff_then<A>(aff_get<A>(buf, t - off), v, ih);
        if (dir == 1 && t + off < 256)
            r = aff_then<A>(aff_get<A>(buf, t + off), v, ih);
        __syncthreads();
        v = r;
        aff_put<A>(buf, t, v);
        __syncthreads();
    }
    return v;
}

// The same scans by lane moves inside each wavefront (wave_aff_scan below)
// and one exchange of the four wavefront totals through LDS (wt, 4 entries):
// inc is the thread's inclusive composition (dir 0: threads 0..t in order;
// dir 1: threads 255..t), exc the exclusive one (identity for the first
// thread in scan order).
template <bool A, typename T, int CH, int NSD>
__device__ __forceinline__ Aff<T, CH, NSD> aff_shfl(const Aff<T, CH, NSD> &a, int src) {
    Aff<T, CH, NSD> r;
    r.lo = A ? shfl(a.lo, src) : 0.0;
    r.hi = A ? shfl(a.hi, src) : 0.0;
#pragma unroll
    for (int b = 0; b < kKB; ++b) {
        r.m[b] = A ? T(1) : shfl(a.m[b], src);
#pragma unroll
        for (int s = 0; s < NSD; ++s)
#pragma unroll
            for (int c = 0; c < CH; ++c)
                r.l[b][s][c] = shfl(a.l[b][s][c], src);
    }
    return r;
}

// A value from another lane by a DPP move (CTRL: the DPP control word, RM:
// the rows that receive it; other lanes keep 0).
template <int CTRL, int RM, typename V> __device__ __forceinline__ V dpp_mov(V v) {
    if constexpr (sizeof(V) == 8) {
        union {
            V t;
            int i[2];
        } u;
        u.t = v;
        u.i[0] = __builtin_amdgcn_update_dpp(0, u.i[0], CTRL, RM, 0xf, false);
        u.i[1] = __builtin_amdgcn_update_dpp(0, u.i[1], CTRL, RM, 0xf, false);
        return u.t;
    } else {
        union {
            V t;
            int i;
        } u;
        u.t = v;
        u.i = __builtin_amdgcn_update_dpp(0, u.i, CTRL, RM, 0xf, false);
        return u.t;
    }
}
template <int CTRL, int RM, bool A, typename T, int CH, int NSD>
__device__ __forceinline__ Aff<T, CH, NSD> aff_dpp(const Aff<T, CH, NSD> &a) {
    Aff<T, CH, NSD> r;
    r.lo = A ? dpp_mov<CTRL, RM>(a.lo) : 0.0;
    r.hi = A ? dpp_mov<CTRL, RM>(a.hi) : 0.0;
#pragma unroll
    for (int b = 0; b < kKB; ++b) {
        r.m[b] = A ? T(1) : dpp_mov<CTRL, RM>(a.m[b]);
#pragma unroll
        for (int s = 0; s < NSD; ++s)
#pragma unroll
            for (int c = 0; c < CH; ++c)
                r.l[b][s][c] = dpp_mov<CTRL, RM>(a.l[b][s][c]);
    }
    return r;
}

// The same with the lanes that have no source lane set to 0 (bound_ctrl), for
// controls that write every row: nothing to clear beforehand.
template <int CTRL, typename V> __device__ __forceinline__ V dpp_movz(V v) {
    if constexpr (sizeof(V) == 8) {
        union {
            V t;
            int i[2];
        } u;
        u.t = v;
        u.i[0] = __builtin_amdgcn_mov_dpp(u.i[0], CTRL, 0xf, 0xf, true);
        u.i[1] = __builtin_amdgcn_mov_dpp(u.i[1], CTRL, 0xf, 0xf, true);
        return u.t;
    } else {
        union {
            V t;
            int i;
        } u;
        u.t = v;
        u.i = __builtin_amdgcn_mov_dpp(u.i, CTRL, 0xf, 0xf, true);
        return u.t;
    }
}
template <int CTRL, bool A, typename T, int CH, int NSD>
__device__ __forceinline__ Aff<T, CH, NSD> aff_dppz(const Aff<T, CH, NSD> &a) {
    Aff<T, CH, NSD> r;
    r.lo = A ? dpp_movz<CTRL>(a.lo) : 0.0;
    r.hi = A ? dpp_movz<CTRL>(a.hi) : 0.0;
#pragma unroll
    for (int b = 0; b < kKB; ++b) {
        r.m[b] = A ? T(1) : dpp_movz<CTRL>(a.m[b]);
#pragma unroll
        for (int s = 0; s < NSD; ++s)
#pragma unroll
            for (int c = 0; c < CH; ++c)
                r.l[b][s][c] = dpp_movz<CTRL>(a.l[b][s][c]);
    }
    return r;
}

// DPP controls: row_shr:n (lane i of a 16-lane row takes lane i - n), row_shl:n
// (lane i + n), row_bcast:15 / :31 (the last lane of row 0 / 1 to the rows
// above it), wave_shr:1 / wave_shl:1 (lane i - 1 / i + 1 across the wave)
constexpr int kDppRowShr = 0x110, kDppRowShl = 0x100, kDppBcast15 = 0x142, kDppBcast31 = 0x143,
              kDppWaveShr1 = 0x138, kDppWaveShl1 = 0x130;

// Inclusive scan of the wavefront's maps in lane order (dir 0: lanes 0..i
// composed in order; dir 1: lanes 63..i).  Within each row of 16 lanes by
// DPP row shifts (1, 2, 4, 8), then across rows: forward by the row
// broadcasts of the last lanes of rows 0 and 1, backward by taking the first
// lane of the next row (rows 0 and 2), then lane 32 (rows 0 and 1).
template <bool A, typename T, int CH, int NSD>
__device__ __forceinline__ Aff<T, CH, NSD> wave_aff_scan(Aff<T, CH, NSD> x, int dir,
                                                         const double (&ih)[kKB]) {
    const int lane = threadIdx.x & 63;
    const int rl = lane & 15, row = lane >> 4;
    if (dir == 0) {
        { const auto o = aff_dppz<kDppRowShr + 1, A>(x); if (rl >= 1) x = aff_then<A>(o, x, ih); }
        { const auto o = aff_dppz<kDppRowShr + 2, A>(x); if (rl >= 2) x = aff_then<A>(o, x, ih); }
        { const auto o = aff_dppz<kDppRowShr + 4, A>(x); if (rl >= 4) x = aff_then<A>(o, x, ih); }
        { const auto o = aff_dppz<kDppRowShr + 8, A>(x); if (rl >= 8) x = aff_then<A>(o, x, ih); }
        { const auto o = aff_dpp<kDppBcast15, 0xa, A>(x); if (row & 1) x = aff_then<A>(o, x, ih); }
        { const auto o = aff_dpp<kDppBcast31, 0xc, A>(x); if (row >= 2) x = aff_then<A>(o, x, ih); }
    } else {
        { const auto o = aff_dppz<kDppRowShl + 1, A>(x); if (rl + 1 < 16) x = aff_then<A>(o, x, ih); }
        { const auto o = aff_dppz<kDppRowShl + 2, A>(x); if (rl + 2 < 16) x = aff_then<A>(o, x, ih); }
        { const auto o = aff_dppz<kDppRowShl + 4, A>(x); if (rl + 4 < 16) x = aff_then<A>(o, x, ih); }
        { const auto o = aff_dppz<kDppRowShl + 8, A>(x); if (rl + 8 < 16) x = aff_then<A>(o, x, ih); }
        {
            const auto o = aff_shfl<A>(x, (16 * (row + 1)) & 63);
            if ((row & 1) == 0)
                x = aff_then<A>(o, x, ih);
        }
        {
            const auto o = aff_shfl<A>(x, 32);
            if (row < 2)
                x = aff_then<A>(o, x, ih);
        }
    }
    return x;
}

template <bool A, typename T, int CH, int NSD>
__device__ __forceinline__ void block_aff_scan2(const Aff<T, CH, NSD> &v, Aff<T, CH, NSD> *wt,
                                                int dir, Aff<T, CH, NSD> &inc,
                                                Aff<T, CH, NSD> &exc, const double (&ih)[kKB]) {
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const Aff<T, CH, NSD> x = wave_aff_scan<A>(v, dir, ih);
    __syncthreads();  // the totals of an earlier scan have been read
    if (lane == (dir ? 0 : 63))
        wt[w] = x;
    __syncthreads();
    Aff<T, CH, NSD> pre;
    aff_identity(pre);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int q = dir ? 3 - k : k;
        if (dir ? (q > w) : (q < w))
            pre = aff_then<A>(pre, wt[q], ih);
    }
    inc = aff_then<A>(pre, x, ih);
    const Aff<T, CH, NSD> nb =
        dir ? aff_dpp<kDppWaveShl1, 0xf, A>(x) : aff_dpp<kDppWaveShr1, 0xf, A>(x);
    exc = (dir ? lane == 63 : lane == 0) ? pre : aff_then<A>(pre, nb, ih);
}

// Which block scan a kernel uses: the LDS tree keeps fewer values in
// registers, which is what float64 density sums (one channel) need to keep
// three wavefronts per SIMD; the wavefront scan needs almost no LDS and fewer
// barriers, which wins for two channels and for float32.
template <typename T, int CH> constexpr bool shfl_scan() {
    return !(std::is_same<T, double>::value && CH == 1);
}

// The coordinates of a whole tile's forward and backward maps, read from the
// tile itself (maps inside a tile carry none when their decays are
// multiplied out).  Segments are aligned blocks of 2 hin items and tiles
// aligned blocks of kKTile, both powers of two, so a segment starts inside the
// tile exactly when one starts at its first item, and one ends inside it
// exactly when one ends at its last item or the sample does.
__device__ __forceinline__ void tile_coords(const KLevelArgs &L, int64_t t0, double &flo,
                                            double &fhi, double &blo, double &bhi) {
    const int64_t seg = 2 * L.hin;
    const int64_t t1 = t0 + kKTile < L.n ? t0 + kKTile : L.n;  // one past the last item
    const bool start = (t0 & (seg - 1)) == 0;
    const bool end = t1 >= L.n || (t1 & (seg - 1)) == 0;
    flo = start ? -INFINITY : L.xs[t0 - 1];
    fhi = L.xs[t1 - 1];
    blo = end ? -INFINITY : -L.xs[t1];
    bhi = -L.xs[t0];
}

template <typename T, int CH, int NSD>
__global__ __launch_bounds__(256) void k_ktile_agg(KLevelArgs L, KBatch kb,
                                                   KTileAgg<T, CH, NSD> *__restrict__ agg) {
    // the wavefront scans also for float64 density sums up to d = 2: only
    // the tile totals are kept, which leaves them the registers of the
    // LDS tree variant
    constexpr bool kShfl = shfl_scan<T, CH>() || NSD <= 2;
    __shared__ Aff<T, CH, NSD> buf[kShfl ? 4 : 256];
    const int64_t base = (int64_t)blockIdx.x * kKTile + (int64_t)threadIdx.x * kKItems;
    T alpha[kKItems + 1][kKB], f[kKItems][kKB], wv[kKItems][CH];
    int sd[kKItems];
    bool val[kKItems];
    ItemPos ps;
    load_items<T, CH, NSD>(L, kb, base, alpha, f, sd, wv, val, ps);
    double ih[kKB];
    scan_ih(kb, L.sc, ih);
    double fi_lo, fi_hi, bi_lo, bi_hi;  // the unused pair of tile_coords
    if constexpr (kShfl) {
        Aff<T, CH, NSD> fi, fe, bi, be;
        block_aff_scan2<!tile_products<T>(), T, CH, NSD>(thread_aff<T, CH, NSD>(alpha, f, sd, wv, val, ps, 0), buf,
                                    0, fi, fe, ih);
        if (threadIdx.x == 255) {
            if constexpr (tile_products<T>())
                tile_coords(L, (int64_t)blockIdx.x * kKTile, fi.lo, fi.hi, bi_lo, bi_hi);
            agg[blockIdx.x].fwd = fi;
        }
        block_aff_scan2<!tile_products<T>(), T, CH, NSD>(thread_aff<T, CH, NSD>(alpha, f, sd, wv, val, ps, 1), buf,
                                    1, bi, be, ih);
        if (threadIdx.x == 0) {
            if constexpr (tile_products<T>())
                tile_coords(L, (int64_t)blockIdx.x * kKTile, fi_lo, fi_hi, bi.lo, bi.hi);
            agg[blockIdx.x].bwd = bi;
        }
    } else {
        Aff<T, CH, NSD> fi = block_aff_scan<!tile_products<T>(), T, CH, NSD>(
            thread_aff<T, CH, NSD>(alpha, f, sd, wv, val, ps, 0), buf, 0, ih);
        if (threadIdx.x == 255) {
            if constexpr (tile_products<T>())
                tile_coords(L, (int64_t)blockIdx.x * kKTile, fi.lo, fi.hi, bi_lo, bi_hi);
            agg[blockIdx.x].fwd = fi;
        }
        Aff<T, CH, NSD> bi = block_aff_scan<!tile_products<T>(), T, CH, NSD>(
            thread_aff<T, CH, NSD>(alpha, f, sd, wv, val, ps, 1), buf, 1, ih);
        if (threadIdx.x == 0) {
            if constexpr (tile_products<T>())
                tile_coords(L, (int64_t)blockIdx.x * kKTile, fi_lo, fi_hi, bi.lo, bi.hi);
            agg[blockIdx.x].bwd = bi;
        }
    }
}

// Tile carries in two steps.  k_kcarry_local: per group of 256 consecutive
// tiles, the exclusive scans of the tile maps inside the group (forward:
// tiles in ascending order; backward: descending; wavefront scans, then the
// four wavefront totals), written over the tile aggregates, and the group
// totals; with one group (car != null) it writes the carries itself.
// k_kcarry_final: per group, the maps of the groups before it (forward) or
// after it (backward) composed in order (by one wavefront's scan of the group
// totals when there are at most 64 groups, else one after the other), then
// per tile its own exclusive map: the state entering the tile.
template <typename T, int CH, int NSD>
__global__ __launch_bounds__(256) void k_kcarry_local(KTileAgg<T, CH, NSD> *__restrict__ agg,
                                                      int64_t nt,
                                                      KTileAgg<T, CH, NSD> *__restrict__ grp,
                                                      KCarry<T, CH, NSD> *__restrict__ car,
                                                      KBatch kb, int sc) {
    __shared__ Aff<T, CH, NSD> wt[4];
    const int t = threadIdx.x;
    double ih[kKB];
    scan_ih(kb, sc, ih);
    const int64_t q = (int64_t)blockIdx.x * 256 + t;
    Aff<T, CH, NSD> fa, ba;
    aff_identity(fa);
    aff_identity(ba);
    if (q < nt) {
        fa = agg[q].fwd;
        ba = agg[q].bwd;
    }
    Aff<T, CH, NSD> fi, fex, bi, bex;
    block_aff_scan2<true, T, CH, NSD>(fa, wt, 0, fi, fex, ih);
    if (t == 255)
        grp[blockIdx.x].fwd = fi;
    block_aff_scan2<true, T, CH, NSD>(ba, wt, 1, bi, bex, ih);
    if (t == 0)
        grp[blockIdx.x].bwd = bi;
    if (q >= nt)
        return;
    if (car) {
        // a single group: the states entering the tiles are the exclusive
        // maps applied to the zero state
#pragma unroll
        for (int b = 0; b < kKB; ++b)
#pragma unroll
            for (int s = 0; s < NSD; ++s)
#pragma unroll
                for (int c = 0; c < CH; ++c) {
                    car[q].F[b][s][c] = fex.l[b][s][c];
                    car[q].B[b][s][c] = bex.l[b][s][c];
                }
    } else {
        agg[q].fwd = fex;
        agg[q].bwd = bex;
    }
}

template <typename T, int CH, int NSD>
__global__ __launch_bounds__(256) void k_kcarry_final(const KTileAgg<T, CH, NSD> *__restrict__ loc,
                                                      int64_t nt,
                                                      const KTileAgg<T, CH, NSD> *__restrict__ grp,
                                                      KCarry<T, CH, NSD> *__restrict__ car,
                                                      KBatch kb, int sc) {
    __shared__ Aff<T, CH, NSD> ent[2];  // the maps entering this group, both ways
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double ih[kKB];
    scan_ih(kb, sc, ih);
    const int64_t g = blockIdx.x, ng = ceil_div_dev(nt, (int64_t)256);
    Aff<T, CH, NSD> cf, cb;
    aff_identity(cf);
    aff_identity(cb);
    if (ng <= 64) {
        // the first wavefront (all its lanes active) scans the group maps,
        // lane j holding group j (identity past the last group)
        if (threadIdx.x < 64) {
            const int j = (int)threadIdx.x;
            Aff<T, CH, NSD> f = cf, b = cb;
            if (j < ng) {
                f = grp[j].fwd;
                b = grp[j].bwd;
            }
            f = wave_aff_scan<true>(f, 0, ih);  // groups 0..j
            b = wave_aff_scan<true>(b, 1, ih);  // groups ng-1 down to j
            // lane g - 1 / g + 1 holds what enters group g; the first and
            // the last group keep the identity
            if (g > 0 && j == g - 1)
                ent[0] = f;
            if (g + 1 < ng && j == g + 1)
                ent[1] = b;
            if (g == 0 && j == 0)
                ent[0] = cf;
            if (g + 1 == ng && j == 0)
                ent[1] = cb;
        }
        __syncthreads();
        cf = ent[0];
        cb = ent[1];
    } else {
        for (int64_t j = 0; j < g; ++j)
            cf = aff_then<true>(cf, grp[j].fwd, ih);
        for (int64_t j = ng - 1; j > g; --j)
            cb = aff_then<true>(cb, grp[j].bwd, ih);
    }
    if (q >= nt)
        return;
    const Aff<T, CH, NSD> ef = loc[q].fwd, eb = loc[q].bwd;
#pragma unroll
    for (int b = 0; b < kKB; ++b) {
        const T mf = aff_m<true>(ef, ih, b), mb = aff_m<true>(eb, ih, b);
#pragma unroll
        for (int s = 0; s < NSD; ++s)
#pragma unroll
            for (int c = 0; c < CH; ++c) {
                car[q].F[b][s][c] = mf * cf.l[b][s][c] + ef.l[b][s][c];
                car[q].B[b][s][c] = mb * cb.l[b][s][c] + eb.l[b][s][c];
            }
    }
}

// Workgroups per CU the apply pass asks the compiler to fit: the float64
// two-channel d = 2 variant otherwise takes every register of a SIMD (one
// wavefront each) for its two scans.
template <typename T, int CH, int NSD> constexpr int kapply_min_blocks() {
    return (std::is_same<T, double>::value && CH == 2 && NSD == 2) ? 2 : 1;
}

template <typename T, int CH, int NSD>
__global__ __launch_bounds__(256, (kapply_min_blocks<T, CH, NSD>())) void k_kapply(KLevelArgs L, KBatch kb,
                                                const KCarry<T, CH, NSD> *__restrict__ car,
                                                const double *hi,
                                                const uint32_t *__restrict__ hmap,
                                                double *lo) {
    __shared__ Aff<T, CH, NSD> buf[shfl_scan<T, CH>() ? 4 : 256];
    const int tid = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * kKTile + (int64_t)tid * kKItems;
    T alpha[kKItems + 1][kKB], f[kKItems][kKB], wv[kKItems][CH];
    int sd[kKItems];
    bool val[kKItems];
    ItemPos ps;
    load_items<T, CH, NSD>(L, kb, base, alpha, f, sd, wv, val, ps);
    double ih[kKB];
    scan_ih(kb, L.sc, ih);
    Aff<T, CH, NSD> fex, bex;
    if constexpr (shfl_scan<T, CH>()) {
        Aff<T, CH, NSD> fin, bin;
        block_aff_scan2<!tile_products<T>(), T, CH, NSD>(thread_aff<T, CH, NSD>(alpha, f, sd, wv, val, ps, 0), buf,
                                    0, fin, fex, ih);
        block_aff_scan2<!tile_products<T>(), T, CH, NSD>(thread_aff<T, CH, NSD>(alpha, f, sd, wv, val, ps, 1), buf,
                                    1, bin, bex, ih);
    } else {
        (void)block_aff_scan<!tile_products<T>(), T, CH, NSD>(thread_aff<T, CH, NSD>(alpha, f, sd, wv, val, ps, 0),
                                         buf, 0, ih);
        if (tid == 0)
            aff_identity(fex);
        else
            fex = aff_get<!tile_products<T>()>(buf, tid - 1);
        __syncthreads();
        (void)block_aff_scan<!tile_products<T>(), T, CH, NSD>(thread_aff<T, CH, NSD>(alpha, f, sd, wv, val, ps, 1),
                                         buf, 1, ih);
        if (tid == 255)
            aff_identity(bex);
        else
            bex = aff_get<!tile_products<T>()>(buf, tid + 1);
    }
    const KCarry<T, CH, NSD> &cr = car[blockIdx.x];
    T recv[kKItems][kKB][CH];
#pragma unroll
    for (int b = 0; b < kKB; ++b) {
        T st[NSD][CH];
        const T mf = aff_m<!tile_products<T>()>(fex, ih, b);
#pragma unroll
        for (int s = 0; s < NSD; ++s)
#pragma unroll
            for (int c = 0; c < CH; ++c)
                st[s][c] = mf * cr.F[b][s][c] + fex.l[b][s][c];
#pragma unroll
        for (int u = 0; u < kKItems; ++u) {
            const int o = L.oneside ? 0 : (sd[u] ^ (NSD - 1));
#pragma unroll
            for (int s = 0; s < NSD; ++s)
#pragma unroll
                for (int c = 0; c < CH; ++c)
                    st[s][c] *= alpha[u][b];
            T add[CH];
#pragma unroll
            for (int c = 0; c < CH; ++c) {
                recv[u][b][c] = get_side<T, CH, NSD>(st, o, c);
                add[c] = f[u][b] * wv[u][c];
            }
            add_side<T, CH, NSD>(st, sd[u], add);
        }
        const T mb = aff_m<!tile_products<T>()>(bex, ih, b);
#pragma unroll
        for (int s = 0; s < NSD; ++s)
#pragma unroll
            for (int c = 0; c < CH; ++c)
                st[s][c] = mb * cr.B[b][s][c] + bex.l[b][s][c];
#pragma unroll
        for (int u = kKItems - 1; u >= 0; --u) {
            const int o = L.oneside ? 0 : (sd[u] ^ (NSD - 1));
            if (!val[u])
                continue;
#pragma unroll
            for (int s = 0; s < NSD; ++s)
#pragma unroll
                for (int c = 0; c < CH; ++c)
                    st[s][c] *= alpha[u + 1][b];
            T add[CH];
#pragma unroll
            for (int c = 0; c < CH; ++c) {
                recv[u][b][c] = f[u][b] * (recv[u][b][c] + get_side<T, CH, NSD>(st, o, c));
                add[c] = f[u][b] * wv[u][c];
            }
            add_side<T, CH, NSD>(st, sd[u], add);
        }
    }
    // lo[p] = hi[hmap[p]] + this level's sums (hi == nullptr: zero; hmap ==
    // nullptr: hi[p], which may be lo itself).  All loads come before the
    // stores, which may overwrite them.
    // (a record of W doubles is 16-byte aligned: moved as double2)
    constexpr int W = kKB * CH;
    static_assert(W % 2 == 0, "records of whole double2");
    double2 hv[kKItems][W / 2];
#pragma unroll
    for (int u = 0; u < kKItems; ++u) {
        const int64_t p = base + u;
        const int64_t src = (hi && val[u]) ? (hmap ? (int64_t)hmap[p] : p) : -1;
#pragma unroll
        for (int i = 0; i < W / 2; ++i)
            hv[u][i] = src >= 0 ? reinterpret_cast<const double2 *>(hi + src * W)[i]
                                : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int u = 0; u < kKItems; ++u) {
        const int64_t p = base + u;
        if (!val[u])
            continue;
        double2 *a = reinterpret_cast<double2 *>(lo + p * W);
#pragma unroll
        for (int i = 0; i < W / 2; ++i) {
            const int b0 = (2 * i) / CH, c0 = (2 * i) % CH;
            const int b1 = (2 * i + 1) / CH, c1 = (2 * i + 1) % CH;
            a[i] = make_double2(hv[u][i].x + (double)recv[u][b0][c0],
                                hv[u][i].y + (double)recv[u][b1][c1]);
        }
    }
}

// lo[p] = hi[map[p]] (map == nullptr: hi[p]), added to lo[p] when add != 0
template <int CH>
__global__ __launch_bounds__(256) void k_kacc_down(const double *__restrict__ hi,
                                                   const uint32_t *__restrict__ map, int64_t n,
                                                   double *__restrict__ lo, int add) {
    // one thread per double of the [n][kKB * CH] arrays: stores coalesced,
    // each record gathered by kKB * CH neighbouring threads
    constexpr int W = kKB * CH;
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= n * W)
        return;
    const int64_t p = e / W;
    const int q = (int)(e - p * W);
    const double v = hi[(map ? (int64_t)map[p] : p) * W + q];
    lo[e] = add ? lo[e] + v : v;
}

__global__ void k_kzero(double *a, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n)
        a[i] = 0.0;
}

__global__ void k_kzero_u32(uint32_t *a, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        a[i] = 0u;
}

// Leave-one-out sums below this are re-evaluated exactly (k_kloo_exact): a
// term lost in the scans is below the smallest normal number of the scan type
// (2.2e-308 in float64, 1.2e-38 in float32), and at most N x (levels) of them
// reach one item, so a sum above the threshold is within about 1e-18
// (float64) / 1e-8 (float32) of its exact value relative to itself.
template <typename T> constexpr double loo_tiny();
template <> constexpr double loo_tiny<double>() { return 1e-280; }
template <> constexpr double loo_tiny<float>() { return 1e-22; }
constexpr int kLooExactGroups = 256;
constexpr int kLooPartGroups = 2048;

// Direct sums inside each 64-item block of a state (one wavefront per block):
// acc[p] += sum over the block's items j != p (with a different bit-0 side
// when need_diff) of w_j exp(-sum_k |x_k,p - x_k,j| / h_k).  Each unordered
// pair is evaluated once: for offsets o = 1..32, lane l pairs with lane
// (l + o) mod 64 (at o = 32 only lanes below 32 do), keeps its own share and
// hands the partner's share to it by a shuffle; sums are taken in o order.
template <typename T, int CH>
__global__ __launch_bounds__(256) void k_kblock_pairs(KState st, int d, int64_t n, KBatch kb,
                                                      int need_diff, double *__restrict__ acc) {
    const int lane = threadIdx.x & 63;
    const int64_t blk = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int64_t p = blk * 64 + lane;
    if (blk * 64 >= n)
        return;
    const int cnt = (int)((n - blk * 64) < 64 ? (n - blk * 64) : 64);
    const bool v = lane < cnt;
    double xx[3], w0 = 0.0, w1 = 0.0;
    int side = 0;
    for (int k = 0; k < 3; ++k)
        xx[k] = v ? st.x[k][p] : 0.0;
    if (v) {
        w0 = st.w0[p];
        w1 = st.w1[p];
        side = st.bits[p] & 1;
    }
    double sum[kKB][CH];
#pragma unroll
    for (int b = 0; b < kKB; ++b)
#pragma unroll
        for (int c = 0; c < CH; ++c)
            sum[b][c] = 0.0;
    for (int o = 1; o <= 32; ++o) {
        const int q = (lane + o) & 63;
        const double y0 = shfl(xx[0], q), y1 = shfl(xx[1], q), y2 = shfl(xx[2], q);
        const double u0 = shfl(w0, q), u1 = shfl(w1, q);
        const int sq = __shfl(side, q, 64);
        const bool pair = v && q < cnt && !(need_diff && sq == side) && (o < 32 || lane < 32);
        double give[kKB][CH];
        const double e0 = fabs(xx[0] - y0), e1 = d > 1 ? fabs(xx[1] - y1) : 0.0,
                     e2 = d > 2 ? fabs(xx[2] - y2) : 0.0;
#pragma unroll
        for (int b = 0; b < kKB; ++b) {
            const T kv =
                pair ? kexp<T>((T)(-(e0 * kb.ih[b][0] + e1 * kb.ih[b][1] + e2 * kb.ih[b][2])))
                     : T(0);
            sum[b][0] += (double)((T)u0 * kv);
            give[b][0] = (double)((T)w0 * kv);
            if (CH > 1) {
                sum[b][CH - 1] += (double)((T)u1 * kv);
                give[b][CH - 1] = (double)((T)w1 * kv);
            }
        }
        // the share of lane (lane - o) mod 64, whose partner this lane is
        const int from = (lane - o) & 63;
#pragma unroll
        for (int b = 0; b < kKB; ++b)
#pragma unroll
            for (int c = 0; c < CH; ++c)
                sum[b][c] += shfl(give[b][c], from);
    }
    if (!v)
        return;
    double *a = acc + p * (kKB * CH);
#pragma unroll
    for (int b = 0; b < kKB; ++b)
#pragma unroll
        for (int c = 0; c < CH; ++c)
            a[b * CH + c] += sum[b][c];
}

// Outputs and per-point score terms from the leave-one-out sums (x1 order).
// mode 0: KDE (channel 0 = w); mode 1: NW (channel 0 = 1, channel 1 = y).
// Per item (x1-sorted order) and bandwidth of the batch: the LOO score term,
// log fhat_{-j} (mode 0) or the squared LOO residual (mode 1).
//
// A leave-one-out sum of channel 0 (the density, or the regression
// denominator) below `tiny` may have lost terms that fell below the smallest
// normal number of the scan's type on the way (every stored factor is <= 1,
// so a lost term is smaller than that number); such an item is appended to
// `list` (entry p * kKB + b; cnt counts them, capacity n * kKB) and its score
// term is left to k_kloo_exact.
template <int CH>
__global__ __launch_bounds__(256) void k_kfinish(const double *__restrict__ acc, KState st,
                                                 int64_t n, KBatch kb, int mode, double tiny,
                                                 double *__restrict__ terms,
                                                 uint32_t *__restrict__ cnt,
                                                 uint32_t *__restrict__ list) {
    int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= n)
        return;
    const double *a = acc + p * (kKB * CH);
    const double w1 = st.w1[p];
    for (int b = 0; b < kb.nb; ++b) {
        const double den = a[b * CH];
        if (!(den >= tiny)) {
            const uint32_t slot = atomicAdd(cnt, 1u);
            list[slot] = (uint32_t)p * kKB + (uint32_t)b;
            continue;
        }
        double t;
        if (mode == 0) {
            t = log(den * kb.norm_loo[b]);
        } else {
            double num = a[b * CH + CH - 1];
            double e = w1 - num / den;
            t = e * e;
        }
        terms[(int64_t)b * n + p] = t;
    }
}

// The score term of an item from its sums relative to the nearest point.
template <int CH>
__device__ __forceinline__ double loo_term(const LooAcc<CH> &r, int mode, double norm_loo,
                                           double yj) {
    if (mode == 0)
        return -r.m + log((r.s[0] + r.c[0]) * norm_loo);
    const double ratio = (r.s[CH - 1] + r.c[CH - 1]) / (r.s[0] + r.c[0]);
    const double er = yj - ratio;
    return er * er;
}

// The score terms of the items k_kfinish set aside, by a sum over every other
// point of the sample.  The first kLooCap items of the list: work units of
// kLooQ items and one of nch chunks of the points (k_kloo_part), each chunk's
// sums combined in a fixed tree of its workgroup, then the chunks of an item
// in order (k_kloo_fin).  Items past kLooCap: one workgroup each, all points
// (k_kloo_exact).  Workgroups step through the units; every one reads the
// same count, so all of them leave the loop together.
constexpr int kLooQ = 4;
constexpr uint32_t kLooCap = 4096;
constexpr int kLooMaxChunks = 64;

template <int CH>
__device__ __forceinline__ void loo_block_reduce(LooAcc<CH> a, LooAcc<CH> *buf, int t) {
    buf[t] = a;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (t < off) {
            LooAcc<CH> x = buf[t];
            loo_merge(x, buf[t + off]);
            buf[t] = x;
        }
        __syncthreads();
    }
}

template <int CH>
__global__ __launch_bounds__(256) void k_kloo_part(KState st, int d, int64_t n, KBatch kb,
                                                   const uint32_t *__restrict__ cnt,
                                                   const uint32_t *__restrict__ list, int nch,
                                                   int64_t chunk, LooAcc<CH> *__restrict__ part) {
    __shared__ LooAcc<CH> buf[256];
    const int t = threadIdx.x;
    const uint32_t nf = *cnt < kLooCap ? *cnt : kLooCap;
    const uint32_t units = ((nf + kLooQ - 1) / kLooQ) * (uint32_t)nch;
    for (uint32_t u = blockIdx.x; u < units; u += gridDim.x) {
        const uint32_t g = u / (uint32_t)nch;
        const int c = (int)(u % (uint32_t)nch);
        const uint32_t q0 = g * kLooQ;
        int64_t qp[kLooQ];
        double qx[kLooQ][3], qih[kLooQ][3];
        LooAcc<CH> acc[kLooQ];
#pragma unroll
        for (int q = 0; q < kLooQ; ++q) {
            const bool vq = q0 + q < nf;
            const uint32_t e = vq ? list[q0 + q] : 0u;
            qp[q] = vq ? (int64_t)(e / kKB) : -1;
            const int b = (int)(e % kKB);
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                qx[q][k] = (vq && k < d) ? st.x[k][qp[q]] : 0.0;
                qih[q][k] = k < d ? kb.ih[b][k] : 0.0;
            }
            loo_init(acc[q]);
        }
        const int64_t i0 = (int64_t)c * chunk;
        const int64_t i1 = i0 + chunk < n ? i0 + chunk : n;
        for (int64_t i = i0 + t; i < i1; i += 256) {
            double xi[3];
#pragma unroll
            for (int k = 0; k < 3; ++k)
                xi[k] = k < d ? st.x[k][i] : 0.0;
            double w[CH];
            w[0] = st.w0[i];
            if (CH > 1)
                w[CH - 1] = st.w1[i];
#pragma unroll
            for (int q = 0; q < kLooQ; ++q) {
                if (qp[q] < 0 || i == qp[q])
                    continue;
                double ei = 0.0;
#pragma unroll
                for (int k = 0; k < 3; ++k)
                    ei += fabs(xi[k] - qx[q][k]) * qih[q][k];
                loo_add(acc[q], ei, exp(-fabs(ei - acc[q].m)), w);
            }
        }
#pragma unroll
        for (int q = 0; q < kLooQ; ++q) {
            loo_block_reduce(acc[q], buf, t);
            if (t == 0 && q0 + q < nf)
                part[(int64_t)(q0 + q) * nch + c] = buf[0];
            __syncthreads();  // buf is rewritten next
        }
    }
}

template <int CH>
__global__ __launch_bounds__(256) void k_kloo_fin(KState st, int64_t n, KBatch kb, int mode,
                                                  const uint32_t *__restrict__ cnt,
                                                  const uint32_t *__restrict__ list, int nch,
                                                  const LooAcc<CH> *__restrict__ part,
                                                  double *__restrict__ terms) {
    const uint32_t nf = *cnt < kLooCap ? *cnt : kLooCap;
    const uint32_t f = blockIdx.x * 256 + threadIdx.x;
    if (f >= nf)
        return;
    const uint32_t e = list[f];
    const int64_t p = e / kKB;
    const int b = (int)(e % kKB);
    LooAcc<CH> r = part[(int64_t)f * nch];
    for (int c = 1; c < nch; ++c)
        loo_merge(r, part[(int64_t)f * nch + c]);
    terms[(int64_t)b * n + p] = loo_term(r, mode, kb.norm_loo[b], st.w1[p]);
}

template <int CH>
__global__ __launch_bounds__(256) void k_kloo_exact(KState st, int d, int64_t n, KBatch kb,
                                                    int mode, const uint32_t *__restrict__ cnt,
                                                    const uint32_t *__restrict__ list,
                                                    double *__restrict__ terms) {
    __shared__ LooAcc<CH> part[256];
    const int t = threadIdx.x;
    const uint32_t nf = *cnt;
    for (uint32_t u = kLooCap + blockIdx.x; u < nf; u += gridDim.x) {
        const uint32_t e = list[u];
        const int64_t p = e / kKB;
        const int b = (int)(e % kKB);
        double q[3], ih[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            q[k] = k < d ? st.x[k][p] : 0.0;
            ih[k] = k < d ? kb.ih[b][k] : 0.0;
        }
        LooAcc<CH> a;
        loo_init(a);
        for (int64_t i = t; i < n; i += 256) {
            if (i == p)
                continue;
            double ei = 0.0;
#pragma unroll
            for (int k = 0; k < 3; ++k)
                if (k < d)
                    ei += fabs(st.x[k][i] - q[k]) * ih[k];
            double w[CH];
            w[0] = st.w0[i];
            if (CH > 1)
                w[CH - 1] = st.w1[i];
            loo_add(a, ei, exp(-fabs(ei - a.m)), w);
        }
        loo_block_reduce(a, part, t);
        if (t == 0)
            terms[(int64_t)b * n + p] = loo_term(part[0], mode, kb.norm_loo[b], st.w1[p]);
        __syncthreads();  // part[] is rewritten for the next item
    }
}

// ------------------------------------------------ direct sums, d = 4 .. 6
// For d >= 4 the orthant recursion would need one nested split per extra
// coordinate (2^(d-1) running sums per item and O(N log^(d-1) N) work); the
// sums are evaluated here directly, every (query, point) pair, relative to
// the query's nearest point as above.  One thread per query (input order),
// the points staged 256 at a time through LDS and read as broadcasts, every
// bandwidth of the batch from the same staged distances.
struct KBatchD {
    double ih[kKB][MECDF_MAX_DIM];
    double norm_full[kKB];
    double norm_loo[kKB];
    int nb;
};

template <typename T, int CH, typename WT, typename OutT>
__global__ __launch_bounds__(256) void k_kdirect(const double *__restrict__ x, int d, int64_t n,
                                                 const WT *__restrict__ w0in,
                                                 const WT *__restrict__ w1in, KBatchD kb, int b0,
                                                 int mode, OutT *__restrict__ out,
                                                 double *__restrict__ terms) {
    __shared__ double sx[MECDF_MAX_DIM][256];
    __shared__ double sw[CH][256];
    const int t = threadIdx.x;
    const int64_t j = (int64_t)blockIdx.x * 256 + t;
    const bool vq = j < n;
    double q[MECDF_MAX_DIM];
#pragma unroll
    for (int k = 0; k < MECDF_MAX_DIM; ++k)
        q[k] = (vq && k < d) ? x[(int64_t)k * n + j] : 0.0;
    LooAcc<CH> acc[kKB];
#pragma unroll
    for (int b = 0; b < kKB; ++b)
        loo_init(acc[b]);
    for (int64_t t0 = 0; t0 < n; t0 += 256) {
        const int64_t i = t0 + t;
        __syncthreads();  // the previous tile has been read
#pragma unroll
        for (int k = 0; k < MECDF_MAX_DIM; ++k)
            if (k < d)
                sx[k][t] = i < n ? x[(int64_t)k * n + i] : 0.0;
        sw[0][t] = i < n ? (w0in ? (double)w0in[i] : 1.0) : 0.0;
        if (CH > 1)
            sw[CH - 1][t] = i < n ? (double)w1in[i] : 0.0;
        __syncthreads();
        const int cnt = (n - t0) < 256 ? (int)(n - t0) : 256;
        for (int u = 0; u < cnt; ++u) {
            if (t0 + u == j)
                continue;
            double dk[MECDF_MAX_DIM];
#pragma unroll
            for (int k = 0; k < MECDF_MAX_DIM; ++k)
                dk[k] = k < d ? fabs(sx[k][u] - q[k]) : 0.0;
            double w[CH];
            w[0] = sw[0][u];
            if (CH > 1)
                w[CH - 1] = sw[CH - 1][u];
#pragma unroll
            for (int b = 0; b < kKB; ++b) {
                if (b >= kb.nb)
                    break;
                double e = 0.0;
#pragma unroll
                for (int k = 0; k < MECDF_MAX_DIM; ++k)
                    e += dk[k] * kb.ih[b][k];
                const T f = kexp<T>((T)(-fabs(e - acc[b].m)));
                loo_add(acc[b], e, (double)f, w);
            }
        }
    }
    if (!vq)
        return;
    const double w0j = w0in ? (double)w0in[j] : 1.0;
    const double w1j = w1in ? (double)w1in[j] : 0.0;
#pragma unroll
    for (int b = 0; b < kKB; ++b) {
        if (b >= kb.nb)
            break;
        const double s0 = acc[b].s[0] + acc[b].c[0];
        const double s1 = acc[b].s[CH - 1] + acc[b].c[CH - 1];
        const double em = exp(-acc[b].m);
        if (out) {
            const double o = mode == 0 ? (w0j + em * s0) * kb.norm_full[b]
                                       : (w1j + em * s1) / (1.0 + em * s0);
            out[(int64_t)(b0 + b) * n + j] = (OutT)o;
        }
        if (terms) {
            double v;
            if (mode == 0) {
                v = -acc[b].m + log(s0 * kb.norm_loo[b]);
            } else {
                const double er = w1j - s1 / s0;
                v = er * er;
            }
            terms[(int64_t)b * n + j] = v;
        }
    }
}

// inv[ids[p]] = p: position of input point i in the x1-sorted order
__global__ __launch_bounds__(256) void k_kinv(const uint32_t *__restrict__ ids, int64_t n,
                                              uint32_t *__restrict__ inv) {
    int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p < n)
        inv[ids[p]] = (uint32_t)p;
}

// The full estimates in input order: point i reads its accumulator record
// (all bandwidths of the batch at once, as 16-byte vectors) from its sorted
// position and its own weights from the caller's arrays in input order (the
// same values the sorted state holds at that position), and each bandwidth's
// row is written coalesced: the density with the point itself (mode 0) or the
// regression ratio with it (mode 1).
template <int CH, typename OutT, typename WT>
__global__ __launch_bounds__(256) void k_kout(const double *__restrict__ acc,
                                              const uint32_t *__restrict__ inv, int64_t n,
                                              KBatch kb, int b0, int mode,
                                              const WT *__restrict__ w0in,
                                              const WT *__restrict__ w1in,
                                              OutT *__restrict__ out) {
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n)
        return;
    const int64_t p = inv[i];
    constexpr int W = kKB * CH;
    static_assert(W % 2 == 0, "records of whole double2");
    const double2 *a = reinterpret_cast<const double2 *>(acc + p * W);
    double r[W];
#pragma unroll
    for (int q = 0; q < W / 2; ++q) {
        const double2 v = a[q];
        r[2 * q] = v.x;
        r[2 * q + 1] = v.y;
    }
    const double w0 = w0in ? (double)w0in[i] : 1.0;
    const double w1 = w1in ? (double)w1in[i] : 0.0;
#pragma unroll
    for (int b = 0; b < kKB; ++b) {
        if (b >= kb.nb)
            break;
        double o;
        if (mode == 0)
            o = (r[b * CH] + w0) * kb.norm_full[b];
        else
            o = (r[b * CH + CH - 1] + w1) / (r[b * CH] + 1.0);
        out[(int64_t)(b0 + b) * n + i] = (OutT)o;
    }
}

// deterministic mean of each row of terms[nb][n]: fixed chunks summed by one
// block each (fixed tree), then the chunk sums of a row by one block
constexpr int kMeanChunk = 4096;

__global__ __launch_bounds__(256) void k_kpartial(const double *__restrict__ terms, int64_t n,
                                                  int64_t nch, double *__restrict__ part) {
    __shared__ double buf[256];
    const int64_t c = blockIdx.x;
    const int b = blockIdx.y;
    const int64_t i0 = c * kMeanChunk;
    double s = 0.0;
    for (int u = 0; u < kMeanChunk / 256; ++u) {
        int64_t i = i0 + (int64_t)u * 256 + threadIdx.x;
        if (i < n)
            s += terms[(int64_t)b * n + i];
    }
    buf[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            buf[threadIdx.x] += buf[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        part[(int64_t)b * nch + c] = buf[0];
}

__global__ __launch_bounds__(256) void k_kmean(const double *__restrict__ part, int64_t nch,
                                               int64_t n, int b0, double *__restrict__ score) {
    __shared__ double buf[256];
    const int b = blockIdx.x;
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < nch; i += 256)
        s += part[(int64_t)b * nch + i];
    buf[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            buf[threadIdx.x] += buf[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        score[b0 + b] = buf[0] / (double)n;
}

static void launch_mean(const double *terms, int64_t n, int nbh, int b0, double *part,
                        double *score, hipStream_t s) {
    int64_t nch = ceil_div(n, kMeanChunk);
    hipLaunchKernelGGL(k_kpartial, dim3((unsigned)nch, (unsigned)nbh), dim3(256), 0, s, terms,
                       n, nch, part);
    hipLaunchKernelGGL(k_kmean, dim3((unsigned)nbh), dim3(256), 0, s, part, nch, n, b0, score);
}

// ----------------------------------------------------------- host driver
static KState take_state(Arena &a, int64_t n) {
    KState s;
    for (int k = 0; k < 3; ++k)
        s.x[k] = a.take<double>((size_t)n);
    s.w0 = a.take<double>((size_t)n);
    s.w1 = a.take<double>((size_t)n);
    s.bits = a.take<uint8_t>((size_t)n);
    s.map = a.take<uint32_t>((size_t)n);
    return s;
}
static void plan_state(ArenaPlan &pl, int64_t n) {
    for (int k = 0; k < 5; ++k)
        pl.add<double>((size_t)n);
    pl.add<uint8_t>((size_t)n);
    pl.add<uint32_t>((size_t)n);
}

template <typename T, int CH, int NSD>
static int run_scan(const KLevelArgs &la, const KBatch &kb, int64_t nt, void *agg_raw,
                    void *grp_raw, void *car_raw, const double *hi, const uint32_t *hmap,
                    double *lo, hipStream_t s) {
    auto *agg = reinterpret_cast<KTileAgg<T, CH, NSD> *>(agg_raw);
    auto *grp = reinterpret_cast<KTileAgg<T, CH, NSD> *>(grp_raw);
    auto *car = reinterpret_cast<KCarry<T, CH, NSD> *>(car_raw);
    // the kernels find an item's segment and split blocks with bit masks
    auto pow2 = [](int64_t v) { return v > 0 && (v & (v - 1)) == 0; };
    if (!pow2(la.ha) || !pow2(la.hb) || !pow2(la.hin)) {
        set_error("kernel sums: block sizes must be powers of two");
        return MECDF_EINVAL;
    }
    const unsigned ng = (unsigned)ceil_div(nt, (int64_t)256);
    {
        ProfScope prof("kde_tile_agg", s);
        hipLaunchKernelGGL((k_ktile_agg<T, CH, NSD>), dim3((unsigned)nt), dim3(256), 0, s, la,
                           kb, agg);
    }
    {
    ProfScope prof("kde_carry", s);
    if (ng == 1) {
        hipLaunchKernelGGL((k_kcarry_local<T, CH, NSD>), dim3(1), dim3(256), 0, s, agg, nt, grp,
                           car, kb, la.sc);
    } else {
        hipLaunchKernelGGL((k_kcarry_local<T, CH, NSD>), dim3(ng), dim3(256), 0, s, agg, nt, grp,
                           (KCarry<T, CH, NSD> *)nullptr, kb, la.sc);
        hipLaunchKernelGGL((k_kcarry_final<T, CH, NSD>), dim3(ng), dim3(256), 0, s, agg, nt,
                           grp, car, kb, la.sc);
    }
    }
    ProfScope prof("kde_apply", s);
    hipLaunchKernelGGL((k_kapply<T, CH, NSD>), dim3((unsigned)nt), dim3(256), 0, s, la, kb, car,
                       hi, hmap, lo);
    MECDF_LAUNCH_CHECK();
    return MECDF_OK;
}

template <typename T, int CH, typename WT, typename OutT>
static int kde_run_t(int d, int64_t n, const double *x, const WT *w0in, const WT *w1in,
                     int nh, const double *h, OutT *out, double *score, int mode,
                     hipStream_t s) {
    // outer merge levels (x1 split): blocks of hs[q] merged into 2 hs[q]
    std::vector<int64_t> hs;
    if (d >= 2)
        for (int64_t hh = kKT; hh < n; hh *= 2)
            hs.push_back(hh);
    const int L = (int)hs.size();
    const int64_t nt = ceil_div(n, kKTile);
    const int64_t nacc = n * kKB * CH;
    // inner levels (d = 3): inside blocks of 2 hs[q], the 64-block sort then
    // merges of h2 = 64 .. hs[q]
    std::vector<int> inner_count(L, 0);
    int nstates = 1 + (d >= 2 ? L + 1 : 0);
    if (d == 3)
        for (int q = 0; q < L; ++q) {
            int c = 1;
            for (int64_t h2 = kKT; h2 <= hs[q]; h2 *= 2)
                ++c;
            inner_count[q] = c;
            nstates += c;
        }
    ArenaPlan pl;
    for (int q = 0; q < 3; ++q)
        pl.add<uint64_t>((size_t)n);
    for (int q = 0; q < 3; ++q)
        pl.add<uint32_t>((size_t)n);
    pl.add<uint32_t>((size_t)n);  // ids
    pl.add<uint32_t>((size_t)n);  // inv
    for (int q = 0; q < nstates; ++q)
        plan_state(pl, n);
    for (int q = 0; q < 4; ++q)
        pl.add<double>((size_t)nacc);
    pl.add<double>((size_t)n * kKB);
    pl.add<KTileAgg<T, CH, 4>>((size_t)nt + 1);
    pl.add<KTileAgg<T, CH, 4>>((size_t)ceil_div(nt, (int64_t)256) + 1);  // tile groups
    pl.add<KCarry<T, CH, 4>>((size_t)nt + 1);
    pl.add<double>((size_t)(ceil_div(n, kMeanChunk) * kKB));
    pl.add<uint32_t>(64);                 // count of items set aside
    pl.add<uint32_t>((size_t)n * kKB);    // their list
    const int loo_nch = (int)std::min<int64_t>(kLooMaxChunks, ceil_div(n, 4096));
    const int64_t loo_chunk = ceil_div(n, loo_nch);
    pl.add<LooAcc<CH>>((size_t)kLooCap * loo_nch);
    radix_plan(pl, n);
    void *wsb = nullptr;
    MECDF_TRY(workspace_reserve(pl.used, &wsb));
    Arena a;
    a.base = (char *)wsb;
    uint64_t *k0 = a.take<uint64_t>(n), *k1 = a.take<uint64_t>(n), *k2 = a.take<uint64_t>(n);
    uint32_t *i0 = a.take<uint32_t>(n), *i1 = a.take<uint32_t>(n), *i2 = a.take<uint32_t>(n);
    uint32_t *ids = a.take<uint32_t>(n);
    uint32_t *inv = a.take<uint32_t>(n);
    KState S0 = take_state(a, n);
    std::vector<KState> So(d >= 2 ? L + 1 : 0);  // So[0]: 64-blocks by x2; So[q+1]: merged 2 hs[q]
    for (auto &st : So)
        st = take_state(a, n);
    std::vector<std::vector<KState>> Si(L);       // inner states of So[q+1]
    if (d == 3)
        for (int q = 0; q < L; ++q) {
            Si[q].resize(inner_count[q]);
            for (auto &st : Si[q])
                st = take_state(a, n);
        }
    double *acc[4];
    for (int q = 0; q < 4; ++q)
        acc[q] = a.take<double>((size_t)nacc);
    double *terms = a.take<double>((size_t)n * kKB);
    void *agg = a.take<KTileAgg<T, CH, 4>>((size_t)nt + 1);
    void *grp = a.take<KTileAgg<T, CH, 4>>((size_t)ceil_div(nt, (int64_t)256) + 1);
    void *car = a.take<KCarry<T, CH, 4>>((size_t)nt + 1);
    double *mpart = a.take<double>((size_t)(ceil_div(n, kMeanChunk) * kKB));
    uint32_t *aside_cnt = a.take<uint32_t>(64);
    uint32_t *aside = a.take<uint32_t>((size_t)n * kKB);
    LooAcc<CH> *loo_part = a.take<LooAcc<CH>>((size_t)kLooCap * loo_nch);
    RadixScratch rs = radix_take(a, n);
    const unsigned nb = (unsigned)ceil_div(n, 256);
    const unsigned nbw = (unsigned)ceil_div(ceil_div(n, 64), 4);
    const unsigned nba = (unsigned)ceil_div(nacc, 256);
    // inner map from So[q+1] to its 64-block state (the outer map So[q+1].map
    // is taken by the next outer merge)
    std::vector<uint32_t *> imap(L, nullptr);

    // ---- h-independent structure
    {
        ProfScope prof("kde_build", s);
        hipLaunchKernelGGL(k_kx_keys, dim3(nb), dim3(256), 0, s, x, n, k0, i0);
        int which = 0;
        MECDF_TRY((radix_sort_bits<uint64_t, uint32_t>(k0, i0, k1, i1, k2, i2, n, 0, 64, rs, s,
                                                       &which)));
        uint32_t *idx = which == 1 ? i1 : (which == 2 ? i2 : i0);
        hipLaunchKernelGGL((k_kgather0<WT>), dim3(nb), dim3(256), 0, s, idx, n, d, x, w0in, w1in,
                           S0, ids);
        if (out)
            hipLaunchKernelGGL(k_kinv, dim3(nb), dim3(256), 0, s, ids, n, inv);
        if (d >= 2) {
            hipLaunchKernelGGL(k_kblocksort, dim3(nbw), dim3(256), 0, s, S0, 1, n, So[0], S0.map);
            for (int q = 0; q < L; ++q)
                hipLaunchKernelGGL(k_kmerge, dim3(nb), dim3(256), 0, s, So[q], 1, n, hs[q], 0,
                                   So[q + 1]);
            if (d == 3) {
                // the last inner state is never merged further, so its map
                // slot holds the map of the 64-block sort of So[q+1]
                for (int q = 0; q < L; ++q) {
                    std::vector<KState> &I = Si[q];
                    imap[q] = I.back().map;
                    hipLaunchKernelGGL(k_kblocksort, dim3(nbw), dim3(256), 0, s, So[q + 1], 2, n,
                                       I[0], imap[q]);
                    int64_t h2 = kKT;
                    for (int r = 1; r < inner_count[q]; ++r, h2 *= 2)
                        hipLaunchKernelGGL(k_kmerge, dim3(nb), dim3(256), 0, s, I[r - 1], 2, n, h2,
                                           1, I[r]);
                }
            }
        }
        MECDF_LAUNCH_CHECK();
    }

    for (int b0 = 0; b0 < nh; b0 += kKB) {
        const int bcount = nh - b0 < kKB ? nh - b0 : kKB;
        KBatch kb{};
        kb.nb = bcount;
        for (int b = 0; b < kKB; ++b) {
            int bb = b0 + (b < kb.nb ? b : 0);
            double prod = 1.0;
            for (int k = 0; k < 3; ++k) {
                kb.ih[b][k] = k < d ? 1.0 / h[bb * d + k] : 0.0;
                if (k < d)
                    prod *= h[bb * d + k];
            }
            kb.norm_full[b] = 1.0 / ((double)(1 << d) * (double)n * prod);
            kb.norm_loo[b] = 1.0 / ((double)(1 << d) * (double)(n - 1) * prod);
        }
        double *ao = acc[0], *an = acc[1];  // outer accumulator ping-pong
        // the levels of d = 1, and of d = 2 when there are any, write every
        // accumulator record themselves
        if (d == 3 || (d == 2 && L == 0))
            hipLaunchKernelGGL(k_kzero, dim3(nba), dim3(256), 0, s, ao, nacc);
        if (d == 1) {
            KLevelArgs la{S0.x[0], 0, nullptr, nullptr, 1, nullptr, nullptr, 1,
                          S0.w0, S0.w1, S0.bits, n, (int64_t)1 << 40, 1};
            MECDF_TRY((run_scan<T, CH, 1>(la, kb, nt, agg, grp, car, nullptr, nullptr, ao, s)));
        } else {
            for (int q = L - 1; q >= 0; --q) {
                const KState &M = So[q + 1];  // blocks of 2 hs[q] sorted by x2, bit 0 = side
                if (d == 2) {
                    // the level above's accumulator comes in through its merge
                    // map (none above the top level)
                    KLevelArgs la{M.x[1], 1, M.x[0], S0.x[0], hs[q], nullptr, nullptr, 1,
                                  M.w0, M.w1, M.bits, n, hs[q], 0};
                    const bool top = q == L - 1;
                    MECDF_TRY((run_scan<T, CH, 2>(la, kb, nt, agg, grp, car, top ? nullptr : ao,
                                                  top ? nullptr : So[q + 1].map, an, s)));
                    std::swap(ao, an);
                    if (q == 0) {
                        ProfScope prof2("kde_down", s);
                        hipLaunchKernelGGL((k_kacc_down<CH>), dim3(nba), dim3(256), 0, s, ao,
                                           So[0].map, n, an, 0);
                        std::swap(ao, an);
                    }
                    continue;
                } else {
                    std::vector<KState> &I = Si[q];
                    double *ai = acc[2], *aj = acc[3];
                    hipLaunchKernelGGL(k_kzero, dim3(nba), dim3(256), 0, s, ai, nacc);
                    // inner levels, top down: I[r] holds blocks of 2 h2 (h2 = 64 << (r-1))
                    for (int r = inner_count[q] - 1; r >= 1; --r) {
                        const int64_t h2 = (int64_t)kKT << (r - 1);
                        const KState &Mi = I[r];
                        KLevelArgs la{Mi.x[2], 2, Mi.x[0], S0.x[0], hs[q], Mi.x[1], M.x[1], h2,
                                      Mi.w0, Mi.w1, Mi.bits, n, h2, 0};
                        MECDF_TRY((run_scan<T, CH, 4>(la, kb, nt, agg, grp, car, ai, nullptr,
                                                      ai, s)));
                        hipLaunchKernelGGL((k_kacc_down<CH>), dim3(nba), dim3(256), 0, s, ai,
                                           I[r - 1].map, n, aj, 0);
                        std::swap(ai, aj);
                    }
                    // ai in I[0] order (64-blocks of M sorted by x3): back to M order
                    hipLaunchKernelGGL((k_kacc_down<CH>), dim3(nba), dim3(256), 0, s, ai, imap[q],
                                       n, aj, 0);
                    // pairs inside the inner 64-blocks (M order) with different x1 sides
                    hipLaunchKernelGGL((k_kblock_pairs<T, CH>), dim3(nbw), dim3(256), 0, s, M, d,
                                       n, kb, 1, aj);
                    hipLaunchKernelGGL((k_kacc_down<CH>), dim3(nba), dim3(256), 0, s, aj, nullptr,
                                       n, ao, 1);
                    MECDF_LAUNCH_CHECK();
                }
                ProfScope prof2("kde_down", s);
                hipLaunchKernelGGL((k_kacc_down<CH>), dim3(nba), dim3(256), 0, s, ao, So[q].map, n,
                                   an, 0);
                std::swap(ao, an);
            }
            // ao in So[0] order (64-blocks of S0 sorted by x2): back to S0 order
            hipLaunchKernelGGL((k_kacc_down<CH>), dim3(nba), dim3(256), 0, s, ao, S0.map, n, an, 0);
            std::swap(ao, an);
            ProfScope prof3("kde_block_pairs", s);
            hipLaunchKernelGGL((k_kblock_pairs<T, CH>), dim3(nbw), dim3(256), 0, s, S0, d, n, kb,
                               0, ao);
        }
        {
            ProfScope prof("kde_finish", s);
            if (score) {
                hipLaunchKernelGGL(k_kzero_u32, dim3(1), dim3(64), 0, s, aside_cnt, 1);
                hipLaunchKernelGGL((k_kfinish<CH>), dim3(nb), dim3(256), 0, s, ao, S0, n, kb,
                                   mode, loo_tiny<T>(), terms, aside_cnt, aside);
                ProfScope prof4("kde_loo_exact", s);
                hipLaunchKernelGGL((k_kloo_part<CH>), dim3(kLooPartGroups), dim3(256), 0, s, S0,
                                   d, n, kb, aside_cnt, aside, loo_nch, loo_chunk, loo_part);
                hipLaunchKernelGGL((k_kloo_fin<CH>), dim3(kLooCap / 256), dim3(256), 0, s, S0, n,
                                   kb, mode, aside_cnt, aside, loo_nch, loo_part, terms);
                hipLaunchKernelGGL((k_kloo_exact<CH>), dim3(kLooExactGroups), dim3(256), 0, s,
                                   S0, d, n, kb, mode, aside_cnt, aside, terms);
            }
            if (out)
                hipLaunchKernelGGL((k_kout<CH, OutT, WT>), dim3(nb), dim3(256), 0, s, ao, inv,
                                   n, kb, b0, mode, w0in, w1in, out);
            if (score)
                launch_mean(terms, n, kb.nb, b0, mpart, score, s);
        }
        MECDF_LAUNCH_CHECK();
    }
    return MECDF_OK;
}

template <typename T, int CH, typename WT, typename OutT>
static int kde_direct_t(int d, int64_t n, const double *x, const WT *w0in, const WT *w1in,
                        int nh, const double *h, OutT *out, double *score, int mode,
                        hipStream_t s) {
    ArenaPlan pl;
    pl.add<double>((size_t)n * kKB);
    pl.add<double>((size_t)(ceil_div(n, kMeanChunk) * kKB));
    void *wsb = nullptr;
    MECDF_TRY(workspace_reserve(pl.used, &wsb));
    Arena a;
    a.base = (char *)wsb;
    double *terms = a.take<double>((size_t)n * kKB);
    double *mpart = a.take<double>((size_t)(ceil_div(n, kMeanChunk) * kKB));
    ProfScope prof("kde_direct", s);
    for (int b0 = 0; b0 < nh; b0 += kKB) {
        KBatchD kb{};
        kb.nb = nh - b0 < kKB ? nh - b0 : kKB;
        for (int b = 0; b < kKB; ++b) {
            const int bb = b0 + (b < kb.nb ? b : 0);
            double prod = 1.0;
            for (int k = 0; k < MECDF_MAX_DIM; ++k) {
                kb.ih[b][k] = k < d ? 1.0 / h[bb * d + k] : 0.0;
                if (k < d)
                    prod *= h[bb * d + k];
            }
            kb.norm_full[b] = 1.0 / ((double)(1 << d) * (double)n * prod);
            kb.norm_loo[b] = 1.0 / ((double)(1 << d) * (double)(n - 1) * prod);
        }
        hipLaunchKernelGGL((k_kdirect<T, CH, WT, OutT>), dim3((unsigned)ceil_div(n, 256)),
                           dim3(256), 0, s, x, d, n, w0in, w1in, kb, b0, mode, out,
                           score ? terms : nullptr);
        if (score)
            launch_mean(terms, n, kb.nb, b0, mpart, score, s);
        MECDF_LAUNCH_CHECK();
    }
    return MECDF_OK;
}

// best[s] = the index in [0, cnt[s]) of the largest of score[off[s] ..
// off[s] + cnt[s]), the lowest index among equal ones (NaN counts as the
// smallest), -1 for an empty list; one thread per list.
__global__ void k_seg_argmax(const double *__restrict__ score, const int64_t *__restrict__ off,
                             int nsets, int *__restrict__ best) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= nsets)
        return;
    const int64_t a = off[i], n = off[i + 1] - off[i];
    int bi = n > 0 ? 0 : -1;
    double bv = n > 0 ? score[a] : 0.0;
    for (int64_t j = 1; j < n; ++j) {
        const double v = score[a + j];
        if (v > bv || (bv != bv && v == v)) {
            bv = v;
            bi = (int)j;
        }
    }
    best[i] = bi;
}

// off: device, nsets + 1 list offsets
int launch_seg_argmax(const double *score, const int64_t *off, int nsets, int *best,
                      hipStream_t s) {
    hipLaunchKernelGGL(k_seg_argmax, dim3((unsigned)ceil_div(nsets, 256)), dim3(256), 0, s, score,
                       off, nsets, best);
    MECDF_LAUNCH_CHECK();
    return MECDF_OK;
}

int lcv_argmax(const double *score, const int *cnt, int nsets, int *best, hipStream_t s) {
    std::vector<int64_t> off((size_t)nsets + 1, 0);
    for (int i = 0; i < nsets; ++i)
        off[i + 1] = off[i] + cnt[i];
    void *wsb = nullptr;
    MECDF_TRY(workspace_reserve(sizeof(int64_t) * off.size(), &wsb));
    MECDF_TRY(upload_small(off.data(), sizeof(int64_t) * off.size(), wsb, s));
    hipLaunchKernelGGL(k_seg_argmax, dim3((unsigned)ceil_div(nsets, 256)), dim3(256), 0, s, score,
                       (const int64_t *)wsb, nsets, best);
    MECDF_LAUNCH_CHECK();
    return MECDF_OK;
}

int kde_run(int d, int64_t N, const double *x, const void *w, int nh, const double *h,
            void *f, double *score, int regression, int prec, hipStream_t s) {
    if (N > (int64_t(1) << 28) || (d == 3 && N > (int64_t(1) << 24)) ||
        (d >= 4 && N > kKdeDirectMaxN)) {
        set_error("kernel sums support N <= 2^28 (2^24 for d = 3, 2^20 for d >= 4)");
        return MECDF_EUNSUPPORTED;
    }
    if (d >= 4) {
        if (!regression) {
            if (prec == MECDF_F64)
                return kde_direct_t<double, 1, double, double>(d, N, x, (const double *)w,
                                                               nullptr, nh, h, (double *)f,
                                                               score, 0, s);
            return kde_direct_t<float, 1, float, float>(d, N, x, (const float *)w, nullptr, nh,
                                                        h, (float *)f, score, 0, s);
        }
        if (prec == MECDF_F64)
            return kde_direct_t<double, 2, double, double>(d, N, x, nullptr, (const double *)w,
                                                           nh, h, (double *)f, score, 1, s);
        return kde_direct_t<float, 2, float, float>(d, N, x, nullptr, (const float *)w, nh, h,
                                                    (float *)f, score, 1, s);
    }
    if (!regression) {
        if (prec == MECDF_F64)
            return kde_run_t<double, 1, double, double>(d, N, x, (const double *)w, nullptr, nh,
                                                        h, (double *)f, score, 0, s);
        return kde_run_t<float, 1, float, float>(d, N, x, (const float *)w, nullptr, nh, h,
                                                 (float *)f, score, 0, s);
    }
    if (prec == MECDF_F64)
        return kde_run_t<double, 2, double, double>(d, N, x, nullptr, (const double *)w, nh, h,
                                                    (double *)f, score, 1, s);
    return kde_run_t<float, 2, float, float>(d, N, x, nullptr, (const float *)w, nh, h,
                                             (float *)f, score, 1, s);
}

}  // namespace mecdf
