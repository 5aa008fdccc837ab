// Kernel path: Laplacian kernel density estimation and Nadaraya-Watson
// regression at the sample points, with leave-one-out CV scores (Section 3.1
// and Appendix D of Langrene & Warin, arXiv 2005.03246).
//
// eq. (Laplacian_decomposition_nD) writes the kernel sum at z as 2^d
// generalized ECDFs, one per sign orthant delta, with weights
// w_i exp(sum_k delta_k x_{k,i} / h_k) and a factor exp(-sum_k delta_k z_k / h_k).
// Appendix D evaluates all orthants in one divide-and-conquer over the points.
// The GPU version for d = 2 keeps that structure:
//
//   * points sorted by x1 once; blocks of kKT = 64 consecutive points (one
//     wavefront) are sorted by x2 in registers; pairs inside a block are
//     summed directly;
//   * merge levels h = 64, 128, ...: sorted blocks A (left in x1) and B are
//     merged by x2.  For a pair (i in A, j in B), x1_i <= c <= x1_j with c the
//     first x1 of B, so the x1 factor splits as exp(-(c - x1_i)/h1) *
//     exp(-(x1_j - c)/h1), both <= 1.  Along the merged x2 order, the x2 factor
//     is a product of the decays exp(-(x2_p - x2_{p-1})/h2) between
//     neighbours.  A forward scan (orthants with delta_2 = +1) and a backward
//     scan (delta_2 = -1) of these decayed sums, per side, give every item the
//     kernel sum over the other side: B items collect the delta_1 = +1
//     orthants from A, A items the delta_1 = -1 orthants from B.  Every factor
//     is at most 1, so the exponential weights of the decomposition never
//     overflow (their orthant shifts are the local split points), and each
//     unordered pair is counted once, at the level where it splits;
//   * the merge structure does not depend on h: it is built once per call and
//     stored; each batch of bandwidths only runs the scans, adding the level
//     contributions into an accumulator kept in the level's order and moved
//     down level by level through the stored merge maps (monotone streams).
//
// d = 1 is the same scan over the sorted sample (the two-sided recursion of
// the 1-D decomposition).  d = 3 is evaluated by an exact tiled pair sum.
// The sums exclude the point itself (leave-one-out); the full estimate adds
// w_j K(0).
#include "common.hpp"
#include "radix.hpp"

namespace mecdf {

constexpr int kKB = 4;     // bandwidths per batch
constexpr int kKT = 64;    // bottom block: one wavefront
constexpr int kKItems = 4;
constexpr int kKTile = 256 * kKItems;

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
    double ih1[kKB];  // 1/h of the merge-scale coordinate (x1)
    double ih2[kKB];  // 1/h of the scanned coordinate (x2)
    double norm_full[kKB];
    double norm_loo[kKB];
    int nb;           // bandwidths used in this batch (<= kKB)
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
                                                  const WT *__restrict__ w1in,
                                                  double *__restrict__ x1, double *__restrict__ x2,
                                                  double *__restrict__ w0, double *__restrict__ w1,
                                                  uint32_t *__restrict__ id) {
    int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= n)
        return;
    uint32_t i = idx[p];
    if (d == 1) {
        x1[p] = 0.0;
        x2[p] = x[i];
    } else {
        x1[p] = x[i];
        x2[p] = x[n + i];
    }
    w0[p] = w0in ? (double)w0in[i] : 1.0;
    w1[p] = w1in ? (double)w1in[i] : 0.0;
    id[p] = i;
}

// One wavefront per block of 64 points (x1 order): bitonic sort by x2 in
// registers.  Writes the block in x2 order and map0[p] = new position.
__global__ __launch_bounds__(256) void k_kblocksort(const double *__restrict__ x1s,
                                                    const double *__restrict__ x2s,
                                                    const double *__restrict__ w0s,
                                                    const double *__restrict__ w1s, int64_t n,
                                                    double *__restrict__ x1, double *__restrict__ x2,
                                                    double *__restrict__ w0, double *__restrict__ w1,
                                                    uint32_t *__restrict__ map0) {
    const int lane = threadIdx.x & 63;
    const int64_t blk = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int64_t p = blk * 64 + lane;
    if (blk * 64 >= n)
        return;
    bool v = p < n;
    uint64_t key = v ? order_key_kde(x2s[p]) : ~0ull;
    int src = lane;
#pragma unroll
    for (int k = 2; k <= 64; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            uint64_t ok = shfl_xor(key, j);
            int os = __shfl_xor(src, j, 64);
            bool up = (lane & k) == 0;
            bool lower = (lane & j) == 0;
            bool less = (ok < key) || (ok == key && os < src);
            bool greater = (ok > key) || (ok == key && os > src);
            bool take = (lower == up) ? less : greater;
            if (take) {
                key = ok;
                src = os;
            }
        }
    }
    // lane r now holds the item of rank r; it came from lane src
    int64_t q = blk * 64 + src;
    int64_t dst = blk * 64 + lane;
    if (q < n) {
        x1[dst] = x1s[q];
        x2[dst] = x2s[q];
        w0[dst] = w0s[q];
        w1[dst] = w1s[q];
        map0[q] = (uint32_t)dst;
    }
}

// Merge of aligned x2-sorted blocks of size h (A then B) into 2h, one thread
// per item; side = 0 for A, 1 for B.
__global__ __launch_bounds__(256) void k_kmerge(const double *__restrict__ x1i,
                                                const double *__restrict__ x2i,
                                                const double *__restrict__ w0i,
                                                const double *__restrict__ w1i, int64_t n,
                                                int64_t h, double *__restrict__ x1o,
                                                double *__restrict__ x2o, double *__restrict__ w0o,
                                                double *__restrict__ w1o, uint8_t *__restrict__ side,
                                                uint32_t *__restrict__ map) {
    int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= n)
        return;
    int64_t s = (p / (2 * h)) * (2 * h);
    int64_t ha = (n - s) < h ? (n - s) : h;
    int64_t hb = (n - s - ha) < h ? (n - s - ha) : h;
    double key = x2i[p];
    bool inA = (p - s) < ha;
    int64_t pos;
    if (inA) {
        const double *B = x2i + s + ha;
        int64_t lo = 0, hi = hb;
        while (lo < hi) {
            int64_t mid = (lo + hi) >> 1;
            if (B[mid] < key)
                lo = mid + 1;
            else
                hi = mid;
        }
        pos = p + lo;
    } else {
        const double *A = x2i + s;
        int64_t lo = 0, hi = ha;
        while (lo < hi) {
            int64_t mid = (lo + hi) >> 1;
            if (A[mid] <= key)
                lo = mid + 1;
            else
                hi = mid;
        }
        pos = s + (p - s - ha) + lo;
    }
    x1o[pos] = x1i[p];
    x2o[pos] = key;
    w0o[pos] = w0i[p];
    w1o[pos] = w1i[p];
    side[pos] = inA ? 0 : 1;
    map[p] = (uint32_t)pos;
}

// ----------------------------------------------------------- scan kernels
// Per item p of a level (merged order, segments of 2h items):
//   alpha_p = exp(-(x2_p - x2_{p-1}) / h2)   (0 at a segment start)
//   beta_p  = exp(-(x2_{p+1} - x2_p) / h2)   (0 before a segment start)
//   f_p     = exp(-|x1_p - c| / h1)          (c = first x1 of the right half)
//   own_p   = f_p w_p on the item's side (sides: 0 = left half, 1 = right half)
// Forward state F_p = alpha_p F_{p-1} + own_p, backward B_p = beta_p B_{p+1} + own_p
// (one value per side and channel).  Item p receives
//   f_p * (alpha_p F_{p-1} + beta_p B_{p+1})   on the other side,
// which is its kernel sum over the other half (in the 1-D case, oneside = 1,
// there is one side and f = 1).  Both recurrences are affine scans,
// state -> m * state + l, evaluated as tile aggregates, tile carries and a
// final pass, with fixed-order tree scans inside each tile.
template <typename T, int CH> struct Aff {
    T m[kKB];
    T l[kKB][2][CH];
};

template <typename T, int CH>
__device__ __forceinline__ void aff_identity(Aff<T, CH> &a) {
#pragma unroll
    for (int b = 0; b < kKB; ++b) {
        a.m[b] = T(1);
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int c = 0; c < CH; ++c)
                a.l[b][s][c] = T(0);
    }
}

// first `x`, then `y`: state -> y.m (x.m state + x.l) + y.l
template <typename T, int CH>
__device__ __forceinline__ Aff<T, CH> aff_then(const Aff<T, CH> &x, const Aff<T, CH> &y) {
    Aff<T, CH> r;
#pragma unroll
    for (int b = 0; b < kKB; ++b) {
        r.m[b] = x.m[b] * y.m[b];
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int c = 0; c < CH; ++c)
                r.l[b][s][c] = y.m[b] * x.l[b][s][c] + y.l[b][s][c];
    }
    return r;
}

template <typename T, int CH> struct KTileAgg {
    Aff<T, CH> fwd;  // items in ascending order
    Aff<T, CH> bwd;  // items in descending order
};
template <typename T, int CH> struct KCarry {
    T F[kKB][2][CH];  // forward state after all earlier tiles
    T B[kKB][2][CH];  // backward state after all later tiles
};

template <typename T> struct KLevelArgs {
    const double *x1, *x2, *w0, *w1;
    const uint8_t *side;
    const double *x1s;  // x1-sorted sample (for the split points)
    int64_t n, h;       // blocks of h merged into segments of 2h
    int oneside;
};

template <typename T, int CH>
__device__ __forceinline__ void kitem(const KLevelArgs<T> &L, const KBatch &kb, int64_t p,
                                      T alpha[kKB], T beta[kKB], T f[kKB], int &sd,
                                      T wv[CH]) {
    const int64_t seg = 2 * L.h;
    const int64_t s = (p / seg) * seg;
    const bool start = (p == s);
    const bool last = (p + 1 >= L.n) || (p + 1 == s + seg);
    double x2 = L.x2[p];
    double x2p = start ? x2 : L.x2[p - 1];
    double x2n = last ? x2 : L.x2[p + 1];
    double c = (s + L.h < L.n) ? L.x1s[s + L.h] : L.x1s[L.n - 1];
    double dx1 = fabs(L.x1[p] - c);
    sd = L.oneside ? 0 : (int)L.side[p];
    wv[0] = (T)L.w0[p];
    if (CH > 1)
        wv[CH - 1] = (T)L.w1[p];
#pragma unroll
    for (int b = 0; b < kKB; ++b) {
        alpha[b] = start ? T(0) : kexp<T>((T)(-(x2 - x2p) * kb.ih2[b]));
        beta[b] = last ? T(0) : kexp<T>((T)(-(x2n - x2) * kb.ih2[b]));
        f[b] = L.oneside ? T(1) : kexp<T>((T)(-dx1 * kb.ih1[b]));
    }
}

// the thread's items as forward and backward affine maps
template <typename T, int CH>
__device__ __forceinline__ void thread_affs(const T alpha[kKItems][kKB],
                                            const T beta[kKItems][kKB],
                                            const T f[kKItems][kKB], const int sd[kKItems],
                                            const T wv[kKItems][CH], const bool val[kKItems],
                                            Aff<T, CH> &fw, Aff<T, CH> &bw) {
    aff_identity(fw);
    aff_identity(bw);
#pragma unroll
    for (int u = 0; u < kKItems; ++u) {
        if (!val[u])
            continue;
#pragma unroll
        for (int b = 0; b < kKB; ++b) {
            fw.m[b] *= alpha[u][b];
#pragma unroll
            for (int s = 0; s < 2; ++s)
#pragma unroll
                for (int c = 0; c < CH; ++c)
                    fw.l[b][s][c] *= alpha[u][b];
#pragma unroll
            for (int c = 0; c < CH; ++c)
                fw.l[b][sd[u]][c] += f[u][b] * wv[u][c];
        }
    }
#pragma unroll
    for (int u = kKItems - 1; u >= 0; --u) {
        if (!val[u])
            continue;
#pragma unroll
        for (int b = 0; b < kKB; ++b) {
            bw.m[b] *= beta[u][b];
#pragma unroll
            for (int s = 0; s < 2; ++s)
#pragma unroll
                for (int c = 0; c < CH; ++c)
                    bw.l[b][s][c] *= beta[u][b];
#pragma unroll
            for (int c = 0; c < CH; ++c)
                bw.l[b][sd[u]][c] += f[u][b] * wv[u][c];
        }
    }
}

template <typename T, int CH>
__device__ __forceinline__ void load_items(const KLevelArgs<T> &L, const KBatch &kb,
                                           int64_t base, T alpha[kKItems][kKB],
                                           T beta[kKItems][kKB], T f[kKItems][kKB],
                                           int sd[kKItems], T wv[kKItems][CH],
                                           bool val[kKItems]) {
#pragma unroll
    for (int u = 0; u < kKItems; ++u) {
        int64_t p = base + u;
        val[u] = p < L.n;
        if (val[u]) {
            kitem<T, CH>(L, kb, p, alpha[u], beta[u], f[u], sd[u], wv[u]);
        } else {
            sd[u] = 0;
#pragma unroll
            for (int b = 0; b < kKB; ++b)
                alpha[u][b] = beta[u][b] = f[u][b] = T(0);
#pragma unroll
            for (int c = 0; c < CH; ++c)
                wv[u][c] = T(0);
        }
    }
}

// Inclusive tree scan of the 256 thread maps in LDS: forward (dir = 0, thread
// t composes threads 0..t) or backward (dir = 1, threads 255..t).
template <typename T, int CH>
__device__ __forceinline__ Aff<T, CH> block_aff_scan(Aff<T, CH> v, Aff<T, CH> *buf, int dir) {
    const int t = threadIdx.x;
    buf[t] = v;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        Aff<T, CH> r = v;
        if (dir == 0 && t >= off)
            r = aff_then(buf[t - off], v);
        if (dir == 1 && t + off < 256)
            r = aff_then(buf[t + off], v);
        __syncthreads();
        v = r;
        buf[t] = v;
        __syncthreads();
    }
    return v;
}

template <typename T, int CH>
__global__ __launch_bounds__(256) void k_ktile_agg(KLevelArgs<T> L, KBatch kb,
                                                   KTileAgg<T, CH> *__restrict__ agg) {
    __shared__ Aff<T, CH> buf[256];
    const int64_t base = (int64_t)blockIdx.x * kKTile + (int64_t)threadIdx.x * kKItems;
    T alpha[kKItems][kKB], beta[kKItems][kKB], f[kKItems][kKB], wv[kKItems][CH];
    int sd[kKItems];
    bool val[kKItems];
    load_items<T, CH>(L, kb, base, alpha, beta, f, sd, wv, val);
    Aff<T, CH> fw, bw;
    thread_affs<T, CH>(alpha, beta, f, sd, wv, val, fw, bw);
    Aff<T, CH> fi = block_aff_scan<T, CH>(fw, buf, 0);
    if (threadIdx.x == 255)
        agg[blockIdx.x].fwd = fi;
    Aff<T, CH> bi = block_aff_scan<T, CH>(bw, buf, 1);
    if (threadIdx.x == 0)
        agg[blockIdx.x].bwd = bi;
}

// Tile carries: one block of kCarryT threads, each owning a contiguous chunk
// of tiles; tree scans over the chunk maps.
constexpr int kCarryT = 512;
template <typename T, int CH>
__global__ __launch_bounds__(kCarryT) void k_kcarry(const KTileAgg<T, CH> *__restrict__ agg,
                                                 int64_t nt, KCarry<T, CH> *__restrict__ car) {
    // the maps are per bandwidth; this kernel handles all kKB at once, so the
    // chunk maps are full Aff values
    __shared__ Aff<T, CH> buf[kCarryT];
    const int t = threadIdx.x;
    const int64_t ch = ceil_div_dev(nt, kCarryT);
    const int64_t t0 = (int64_t)t * ch;
    const int64_t t1 = t0 + ch < nt ? t0 + ch : nt;
    // forward
    Aff<T, CH> v;
    aff_identity(v);
    for (int64_t q = t0; q < t1; ++q)
        v = aff_then(v, agg[q].fwd);
    buf[t] = v;
    __syncthreads();
    for (int off = 1; off < kCarryT; off <<= 1) {
        Aff<T, CH> r = v;
        if (t >= off)
            r = aff_then(buf[t - off], v);
        __syncthreads();
        v = r;
        buf[t] = v;
        __syncthreads();
    }
    Aff<T, CH> ex;
    if (t == 0)
        aff_identity(ex);
    else
        ex = buf[t - 1];
    __syncthreads();
    for (int64_t q = t0; q < t1; ++q) {
#pragma unroll
        for (int b = 0; b < kKB; ++b)
#pragma unroll
            for (int s = 0; s < 2; ++s)
#pragma unroll
                for (int c = 0; c < CH; ++c)
                    car[q].F[b][s][c] = ex.l[b][s][c];
        ex = aff_then(ex, agg[q].fwd);
    }
    // backward (from the last tile)
    aff_identity(v);
    for (int64_t q = t1 - 1; q >= t0; --q)
        v = aff_then(v, agg[q].bwd);
    buf[t] = v;
    __syncthreads();
    for (int off = 1; off < kCarryT; off <<= 1) {
        Aff<T, CH> r = v;
        if (t + off < kCarryT)
            r = aff_then(buf[t + off], v);
        __syncthreads();
        v = r;
        buf[t] = v;
        __syncthreads();
    }
    if (t == kCarryT - 1)
        aff_identity(ex);
    else
        ex = buf[t + 1];
    for (int64_t q = t1 - 1; q >= t0; --q) {
#pragma unroll
        for (int b = 0; b < kKB; ++b)
#pragma unroll
            for (int s = 0; s < 2; ++s)
#pragma unroll
                for (int c = 0; c < CH; ++c)
                    car[q].B[b][s][c] = ex.l[b][s][c];
        ex = aff_then(ex, agg[q].bwd);
    }
}

template <typename T, int CH>
__global__ __launch_bounds__(256) void k_kapply(KLevelArgs<T> L, KBatch kb,
                                                const KCarry<T, CH> *__restrict__ car,
                                                double *__restrict__ acc) {
    __shared__ Aff<T, CH> buf[256];
    const int tid = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * kKTile + (int64_t)tid * kKItems;
    T alpha[kKItems][kKB], beta[kKItems][kKB], f[kKItems][kKB], wv[kKItems][CH];
    int sd[kKItems];
    bool val[kKItems];
    load_items<T, CH>(L, kb, base, alpha, beta, f, sd, wv, val);
    Aff<T, CH> fw, bw;
    thread_affs<T, CH>(alpha, beta, f, sd, wv, val, fw, bw);
    // forward state entering this thread
    Aff<T, CH> fi = block_aff_scan<T, CH>(fw, buf, 0);
    Aff<T, CH> fex;
    if (tid == 0)
        aff_identity(fex);
    else
        fex = buf[tid - 1];
    __syncthreads();
    Aff<T, CH> bi = block_aff_scan<T, CH>(bw, buf, 1);
    Aff<T, CH> bex;
    if (tid == 255)
        aff_identity(bex);
    else
        bex = buf[tid + 1];
    (void)fi;
    (void)bi;
    const KCarry<T, CH> &cr = car[blockIdx.x];
    T recv[kKItems][kKB][CH];
#pragma unroll
    for (int b = 0; b < kKB; ++b) {
        T st[2][CH];
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int c = 0; c < CH; ++c)
                st[s][c] = fex.m[b] * cr.F[b][s][c] + fex.l[b][s][c];
#pragma unroll
        for (int u = 0; u < kKItems; ++u) {
            const int o = L.oneside ? 0 : 1 - sd[u];
#pragma unroll
            for (int s = 0; s < 2; ++s)
#pragma unroll
                for (int c = 0; c < CH; ++c)
                    st[s][c] *= alpha[u][b];
#pragma unroll
            for (int c = 0; c < CH; ++c) {
                recv[u][b][c] = st[o][c];
                st[sd[u]][c] += f[u][b] * wv[u][c];
            }
        }
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int c = 0; c < CH; ++c)
                st[s][c] = bex.m[b] * cr.B[b][s][c] + bex.l[b][s][c];
#pragma unroll
        for (int u = kKItems - 1; u >= 0; --u) {
            const int o = L.oneside ? 0 : 1 - sd[u];
            if (!val[u])
                continue;
#pragma unroll
            for (int s = 0; s < 2; ++s)
#pragma unroll
                for (int c = 0; c < CH; ++c)
                    st[s][c] *= beta[u][b];
#pragma unroll
            for (int c = 0; c < CH; ++c) {
                recv[u][b][c] = f[u][b] * (recv[u][b][c] + st[o][c]);
                st[sd[u]][c] += f[u][b] * wv[u][c];
            }
        }
    }
#pragma unroll
    for (int u = 0; u < kKItems; ++u) {
        int64_t p = base + u;
        if (!val[u])
            continue;
        double *a = acc + p * (kKB * CH);
#pragma unroll
        for (int b = 0; b < kKB; ++b)
#pragma unroll
            for (int c = 0; c < CH; ++c)
                a[b * CH + c] += (double)recv[u][b][c];
    }
}

template <int CH>
__global__ __launch_bounds__(256) void k_kacc_down(const double *__restrict__ hi,
                                                   const uint32_t *__restrict__ map, int64_t n,
                                                   double *__restrict__ lo) {
    int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= n)
        return;
    const double *s = hi + (int64_t)map[p] * (kKB * CH);
    double *d = lo + p * (kKB * CH);
#pragma unroll
    for (int q = 0; q < kKB * CH; ++q)
        d[q] = s[q];
}

__global__ void k_kzero(double *a, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n)
        a[i] = 0.0;
}

// Bottom: gather the accumulated sums to x1 order, add the pairs inside each
// 64-block by direct evaluation, and produce the outputs and per-point score
// terms.  mode 0: KDE (channel 0 = w); mode 1: NW (channel 0 = 1, 1 = y).
template <typename T, int CH, typename OutT>
__global__ __launch_bounds__(256) void k_kbottom(const double *__restrict__ accS,
                                                 const uint32_t *__restrict__ map0,
                                                 const double *__restrict__ x1s,
                                                 const double *__restrict__ x2s,
                                                 const double *__restrict__ w0s,
                                                 const double *__restrict__ w1s,
                                                 const uint32_t *__restrict__ ids, int64_t n,
                                                 int d, int brute, KBatch kb, int b0,
                                                 int mode, OutT *__restrict__ out,
                                                 double *__restrict__ terms) {
    const int lane = threadIdx.x & 63;
    const int64_t blk = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int64_t p = blk * 64 + lane;
    if (blk * 64 >= n)
        return;
    const bool v = p < n;
    double sum[kKB][CH];
    double x1 = v ? x1s[p] : 0.0, x2 = v ? x2s[p] : 0.0;
    double w0 = v ? w0s[p] : 0.0, w1 = v ? w1s[p] : 0.0;
    if (v) {
        const double *a = accS + (int64_t)(map0 ? map0[p] : (uint32_t)p) * (kKB * CH);
#pragma unroll
        for (int b = 0; b < kKB; ++b)
#pragma unroll
            for (int c = 0; c < CH; ++c)
                sum[b][c] = a[b * CH + c];
    }
    if (brute) {
        // pairs inside the block: lane j broadcasts its point
        int64_t bstart = blk * 64;
        int cnt = (int)((n - bstart) < 64 ? (n - bstart) : 64);
        for (int j = 0; j < cnt; ++j) {
            double y1 = shfl(x1, j), y2 = shfl(x2, j);
            double u0 = shfl(w0, j), u1 = shfl(w1, j);
            if (!v || j == lane)
                continue;
            double e1 = fabs(x1 - y1), e2 = fabs(x2 - y2);
#pragma unroll
            for (int b = 0; b < kKB; ++b) {
                T kv = kexp<T>((T)(-(e1 * kb.ih1[b] + e2 * kb.ih2[b])));
                sum[b][0] += (double)((T)u0 * kv);
                if (CH > 1)
                    sum[b][CH - 1] += (double)((T)u1 * kv);
            }
        }
    }
    if (!v)
        return;
    const uint32_t id = ids[p];
    for (int b = 0; b < kb.nb; ++b) {
        double o, t;
        if (mode == 0) {
            o = (sum[b][0] + w0) * kb.norm_full[b];
            double floo = sum[b][0] * kb.norm_loo[b];
            t = log(floo);
        } else {
            double num = sum[b][CH - 1], den = sum[b][0];
            o = (num + w1) / (den + 1.0);
            double mloo = num / den;
            double e = w1 - mloo;
            t = e * e;
        }
        if (out)
            out[(int64_t)(b0 + b) * n + id] = (OutT)o;
        terms[(int64_t)b * n + p] = t;
    }
}

// Exact pair sum for any d <= 3 (used for d = 3): thread = query, data tiles
// staged in LDS.
template <typename T, int CH, typename OutT>
__global__ __launch_bounds__(256) void k_kbrute_all(const double *__restrict__ x, int64_t n,
                                                    int d, const double *__restrict__ w0g,
                                                    const double *__restrict__ w1g,
                                                    const double *__restrict__ ihk /*[kKB][3]*/,
                                                    KBatch kb, int b0, int mode,
                                                    OutT *__restrict__ out,
                                                    double *__restrict__ terms) {
    __shared__ double sx[3][256];
    __shared__ double sw0[256], sw1[256];
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const bool v = q < n;
    double xq[3] = {0.0, 0.0, 0.0};
    if (v)
        for (int k = 0; k < d; ++k)
            xq[k] = x[(int64_t)k * n + q];
    double ih[kKB][3];
    for (int b = 0; b < kKB; ++b)
        for (int k = 0; k < 3; ++k)
            ih[b][k] = ihk[b * 3 + k];
    double sum[kKB][CH];
    for (int b = 0; b < kKB; ++b)
        for (int c = 0; c < CH; ++c)
            sum[b][c] = 0.0;
    for (int64_t t0 = 0; t0 < n; t0 += 256) {
        __syncthreads();
        int64_t i = t0 + threadIdx.x;
        if (i < n) {
            for (int k = 0; k < d; ++k)
                sx[k][threadIdx.x] = x[(int64_t)k * n + i];
            sw0[threadIdx.x] = w0g ? w0g[i] : 1.0;
            sw1[threadIdx.x] = w1g ? w1g[i] : 0.0;
        }
        __syncthreads();
        int cnt = (int)((n - t0) < 256 ? (n - t0) : 256);
        for (int j = 0; j < cnt; ++j) {
            if (t0 + j == q)
                continue;
            double e[3];
            for (int k = 0; k < 3; ++k)
                e[k] = k < d ? fabs(xq[k] - sx[k][j]) : 0.0;
#pragma unroll
            for (int b = 0; b < kKB; ++b) {
                T kv = kexp<T>((T)(-(e[0] * ih[b][0] + e[1] * ih[b][1] + e[2] * ih[b][2])));
                sum[b][0] += (double)((T)sw0[j] * kv);
                if (CH > 1)
                    sum[b][CH - 1] += (double)((T)sw1[j] * kv);
            }
        }
    }
    if (!v)
        return;
    double w0 = w0g ? w0g[q] : 1.0, w1 = w1g ? w1g[q] : 0.0;
    for (int b = 0; b < kb.nb; ++b) {
        double o, t;
        if (mode == 0) {
            o = (sum[b][0] + w0) * kb.norm_full[b];
            t = log(sum[b][0] * kb.norm_loo[b]);
        } else {
            double num = sum[b][CH - 1], den = sum[b][0];
            o = (num + w1) / (den + 1.0);
            double e = w1 - num / den;
            t = e * e;
        }
        if (out)
            out[(int64_t)(b0 + b) * n + q] = (OutT)o;
        terms[(int64_t)b * n + q] = t;
    }
}

__global__ __launch_bounds__(256) void k_kto_f64(const float *__restrict__ in, int64_t n,
                                                 double *__restrict__ out) {
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n)
        out[i] = (double)in[i];
}

// deterministic mean of each row of terms[nb][n]: fixed chunks of kMeanChunk
// items summed by one block each (fixed tree), then the chunk sums of a row
// summed by one block (fixed tree)
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
template <typename T, int CH, typename WT, typename OutT>
static int kde_run_t(int d, int64_t n, const double *x, const WT *w0in, const WT *w1in,
                     int nh, const double *h, OutT *out, double *score, int mode,
                     hipStream_t s) {
    std::vector<int64_t> hs;  // merge levels: blocks of h merged into 2h
    if (d == 2)
        for (int64_t hh = kKT; hh < n; hh *= 2)
            hs.push_back(hh);
    const int L = (int)hs.size();
    const int64_t nt = ceil_div(n, kKTile);
    ArenaPlan pl;
    pl.add<uint64_t>((size_t)n);
    pl.add<uint64_t>((size_t)n);
    pl.add<uint64_t>((size_t)n);
    pl.add<uint32_t>((size_t)n);
    pl.add<uint32_t>((size_t)n);
    pl.add<uint32_t>((size_t)n);
    for (int q = 0; q < 5; ++q)
        pl.add<double>((size_t)n);  // x1s x2s w0s w1s + x (f64 copy)
    pl.add<uint32_t>((size_t)n);    // ids
    pl.add<uint32_t>((size_t)n);    // map0
    for (int q = 0; q <= L; ++q) {  // states S_64, S_128, ...
        for (int r = 0; r < 4; ++r)
            pl.add<double>((size_t)n);
        pl.add<uint8_t>((size_t)n);
        pl.add<uint32_t>((size_t)n);
    }
    pl.add<double>((size_t)n * kKB * CH);
    pl.add<double>((size_t)n * kKB * CH);
    pl.add<double>((size_t)n * kKB);
    pl.add<KTileAgg<T, CH>>((size_t)nt + 1);
    pl.add<KCarry<T, CH>>((size_t)nt + 1);
    pl.add<double>(3 * kKB);
    pl.add<double>((size_t)n);  // w0 / w1 as double (brute path)
    pl.add<double>((size_t)n);
    pl.add<double>((size_t)(ceil_div(n, kMeanChunk) * kKB));
    radix_plan(pl, n);
    void *wsb = nullptr;
    MECDF_TRY(workspace_reserve(pl.used, &wsb));
    Arena a;
    a.base = (char *)wsb;
    uint64_t *k0 = a.take<uint64_t>(n), *k1 = a.take<uint64_t>(n), *k2 = a.take<uint64_t>(n);
    uint32_t *i0 = a.take<uint32_t>(n), *i1 = a.take<uint32_t>(n), *i2 = a.take<uint32_t>(n);
    double *x1s = a.take<double>(n), *x2s = a.take<double>(n), *w0s = a.take<double>(n),
           *w1s = a.take<double>(n), *xspare = a.take<double>(n);
    (void)xspare;
    uint32_t *ids = a.take<uint32_t>(n);
    uint32_t *map0 = a.take<uint32_t>(n);
    struct St {
        double *x1, *x2, *w0, *w1;
        uint8_t *side;
        uint32_t *map;
    };
    std::vector<St> st(L + 1);
    for (int q = 0; q <= L; ++q) {
        st[q].x1 = a.take<double>(n);
        st[q].x2 = a.take<double>(n);
        st[q].w0 = a.take<double>(n);
        st[q].w1 = a.take<double>(n);
        st[q].side = a.take<uint8_t>(n);
        st[q].map = a.take<uint32_t>(n);
    }
    double *accA = a.take<double>((size_t)n * kKB * CH);
    double *accB = a.take<double>((size_t)n * kKB * CH);
    double *terms = a.take<double>((size_t)n * kKB);
    KTileAgg<T, CH> *agg = a.take<KTileAgg<T, CH>>((size_t)nt + 1);
    KCarry<T, CH> *car = a.take<KCarry<T, CH>>((size_t)nt + 1);
    double *ihk = a.take<double>(3 * kKB);
    double *w0d = a.take<double>(n), *w1d = a.take<double>(n);
    double *mpart = a.take<double>((size_t)(ceil_div(n, kMeanChunk) * kKB));
    RadixScratch rs = radix_take(a, n);
    const unsigned nb = (unsigned)ceil_div(n, 256);
    const unsigned nbw = (unsigned)ceil_div(ceil_div(n, 64), 4);

    if (d == 3) {
        // exact pair sums; weights as double
        const double *w0p = nullptr, *w1p = nullptr;
        if (w0in) {
            if constexpr (std::is_same<WT, float>::value)
                hipLaunchKernelGGL(k_kto_f64, dim3(nb), dim3(256), 0, s, (const float *)w0in, n, w0d);
            else
                MECDF_TRY_HIP(hipMemcpyAsync(w0d, w0in, n * 8, hipMemcpyDeviceToDevice, s));
            w0p = w0d;
        }
        if (w1in) {
            if constexpr (std::is_same<WT, float>::value)
                hipLaunchKernelGGL(k_kto_f64, dim3(nb), dim3(256), 0, s, (const float *)w1in, n, w1d);
            else
                MECDF_TRY_HIP(hipMemcpyAsync(w1d, w1in, n * 8, hipMemcpyDeviceToDevice, s));
            w1p = w1d;
        }
        for (int b0 = 0; b0 < nh; b0 += kKB) {
            KBatch kb{};
            kb.nb = nh - b0 < kKB ? nh - b0 : kKB;
            double ihv[3 * kKB];
            for (int b = 0; b < kKB; ++b) {
                int bb = b0 + (b < kb.nb ? b : 0);
                double prod = 1.0;
                for (int k = 0; k < 3; ++k) {
                    ihv[b * 3 + k] = k < d ? 1.0 / h[bb * d + k] : 0.0;
                    if (k < d)
                        prod *= h[bb * d + k];
                }
                kb.norm_full[b] = 1.0 / ((double)(1 << d) * (double)n * prod);
                kb.norm_loo[b] = 1.0 / ((double)(1 << d) * (double)(n - 1) * prod);
            }
            MECDF_TRY(upload_small(ihv, sizeof(ihv), ihk, s));
            {
                ProfScope prof("kde_pairs", s);
                hipLaunchKernelGGL((k_kbrute_all<T, CH, OutT>), dim3(nb), dim3(256), 0, s, x, n, d,
                                   w0p, w1p, ihk, kb, b0, mode, out, terms);
            }
            if (score)
                launch_mean(terms, n, kb.nb, b0, mpart, score, s);
            MECDF_LAUNCH_CHECK();
        }
        return MECDF_OK;
    }

    // ---- h-independent structure
    {
        ProfScope prof("kde_build", s);
        hipLaunchKernelGGL(k_kx_keys, dim3(nb), dim3(256), 0, s, x, n, k0, i0);
        int which = 0;
        MECDF_TRY((radix_sort_bits<uint64_t, uint32_t>(k0, i0, k1, i1, k2, i2, n, 0, 64, rs, s,
                                                       &which)));
        uint32_t *idx = which == 1 ? i1 : (which == 2 ? i2 : i0);
        hipLaunchKernelGGL((k_kgather0<WT>), dim3(nb), dim3(256), 0, s, idx, n, d, x, w0in, w1in,
                           x1s, x2s, w0s, w1s, ids);
        if (d == 2) {
            hipLaunchKernelGGL(k_kblocksort, dim3(nbw), dim3(256), 0, s, x1s, x2s, w0s, w1s, n,
                               st[0].x1, st[0].x2, st[0].w0, st[0].w1, map0);
            for (int q = 0; q < L; ++q)
                hipLaunchKernelGGL(k_kmerge, dim3(nb), dim3(256), 0, s, st[q].x1, st[q].x2,
                                   st[q].w0, st[q].w1, n, hs[q], st[q + 1].x1, st[q + 1].x2,
                                   st[q + 1].w0, st[q + 1].w1, st[q + 1].side, st[q].map);
        }
        MECDF_LAUNCH_CHECK();
    }

    for (int b0 = 0; b0 < nh; b0 += kKB) {
        KBatch kb{};
        kb.nb = nh - b0 < kKB ? nh - b0 : kKB;
        for (int b = 0; b < kKB; ++b) {
            int bb = b0 + (b < kb.nb ? b : 0);
            double h1 = h[bb * d + 0];
            double h2 = d == 2 ? h[bb * d + 1] : h1;
            double prod = d == 2 ? h1 * h2 : h1;
            kb.ih1[b] = 1.0 / h1;
            kb.ih2[b] = 1.0 / h2;
            kb.norm_full[b] = 1.0 / ((double)(1 << d) * (double)n * prod);
            kb.norm_loo[b] = 1.0 / ((double)(1 << d) * (double)(n - 1) * prod);
        }
        double *acc = accA, *accn = accB;
        const unsigned nba = (unsigned)ceil_div(n * kKB * CH, 256);
        hipLaunchKernelGGL(k_kzero, dim3(nba), dim3(256), 0, s, acc, n * kKB * CH);
        if (d == 1) {
            KLevelArgs<T> la{x1s, x2s, w0s, w1s, nullptr, x1s, n, (int64_t)1 << 40, 1};
            ProfScope prof("kde_scan", s);
            hipLaunchKernelGGL((k_ktile_agg<T, CH>), dim3((unsigned)nt), dim3(256), 0, s, la, kb, agg);
            hipLaunchKernelGGL((k_kcarry<T, CH>), dim3(1), dim3(kCarryT), 0, s, agg, nt, car);
            hipLaunchKernelGGL((k_kapply<T, CH>), dim3((unsigned)nt), dim3(256), 0, s, la, kb, car, acc);
        } else {
            for (int q = L - 1; q >= 0; --q) {
                KLevelArgs<T> la{st[q + 1].x1, st[q + 1].x2, st[q + 1].w0, st[q + 1].w1,
                                 st[q + 1].side, x1s, n, hs[q], 0};
                {
                    ProfScope prof("kde_scan", s);
                    hipLaunchKernelGGL((k_ktile_agg<T, CH>), dim3((unsigned)nt), dim3(256), 0, s,
                                       la, kb, agg);
                    hipLaunchKernelGGL((k_kcarry<T, CH>), dim3(1), dim3(kCarryT), 0, s, agg, nt, car);
                    hipLaunchKernelGGL((k_kapply<T, CH>), dim3((unsigned)nt), dim3(256), 0, s, la,
                                       kb, car, acc);
                }
                ProfScope prof2("kde_down", s);
                hipLaunchKernelGGL((k_kacc_down<CH>), dim3(nb), dim3(256), 0, s, acc, st[q].map, n,
                                   accn);
                std::swap(acc, accn);
            }
        }
        {
            ProfScope prof("kde_bottom", s);
            hipLaunchKernelGGL((k_kbottom<T, CH, OutT>), dim3(nbw), dim3(256), 0, s, acc,
                               d == 2 ? map0 : nullptr, x1s, x2s, w0s, w1s, ids, n, d,
                               d == 2 ? 1 : 0, kb, b0, mode, out, terms);
        }
        if (score)
            launch_mean(terms, n, kb.nb, b0, mpart, score, s);
        MECDF_LAUNCH_CHECK();
    }
    return MECDF_OK;
}

int kde_run(int d, int64_t N, const double *x, const void *w, int nh, const double *h,
            void *f, double *score, int regression, int prec, hipStream_t s) {
    if (N > (int64_t(1) << 30)) {
        set_error("kernel sums support N <= 2^30");
        return MECDF_EUNSUPPORTED;
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
