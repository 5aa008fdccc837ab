// Grid path: generalized ECDF / ESF at every node of a rectilinear grid
// (Section 2.1 of Langrene & Warin, arXiv 2005.03246).
//
// The paper bins the points into the local sums s of eq. (partial_sums)
// (Appendix A, by per-axis sorting or mesh division) and then runs the
// nested running sums of its lexicographic sweep, which amount to a d-fold
// prefix sum (eq. (ECDF_decomposition)).  On the GPU the same sums are formed
// as follows, deterministically (no floating-point atomics):
//
//   k_cellkey   per point, the cell index c_k = #{nodes of axis k < x_k} of
//               every axis (exact comparisons; a mesh-division guess checked
//               against the two neighbouring nodes, binary search otherwise),
//               packed into a 32-bit key whose low bd bits hold the last-axis
//               cell and whose upper bits identify the line (the cells of axes
//               0..d-2).  One radix tile per block, which also counts the
//               tile's digits for the first radix pass.
//   radix sort  stable LSD passes on the line bits: each line's points become
//               contiguous, in input order.
//   k_line_bounds  first sorted position of every line.
//   k_line_wave / k_line
//               one wavefront (many short lines) or one workgroup (few long
//               lines) per line: the line's points are binned into the
//               M_last+1 cells of the last axis, 64 at a time (lanes with
//               equal cells found by ballots; the lowest lane of a group adds
//               the group's values in lane order; chunks in input order),
//               followed by the inclusive prefix along the last axis (ECDF)
//               and the exclusive suffix (ESF), written as rows of the output.
//   k_axis_scan the remaining d-1 axes: inclusive prefix (ECDF) or inclusive
//               suffix over node rows (ESF) along axis k, in place, coalesced
//               across the contiguous trailing axes, both arrays in one
//               launch; the last pass divides by N.
//
// The ECDF at node j only needs cells c <= j on every axis, the ESF only cells
// c >= j+1 (eq. (ESF)); so the ECDF array holds the cells 0..M_k-1 of each
// axis and the ESF array the cells 1..M_k shifted down by one, and both
// arrays have exactly the output shape prod(M_k).
#include <algorithm>

#include "cells.hpp"
#include "common.hpp"
#include "radix.hpp"

namespace mecdf {

struct GridInfo {
    int d;
    int M[MECDF_MAX_DIM];
    int off[MECDF_MAX_DIM];
    uint32_t C[MECDF_MAX_DIM];
    int bd;      // bits holding the last-axis cell index (values 0..M_last)
    uint32_t L;  // number of lines; points with a NaN coordinate go to line L
    // Key layout of the line part.  packed != 0: each axis k < d-1 has its own
    // bit field [sh[k], sh[k] + nb[k]) (axis 0 has room for one extra value,
    // M_0 + 1, that marks a dropped point), so each radix pass sorts on one
    // axis's cells.  packed == 0: the mixed-radix line index sits above bd.
    int packed;
    int sh[MECDF_MAX_DIM];
    int nb[MECDF_MAX_DIM];
    // per axis: first and last node, and (M_k - 1) / (last - first), the
    // factor of the mesh-division guess
    double z0[MECDF_MAX_DIM];
    double zl[MECDF_MAX_DIM];
    double gs[MECDF_MAX_DIM];
};

// mixed-radix line index of a key (L for a dropped point)
__device__ __forceinline__ uint32_t key_line(uint32_t key, const GridInfo &g) {
    if (!g.packed)
        return key >> g.bd;
    uint32_t c0 = (key >> g.sh[0]) & ((1u << g.nb[0]) - 1u);
    if (c0 >= g.C[0])
        return g.L;
    uint32_t line = c0;
    for (int k = 1; k < g.d - 1; ++k)
        line = line * g.C[k] + ((key >> g.sh[k]) & ((1u << g.nb[k]) - 1u));
    return line;
}



// One radix tile (kRadixTile consecutive points) per block.  With hist != null
// the block also writes the tile's counts of the key digit [hshift, hshift +
// hbits), which are the counts the first radix pass needs.  The kernel also
// sets mark[0..nmark) to all ones and *zero1 to 0 (see below).
template <int D, bool kLds>
__global__ __launch_bounds__(256) void k_cellkey(const double *__restrict__ x,
                                                 int64_t n, GridInfo g,
                                                 const double *__restrict__ nodes_g,
                                                 int total_nodes,
                                                 uint32_t *__restrict__ keys,
                                                 uint32_t *__restrict__ hist,
                                                 int hshift, int hbits,
                                                 uint32_t *__restrict__ mark,
                                                 int64_t nmark,
                                                 uint32_t *__restrict__ zero1) {
    extern __shared__ double s_nodes[];
    // set-up for the line kernels, which run after the sort: line ranges
    // marked empty, heavy-line counter cleared
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < nmark;
         i += (int64_t)gridDim.x * 256)
        mark[i] = 0xffffffffu;
    if (blockIdx.x == 0 && threadIdx.x == 0)
        *zero1 = 0u;
    __shared__ uint32_t h[kRadixMaxDigits];
    const int R = 1 << hbits;
    if (hist)
        for (int i = threadIdx.x; i < R; i += 256)
            h[i] = 0;
    if constexpr (kLds) {
        for (int i = threadIdx.x; i < total_nodes; i += 256)
            s_nodes[i] = nodes_g[i];
    }
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kRadixTile;
    constexpr int kKeyPts = D <= 3 ? 8 : 4;  // points per thread per load group
    for (int grp = 0; grp < kRadixItems / kKeyPts; ++grp) {
        const int64_t b = base + (int64_t)grp * kKeyPts * 256 + threadIdx.x;
        double v[kKeyPts][D];
#pragma unroll
        for (int q = 0; q < kKeyPts; ++q) {
            int64_t i = b + (int64_t)q * 256;
#pragma unroll
            for (int k = 0; k < D; ++k)
                v[q][k] = i < n ? __builtin_nontemporal_load(x + (int64_t)k * n + i) : 0.0;
        }
#pragma unroll
        for (int q = 0; q < kKeyPts; ++q) {
            int64_t i = b + (int64_t)q * 256;
            if (i >= n)
                break;
            uint32_t line = 0, packed = 0, clast = 0;
            bool bad = false;
#pragma unroll
            for (int k = 0; k < D; ++k) {
                double vv = v[q][k];
                bad |= (vv != vv);
                uint32_t c;
                if constexpr (kLds)
                    c = cell_index(s_nodes + g.off[k], g.M[k], g.z0[k], g.zl[k], g.gs[k], vv);
                else
                    c = cell_index(nodes_g + g.off[k], g.M[k], g.z0[k], g.zl[k], g.gs[k], vv);
                if (k < D - 1) {
                    line = line * g.C[k] + c;
                    packed |= c << g.sh[k];
                } else {
                    clast = c;
                }
            }
            uint32_t key;
            if (g.packed)
                key = bad ? (g.C[0] << g.sh[0]) : (packed | clast);
            else
                key = bad ? (g.L << g.bd) : ((line << g.bd) | clast);
            keys[i] = key;
            if (hist)
                atomicAdd(&h[(key >> hshift) & (uint32_t)(R - 1)], 1u);
        }
    }
    if (hist) {
        __syncthreads();
        for (int i = threadIdx.x; i < R; i += 256)
            hist[(int64_t)blockIdx.x * R + i] = h[i];
    }
}

template <int D>
static void launch_cellkey(bool lds, int64_t nb, hipStream_t s, const double *x,
                           int64_t N, const GridInfo &g, const double *nodes,
                           int total_nodes, uint32_t *k0, uint32_t *hist,
                           int hshift, int hbits, uint32_t *mark, int64_t nmark,
                           uint32_t *zero1) {
    if (lds)
        hipLaunchKernelGGL((k_cellkey<D, true>), dim3((unsigned)nb), dim3(256),
                           sizeof(double) * total_nodes, s, x, N, g, nodes,
                           total_nodes, k0, hist, hshift, hbits, mark, nmark, zero1);
    else
        hipLaunchKernelGGL((k_cellkey<D, false>), dim3((unsigned)nb), dim3(256), 0,
                           s, x, N, g, nodes, total_nodes, k0, hist, hshift, hbits,
                           mark, nmark, zero1);
}

// Sorted range [lbnd[2l], lbnd[2l+1]) of every non-empty line l; the entries
// of empty lines keep the marker kNoLine (set before the sort).  A line starts
// where the bits above the last-axis cell change.  Four consecutive keys per
// thread (one 16-byte load; keys is 16-byte aligned) and the key before them.
constexpr uint32_t kNoLine = 0xffffffffu;

__global__ __launch_bounds__(256) void k_line_bounds(const uint32_t *__restrict__ keys,
                                                     int64_t n, GridInfo g,
                                                     uint32_t *__restrict__ lbnd) {
    const int64_t p0 = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 4;
    if (p0 >= n)
        return;
    uint32_t k[4];
    if (p0 + 4 <= n) {
        const uint4 q = *reinterpret_cast<const uint4 *>(keys + p0);
        k[0] = q.x;
        k[1] = q.y;
        k[2] = q.z;
        k[3] = q.w;
    } else {
#pragma unroll
        for (int u = 0; u < 4; ++u)
            k[u] = p0 + u < n ? keys[p0 + u] : 0u;
    }
    uint32_t pk = p0 > 0 ? keys[p0 - 1] : 0u;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int64_t p = p0 + u;
        if (p >= n)
            break;
        if (p == 0 || (k[u] >> g.bd) != (pk >> g.bd)) {
            lbnd[2 * (int64_t)key_line(k[u], g)] = (uint32_t)p;
            if (p > 0)
                lbnd[2 * (int64_t)key_line(pk, g) + 1] = (uint32_t)p;
        }
        if (p == n - 1)
            lbnd[2 * (int64_t)key_line(k[u], g) + 1] = (uint32_t)n;
        pk = k[u];
    }
}

__global__ void k_fill_u32(uint32_t *a, int64_t n, uint32_t v) {
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n)
        a[i] = v;
}

// accumulator of a bin: exact int64 counts, float64, or Kahan float32
template <typename T> struct BinAcc {
    T v;
    __device__ __forceinline__ void zero() { v = T(0); }
    __device__ __forceinline__ void add(T a) { v += a; }
    __device__ __forceinline__ T get() const { return v; }
};
template <> struct BinAcc<float> {
    KahanF k;
    __device__ __forceinline__ void zero() { k.s = 0.f; k.c = 0.f; }
    __device__ __forceinline__ void add(float a) { k.add(a); }
    __device__ __forceinline__ float get() const { return k.get(); }
};

template <typename T> __device__ __forceinline__ T finish(T v, int scale, double N) {
    if constexpr (std::is_same<T, int64_t>::value) {
        return v;
    } else {
        return scale ? (T)((double)v / N) : v;
    }
}


// Row offsets of a line in the ECDF array (cells <= M_k-1 on axes 0..d-2) and
// in the ESF array (cells >= 1, shifted down by one); doE / doS say whether the
// line has a row there.
__device__ __forceinline__ void line_rows(int64_t line, const GridInfo &g, int64_t &rowE,
                                          int64_t &rowS, bool &doE, bool &doS) {
    rowE = 0;
    rowS = 0;
    int64_t t = line;
    int64_t mul = 1;
    for (int k = g.d - 2; k >= 0; --k) {
        int64_t c = t % g.C[k];
        t /= g.C[k];
        doE = doE && (c <= g.M[k] - 1);
        doS = doS && (c >= 1);
        rowE += c * mul;
        rowS += (c - 1) * mul;
        mul *= g.M[k];
    }
}

// Bin one chunk of 64 sorted points (lane i holds point p0 + i when v) into
// bins.  The lanes holding the same cell are found through the LDS word
// mask[c]: cleared by its lanes, then each lane ORs in its own bit (the result
// does not depend on the order of the ORs).  A lane's rank among its peers
// (lower lanes first) orders the adds: in round r, the lanes of rank r add
// their values, one lane per cell, so every bin receives its points in lane
// order.
template <typename T, bool kPay>
__device__ __forceinline__ void bin_chunk(BinAcc<T> *bins, uint64_t *mask, bool v, uint32_t c,
                                          T val, uint64_t lt, int lane) {
    if (v)
        mask[c] = 0ull;
    wave_lds_fence();
    if (v)
        atomicOr(reinterpret_cast<unsigned long long *>(mask + c), 1ull << lane);
    wave_lds_fence();
    const uint64_t peers = v ? mask[c] : 0ull;
    const int rank = (int)__popcll(peers & lt);
    if constexpr (!kPay)
        val = T(1);
    if constexpr (std::is_same<T, float>::value) {
        // compensated bins: read-modify-write, one round after the other
        for (int r = 0; __ballot(v && rank >= r) != 0ull; ++r) {
            if (v && rank == r)
                bins[c].add(val);
            wave_lds_fence();
        }
    } else {
        // one lane per cell in each round, so the LDS atomic adds never
        // collide and each equals the plain add; they are issued round after
        // round without waiting for one another
        for (int r = 0; __ballot(v && rank >= r) != 0ull; ++r) {
            if (v && rank == r) {
                if constexpr (std::is_same<T, double>::value)
                    atomicAdd(&bins[c].v, val);
                else
                    atomicAdd(reinterpret_cast<unsigned long long *>(&bins[c].v),
                              (unsigned long long)val);
            }
        }
        wave_lds_fence();
    }
}

// Last-axis scans of one line's bins by one wavefront (each lane owns a
// contiguous run of cells): inclusive prefix into Pout (ECDF), exclusive
// suffix into Qout (ESF), cells 0..Ml-1.
template <typename T>
__device__ __forceinline__ void line_scans(const BinAcc<T> *bins, int Cl, bool doE, bool doS,
                                           T *Pout, T *Qout, int lane) {
    const int Ml = Cl - 1;
    const int ch = (Cl + 63) / 64;
    const int b0 = lane * ch < Cl ? lane * ch : Cl;
    const int b1 = b0 + ch < Cl ? b0 + ch : Cl;
    BinAcc<T> tot;
    tot.zero();
    for (int c = b0; c < b1; ++c)
        tot.add(bins[c].get());
    const T tv = tot.get();
    if (doE) {
        T inc = wave_inclusive_scan(tv);
        T ex = shfl_up(inc, 1);
        if (lane == 0)
            ex = T(0);
        BinAcc<T> run;
        run.zero();
        run.add(ex);
        for (int c = b0; c < b1; ++c) {
            run.add(bins[c].get());
            if (c < Ml)
                Pout[c] = run.get();
        }
    }
    if (doS) {
        T sinc = wave_inclusive_suffix(tv);
        T sex = shfl_down(sinc, 1);
        if (lane == 63)
            sex = T(0);
        BinAcc<T> run;
        run.zero();
        run.add(sex);
        for (int c = b1 - 1; c >= b0; --c) {
            if (c < Ml)
                Qout[c] = run.get();
            run.add(bins[c].get());
        }
    }
}

// Bin the chunks first, first + stride, ... (below e0) of 64 sorted points,
// in that order, kB chunks' loads in flight at a time.
template <typename T, typename P, int kB>
__device__ __forceinline__ void bin_chunks(BinAcc<T> *bins, uint64_t *mask,
                                           const uint32_t *__restrict__ keys,
                                           const P *__restrict__ pay, uint32_t first,
                                           uint32_t e0, uint32_t stride, int bd,
                                           uint64_t lt, int lane) {
    constexpr bool kPay = !std::is_same<P, NoPayload>::value;
    const uint32_t cmask = (1u << bd) - 1u;
    for (uint32_t b0 = first; b0 < e0; b0 += kB * stride) {
        uint32_t kk[kB];
        T vv[kB];
#pragma unroll
        for (int j = 0; j < kB; ++j) {
            const uint32_t p = b0 + j * stride + lane;
            kk[j] = 0u;
            vv[j] = T(0);
            if (p < e0) {
                kk[j] = keys[p];
                if constexpr (kPay)
                    vv[j] = (T)pay[p];
            }
        }
#pragma unroll
        for (int j = 0; j < kB; ++j) {
            const uint32_t c0 = b0 + j * stride;
            if (c0 < e0)  // uniform over the wave
                bin_chunk<T, kPay>(bins, mask, c0 + lane < e0, kk[j] & cmask, vv[j], lt, lane);
        }
    }
}

constexpr int kLineWaves = 4;         // waves per block of the wave kernel
constexpr int kLineBatch = 8;         // chunks loaded together
constexpr uint32_t kHeavyLine = 16384;  // longer lines go to the block kernel
constexpr int kHeavyWaves = 8;

// LDS of the block kernel with kW waves: the bins and the peer masks of every
// wave; after the bins are combined into the first set, the prefix and suffix
// rows reuse the second and third.
template <int kW> inline size_t line_lds_bytes(int Cl) { return (size_t)2 * kW * Cl * 8; }

// One workgroup of kW wavefronts per line: line blockIdx.x, or, when list is
// not null, the lines list[i] for i = blockIdx.x, blockIdx.x + gridDim.x, ...
// below *count.  Wave w bins the chunks w, w+kW, ... of 64 points into its own
// bins; the bin sets are then combined in wave order, so every sum is taken
// in an order fixed by the input order alone.
template <typename T, typename P, int kW>
__device__ void line_block(int64_t line, uint2 range, const uint32_t *__restrict__ keys,
                           const P *__restrict__ pay, const GridInfo &g, T *__restrict__ F,
                           T *__restrict__ Fbar, int scale, double N, char *s_raw) {
    const int tid = threadIdx.x;
    const int w = tid >> 6;
    const int lane = tid & 63;
    const int Cl = (int)g.C[g.d - 1];
    const int Ml = Cl - 1;

    int64_t rowE, rowS;
    bool doE = F != nullptr, doS = Fbar != nullptr;
    line_rows(line, g, rowE, rowS, doE, doS);
    if (!doE && !doS)
        return;  // uniform over the block

    BinAcc<T> *bins = reinterpret_cast<BinAcc<T> *>(s_raw);
    BinAcc<T> *mybins = bins + (size_t)w * Cl;
    uint64_t *mymask = reinterpret_cast<uint64_t *>(bins + (size_t)kW * Cl) + (size_t)w * Cl;
    T *Pout = reinterpret_cast<T *>(bins + Cl);
    T *Qout = reinterpret_cast<T *>(bins + 2 * (size_t)Cl);
    for (int c = lane; c < Cl; c += 64)
        mybins[c].zero();
    wave_lds_fence();

    uint32_t s0 = range.x, e0 = range.y;
    if (s0 == kNoLine)
        s0 = e0 = 0u;
    bin_chunks<T, P, kLineBatch>(mybins, mymask, keys, pay, s0 + (uint32_t)w * 64u, e0,
                                 64u * kW, g.bd, lanemask_lt(), lane);
    __syncthreads();
    // combine the wave bins in wave order into bins[0]
    for (int c = tid; c < Cl; c += kW * 64) {
        BinAcc<T> t;
        t.zero();
        for (int q = 0; q < kW; ++q)
            t.add(bins[(size_t)q * Cl + c].get());
        bins[c] = t;
    }
    __syncthreads();
    if (w == 0)
        line_scans<T>(bins, Cl, doE, doS, Pout, Qout, lane);
    __syncthreads();
    if (doE) {
        T *dst = F + rowE * Ml;
        for (int j = tid; j < Ml; j += kW * 64)
            dst[j] = finish(Pout[j], scale, N);
    }
    if (doS) {
        T *dst = Fbar + rowS * Ml;
        for (int j = tid; j < Ml; j += kW * 64)
            dst[j] = finish(Qout[j], scale, N);
    }
}

template <typename T, typename P, int kW>
__global__ __launch_bounds__(kW * 64) void k_line(const uint32_t *__restrict__ keys,
                                                  const P *__restrict__ pay,
                                                  const uint32_t *__restrict__ lbnd,
                                                  const uint32_t *__restrict__ list,
                                                  const uint32_t *__restrict__ count,
                                                  GridInfo g, T *__restrict__ F,
                                                  T *__restrict__ Fbar, int scale,
                                                  double N) {
    extern __shared__ __attribute__((aligned(16))) char s_raw[];
    const uint2 *rng = reinterpret_cast<const uint2 *>(lbnd);
    if (!list) {
        line_block<T, P, kW>(blockIdx.x, rng[blockIdx.x], keys, pay, g, F, Fbar, scale, N,
                             s_raw);
        return;
    }
    // the next line and its range are loaded one line ahead
    const uint32_t n = *count;
    uint32_t i = blockIdx.x;
    uint32_t nl = i < n ? list[i] : 0u;
    uint2 nr = i < n ? rng[nl] : make_uint2(0u, 0u);
    for (; i < n; i += gridDim.x) {
        const uint32_t cl = nl;
        const uint2 cr = nr;
        if (i + gridDim.x < n) {
            nl = list[i + gridDim.x];
            nr = rng[nl];
        }
        __syncthreads();  // the previous line's LDS reads are done
        line_block<T, P, kW>(cl, cr, keys, pay, g, F, Fbar, scale, N, s_raw);
    }
}

// Variant for many short lines: one wavefront per line, the waves of the grid
// taking lines in turn (wave i of the grid: lines i, i + total waves, ...), no
// block barriers.  Chunks are binned as in k_line, in input order.  Lines
// longer than kHeavyLine points are appended to list[] (in any order) for
// k_line.  Per wave, LDS holds the bins (overwritten by the prefix row) and
// the peer masks (overwritten by the suffix row).  Empty lines only write
// their rows of zeros.
constexpr int kWaveLineMaxCells = 1024;
template <typename T> inline size_t line_wave_lds_bytes(int Cl) {
    return (size_t)kLineWaves * ((size_t)Cl * sizeof(BinAcc<T>) + (size_t)Cl * 8);
}

template <typename T, typename P>
__global__ __launch_bounds__(256) void k_line_wave(const uint32_t *__restrict__ keys,
                                                   const P *__restrict__ pay,
                                                   const uint32_t *__restrict__ lbnd,
                                                   uint32_t *__restrict__ list,
                                                   uint32_t *__restrict__ count,
                                                   GridInfo g, T *__restrict__ F,
                                                   T *__restrict__ Fbar, int scale,
                                                   double N) {
    extern __shared__ __attribute__((aligned(16))) char s_raw[];
    const int w = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int Cl = (int)g.C[g.d - 1];
    const int Ml = Cl - 1;
    char *wb = s_raw + (size_t)w * ((size_t)Cl * sizeof(BinAcc<T>) + (size_t)Cl * 8);
    BinAcc<T> *bins = reinterpret_cast<BinAcc<T> *>(wb);
    uint64_t *mask = reinterpret_cast<uint64_t *>(wb + (size_t)Cl * sizeof(BinAcc<T>));
    T *Qout = reinterpret_cast<T *>(mask);
    const uint64_t lt = lanemask_lt();
    const int64_t nwaves = (int64_t)gridDim.x * kLineWaves;

    // the next line's range is loaded one line ahead
    int64_t line = (int64_t)blockIdx.x * kLineWaves + w;
    uint2 nb = line < (int64_t)g.L ? reinterpret_cast<const uint2 *>(lbnd)[line]
                                   : make_uint2(0u, 0u);
    for (; line < (int64_t)g.L; line += nwaves) {
        const uint2 cb = nb;
        if (line + nwaves < (int64_t)g.L)
            nb = reinterpret_cast<const uint2 *>(lbnd)[line + nwaves];
        int64_t rowE, rowS;
        bool doE = F != nullptr, doS = Fbar != nullptr;
        line_rows(line, g, rowE, rowS, doE, doS);
        if (!doE && !doS)
            continue;  // uniform over the wave
        uint32_t s0 = cb.x, e0 = cb.y;
        if (s0 == kNoLine)
            s0 = e0 = 0u;
        if (e0 - s0 > kHeavyLine) {
            if (lane == 0)
                list[atomicAdd(count, 1u)] = (uint32_t)line;
            continue;  // uniform over the wave
        }
        if (s0 == e0) {
            if (doE)
                for (int j = lane; j < Ml; j += 64)
                    F[rowE * Ml + j] = T(0);
            if (doS)
                for (int j = lane; j < Ml; j += 64)
                    Fbar[rowS * Ml + j] = T(0);
            continue;
        }
        for (int c = lane; c < Cl; c += 64)
            bins[c].zero();
        wave_lds_fence();
        bin_chunks<T, P, kLineBatch>(bins, mask, keys, pay, s0, e0, 64u, g.bd, lt, lane);

        // last-axis scans: suffix row into Qout, then the prefix row in place
        // of the bins (each lane reads and writes only its own cells)
        const int ch = (Cl + 63) / 64;
        const int b0 = lane * ch < Cl ? lane * ch : Cl;
        const int b1 = b0 + ch < Cl ? b0 + ch : Cl;
        BinAcc<T> tot;
        tot.zero();
        for (int c = b0; c < b1; ++c)
            tot.add(bins[c].get());
        const T tv = tot.get();
        if (doS) {
            T sinc = wave_inclusive_suffix(tv);
            T sex = shfl_down(sinc, 1);
            if (lane == 63)
                sex = T(0);
            BinAcc<T> run;
            run.zero();
            run.add(sex);
            for (int c = b1 - 1; c >= b0; --c) {
                if (c < Ml)
                    Qout[c] = run.get();
                run.add(bins[c].get());
            }
        }
        // the prefix value of cell c goes to the first bytes of bins[c]
        constexpr int kPs = (int)(sizeof(BinAcc<T>) / sizeof(T));
        T *Pout = reinterpret_cast<T *>(bins);
        if (doE) {
            T inc = wave_inclusive_scan(tv);
            T ex = shfl_up(inc, 1);
            if (lane == 0)
                ex = T(0);
            BinAcc<T> run;
            run.zero();
            run.add(ex);
            for (int c = b0; c < b1; ++c) {
                run.add(bins[c].get());
                if (c < Ml)
                    Pout[c * kPs] = run.get();  // bins[c] was read just above
            }
        }
        wave_lds_fence();
        if (doE) {
            T *dst = F + rowE * Ml;
            for (int j = lane; j < Ml; j += 64)
                dst[j] = finish(Pout[j * kPs], scale, N);
        }
        if (doS) {
            T *dst = Fbar + rowS * Ml;
            for (int j = lane; j < Ml; j += 64)
                dst[j] = finish(Qout[j], scale, N);
        }
        wave_lds_fence();  // reads of this line's rows precede the next zeroing
    }
}

// In-place inclusive prefix along one axis of an array viewed as
// [outer][Mk][inner]; one thread per (outer, inner) column.  blockIdx.y = 0
// scans A (suffix scan if sufA != 0), blockIdx.y = 1 scans B as a suffix
// scan, so the ECDF and ESF arrays share one launch.
template <typename T>
__global__ __launch_bounds__(256) void k_axis_scan(T *__restrict__ A, T *__restrict__ B,
                                                   int64_t outer, int64_t Mk,
                                                   int64_t inner, int sufA, int scale,
                                                   double N) {
    // consecutive column blocks on one XCD (the rows of neighbouring blocks
    // share a line at each end)
    int64_t t = xcd_tile(blockIdx.x, gridDim.x) * 256 + threadIdx.x;
    if (t >= outer * inner)
        return;
    T *arr = blockIdx.y ? B : A;
    const int suffix = blockIdx.y ? 1 : sufA;
    int64_t o = t / inner;
    int64_t i = t - o * inner;
    T *col = arr + o * Mk * inner + i;
    BinAcc<T> run;
    run.zero();
    constexpr int U = 8;  // rows in flight per thread (8: 1 % faster than 16, 24 slower)
    int64_t j = 0;
    for (; j + U <= Mk; j += U) {
        T v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            int64_t jj = suffix ? (Mk - 1 - (j + u)) : (j + u);
            v[u] = col[jj * inner];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            int64_t jj = suffix ? (Mk - 1 - (j + u)) : (j + u);
            run.add(v[u]);
            col[jj * inner] = finish(run.get(), scale, N);
        }
    }
    for (; j < Mk; ++j) {
        int64_t jj = suffix ? (Mk - 1 - j) : j;
        run.add(col[jj * inner]);
        col[jj * inner] = finish(run.get(), scale, N);
    }
}

template <typename T, typename P>
static int grid_run_t(int d, int64_t N, const double *x, const P *y,
                      const int64_t *M, const double *z, T *F, T *Fbar,
                      hipStream_t s) {
    GridInfo g{};
    g.d = d;
    int total_nodes = 0;
    for (int k = 0; k < d; ++k) {
        g.M[k] = (int)M[k];
        g.off[k] = total_nodes;
        g.C[k] = (uint32_t)(M[k] + 1);
        g.z0[k] = z[total_nodes];
        g.zl[k] = z[total_nodes + M[k] - 1];
        g.gs[k] = g.zl[k] > g.z0[k] ? (double)(M[k] - 1) / (g.zl[k] - g.z0[k]) : 0.0;
        total_nodes += (int)M[k];
    }
    uint64_t L = 1;
    for (int k = 0; k < d - 1; ++k)
        L *= g.C[k];
    g.L = (uint32_t)L;
    g.bd = bits_for((uint64_t)M[d - 1]);
    const int lb = bits_for(L);  // line values 0..L (L = dropped)
    {
        int tot = g.bd;
        for (int k = d - 2; k >= 0; --k) {
            g.nb[k] = bits_for((uint64_t)M[k] + (k == 0 ? 1 : 0));
            g.sh[k] = tot;
            tot += g.nb[k];
        }
        g.packed = (d >= 2 && tot <= 32) ? 1 : 0;
    }
    const int Cl = (int)g.C[d - 1];
    const int Ml = Cl - 1;

    int64_t total_out = 1;
    for (int k = 0; k < d; ++k)
        total_out *= M[k];

    ArenaPlan pl;
    pl.add<double>((size_t)total_nodes);
    pl.add<uint32_t>((size_t)N);  // keys in input order
    pl.add<uint32_t>((size_t)N);
    pl.add<uint32_t>((size_t)N);
    if constexpr (!std::is_same<P, NoPayload>::value) {
        pl.add<P>((size_t)N);
        pl.add<P>((size_t)N);
    }
    pl.add<uint32_t>(2 * ((size_t)L + 1));  // line ranges (line L: dropped points)
    pl.add<uint32_t>((size_t)L + 1);        // heavy-line list and its counter
    radix_plan(pl, N);
    void *wsb = nullptr;
    MECDF_TRY(workspace_reserve(pl.used, &wsb));
    Arena a;
    a.base = (char *)wsb;
    double *nodes = a.take<double>((size_t)total_nodes);
    uint32_t *k0 = a.take<uint32_t>((size_t)N);
    uint32_t *k1 = a.take<uint32_t>((size_t)N);
    uint32_t *k2 = a.take<uint32_t>((size_t)N);
    P *p1 = nullptr, *p2 = nullptr;
    if constexpr (!std::is_same<P, NoPayload>::value) {
        p1 = a.take<P>((size_t)N);
        p2 = a.take<P>((size_t)N);
    }
    uint32_t *lbnd = a.take<uint32_t>(2 * ((size_t)L + 1));
    uint32_t *hlist = a.take<uint32_t>((size_t)L + 1);
    uint32_t *hcount = hlist + L;
    RadixScratch rs = radix_take(a, N);

    MECDF_TRY(upload_small(z, sizeof(double) * total_nodes, nodes, s));

    const uint32_t *ks = k0;
    const P *ps = y;
    if (N > 0) {
        const int64_t ntiles = ceil_div(N, kRadixTile);
        bool lds = total_nodes <= 12288;
        // the first radix pass's digit, whose per-tile counts k_cellkey writes
        int hshift = -1, hbits = 0;
        if (g.packed) {
            hshift = g.sh[d - 2];
            hbits = g.nb[d - 2] < kRadixMaxBits ? g.nb[d - 2] : kRadixMaxBits;
        } else if (lb > 0) {
            hshift = g.bd;
            hbits = lb < kRadixMaxBits ? lb : kRadixMaxBits;
        }
        uint32_t *h0 = hshift >= 0 ? rs.hist : nullptr;
        {
            ProfScope prof1("grid_cellkey", s);
            switch (d) {
#define MECDF_CK(D) launch_cellkey<D>(lds, ntiles, s, x, N, g, nodes, total_nodes, k0, h0, \
                                      hshift < 0 ? 0 : hshift, hbits, lbnd,             \
                                      2 * ((int64_t)L + 1), hcount)
            case 1: MECDF_CK(1); break;
            case 2: MECDF_CK(2); break;
            case 3: MECDF_CK(3); break;
            case 4: MECDF_CK(4); break;
            case 5: MECDF_CK(5); break;
            default: MECDF_CK(6); break;
#undef MECDF_CK
            }
        }
        MECDF_LAUNCH_CHECK();
        int which = 0;
        if (g.packed) {
            // one pass (or more, for axes over 9 bits) per axis, last line axis first
            const uint32_t *ck = k0;
            const P *cp = y;
            int cur = 0;
            for (int k = d - 2; k >= 0; --k) {
                for (int b = g.sh[k]; b < g.sh[k] + g.nb[k]; b += kRadixMaxBits) {
                    int bits = g.sh[k] + g.nb[k] - b;
                    bits = bits < kRadixMaxBits ? bits : kRadixMaxBits;
                    uint32_t *nk = (cur == 1) ? k2 : k1;
                    P *np = (cur == 1) ? p2 : p1;
                    const bool first = (k == d - 2 && b == g.sh[k]);
                    MECDF_TRY((radix_pass<uint32_t, P>(ck, cp, nk, np, N, b, bits, rs, s,
                                                       first && h0 != nullptr)));
                    cur = (cur == 1) ? 2 : 1;
                    ck = nk;
                    cp = np;
                }
            }
            which = cur;
        } else {
            MECDF_TRY((radix_sort_bits<uint32_t, P>(k0, y, k1, p1, k2, p2, N, g.bd,
                                                    g.bd + lb, rs, s, &which,
                                                    h0 != nullptr)));
        }
        ks = which == 0 ? k0 : (which == 1 ? k1 : k2);
        ps = which == 0 ? y : (which == 1 ? p1 : p2);
        ProfScope prof2("grid_line_bounds", s);
        hipLaunchKernelGGL(k_line_bounds, dim3((unsigned)ceil_div(N, 1024)), dim3(256), 0, s,
                           ks, N, g, lbnd);
        MECDF_LAUNCH_CHECK();
    } else {
        hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)ceil_div(2 * (L + 1), 256)), dim3(256),
                           0, s, lbnd, 2 * ((int64_t)L + 1), kNoLine);
        hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(256), 0, s, hcount, (int64_t)1, 0u);
        MECDF_LAUNCH_CHECK();
    }

    // Lines: short ones one per wavefront; long ones (or all, when there are
    // few lines or the last axis is long) one per workgroup.
    const size_t wave_bytes = line_wave_lds_bytes<T>(Cl);
    const bool wave_path = L >= 1024 && Cl <= kWaveLineMaxCells && wave_bytes <= 64 * 1024;
    if (wave_path) {
        ProfScope prof3("grid_line", s);
        // one line per wavefront: the workgroup dispatcher then balances
        // lines of very different lengths, and more lines are in flight
        const int64_t nblk = std::min<int64_t>(ceil_div(L, kLineWaves), 1 << 20);
        hipLaunchKernelGGL((k_line_wave<T, P>), dim3((unsigned)nblk), dim3(256), wave_bytes, s,
                           ks, ps, lbnd, hlist, hcount, g, F, Fbar, d == 1 ? 1 : 0,
                           (double)N);
        MECDF_LAUNCH_CHECK();
    }
    {
        // at most N / (kHeavyLine + 1) lines are heavy; each block loops over
        // its share of them
        const int64_t nblk =
            wave_path ? std::min<int64_t>(std::min<int64_t>(L, N / (kHeavyLine + 1) + 1), 2048)
                      : (int64_t)L;
        const uint32_t *lst = wave_path ? hlist : nullptr;
        ProfScope prof3("grid_line_block", s);
        size_t lb_bytes = line_lds_bytes<kHeavyWaves>(Cl);
        if (lb_bytes <= 64 * 1024) {
            hipLaunchKernelGGL((k_line<T, P, kHeavyWaves>), dim3((unsigned)nblk),
                               dim3(kHeavyWaves * 64), lb_bytes, s, ks, ps, lbnd, lst, hcount,
                               g, F, Fbar, d == 1 ? 1 : 0, (double)N);
        } else if (line_lds_bytes<4>(Cl) <= 160 * 1024) {
            lb_bytes = line_lds_bytes<4>(Cl);
            if (lb_bytes > 64 * 1024)
                MECDF_TRY_HIP(hipFuncSetAttribute((const void *)k_line<T, P, 4>,
                                                  hipFuncAttributeMaxDynamicSharedMemorySize,
                                                  (int)lb_bytes));
            hipLaunchKernelGGL((k_line<T, P, 4>), dim3((unsigned)nblk), dim3(256), lb_bytes,
                               s, ks, ps, lbnd, lst, hcount, g, F, Fbar, d == 1 ? 1 : 0,
                               (double)N);
        } else {
            // the longest last axes (up to 5119 cells): two wavefronts per line
            lb_bytes = line_lds_bytes<2>(Cl);
            if (lb_bytes > 160 * 1024) {
                set_error("last grid axis too large for the line kernel");
                return MECDF_EUNSUPPORTED;
            }
            MECDF_TRY_HIP(hipFuncSetAttribute((const void *)k_line<T, P, 2>,
                                              hipFuncAttributeMaxDynamicSharedMemorySize,
                                              (int)lb_bytes));
            hipLaunchKernelGGL((k_line<T, P, 2>), dim3((unsigned)nblk), dim3(128), lb_bytes,
                               s, ks, ps, lbnd, lst, hcount, g, F, Fbar, d == 1 ? 1 : 0,
                               (double)N);
        }
        MECDF_LAUNCH_CHECK();
    }

    // remaining axes, innermost first; the last pass divides by N
    for (int k = d - 2; k >= 0; --k) {
        int64_t outer = 1, inner = 1;
        for (int q = 0; q < k; ++q)
            outer *= M[q];
        for (int q = k + 1; q < d; ++q)
            inner *= M[q];
        int64_t nthreads = outer * inner;
        int64_t nbk = ceil_div(nthreads, 256);
        int scale = (k == 0) ? 1 : 0;
        ProfScope prof4("grid_axis_scan", s);
        if (F && Fbar)
            hipLaunchKernelGGL(k_axis_scan<T>, dim3((unsigned)nbk, 2), dim3(256), 0, s, F,
                               Fbar, outer, (int64_t)M[k], inner, 0, scale, (double)N);
        else if (F || Fbar)
            hipLaunchKernelGGL(k_axis_scan<T>, dim3((unsigned)nbk, 1), dim3(256), 0, s,
                               F ? F : Fbar, (T *)nullptr, outer, (int64_t)M[k], inner,
                               F ? 0 : 1, scale, (double)N);
        MECDF_LAUNCH_CHECK();
    }
    (void)total_out;
    (void)Ml;
    return MECDF_OK;
}

int grid_run(int d, int64_t N, const double *x, const void *y,
             const int64_t *M, const double *z, void *F, void *Fbar, int prec,
             hipStream_t s) {
    if (y == nullptr)
        return grid_run_t<int64_t, NoPayload>(d, N, x, nullptr, M, z,
                                              (int64_t *)F, (int64_t *)Fbar, s);
    if (prec == MECDF_F64)
        return grid_run_t<double, double>(d, N, x, (const double *)y, M, z,
                                          (double *)F, (double *)Fbar, s);
    return grid_run_t<float, float>(d, N, x, (const float *)y, M, z, (float *)F,
                                    (float *)Fbar, s);
}

}  // namespace mecdf
