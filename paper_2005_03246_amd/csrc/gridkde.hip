// Kernel sums at the nodes of a rectilinear grid: the "fast summation" kernel
// density estimate and Nadaraya-Watson regression of Section 3 (eq.
// (Laplacian_kde_nD) evaluated through the decomposition of eq.
// (Laplacian_decomposition_nD) on the grid of Section 2.1), and the same for
// the additive multivariate Matern-3/2 kernel of Appendix C (eq.
// (Matern32_average) through eq. (Matern32_decomposition_nD)), in Langrene &
// Warin, arXiv 2005.03246.
//
// Along one axis, a point x in cell c (z_{c-1} < x <= z_c) reaches the nodes
// j >= c through exp(-(z_j - x)/h) = exp(-(z_j - z_c)/h) exp(-(z_c - x)/h)
// and the nodes j <= c-1 through exp(-(x - z_{c-1})/h) = exp(-(z_{c-1} -
// z_j)/h) exp(-(x - z_{c-1})/h).  So each point puts, for every corner choice
// delta in {up, down}^d, the weight w prod_k (its factor to the cell's upper
// or lower node on axis k) into the bin of that corner node, and the 2^d bin
// arrays are scanned along every axis with the decays between neighbouring
// nodes: forward where delta_k = up, backward where down.  The estimate at a
// node is the sum of the 2^d scanned arrays.  Every factor is at most 1.
//
// The Matern-3/2 kernel (1 + sum_l |u_l|) exp(-sum_k |u_k|) needs, besides
// the plain sum S, one channel T_l per axis holding sum w |x_l - z_l|/h_l
// exp(-...): the paper's 2^d (d+1) channels.  Along the scan of axis l the
// pair (S, T_l) moves by the affine step T <- dec (T + g S), S <- dec S,
// with g the node gap over h (the distance of every point already summed
// grows by g), so all terms stay positive; along the other axes T_l scans
// like S.
//
// Operators along different axes commute, so after the scan along axis k the
// two arrays of each corner pair that differ only on axis k take the same
// operators from then on: they are added as the scan writes them, and the
// scan of axis k + 1 works on half as many arrays.  The Matern channels of
// the axes already scanned are added the same way into one channel R.
//
//   k_gk_keys      the cell of every point (exact comparisons with the
//                  nodes), one linear key per cell; points with a NaN
//                  coordinate get a key after every cell
//   radix sort     stable: each cell's points are contiguous, in input order
//   k_gk_gather    coordinates and weights in that order, once per call
//   k_gk_starts    the first sorted position of every cell
//   k_gk_bins      one thread per cell (and corner group) adds its points'
//                  corner weights in input order (float64, Neumaier), for up
//                  to four bandwidths of the group at once, and writes every
//                  bin of its corners; each bin of each corner array belongs
//                  to exactly one cell
//   k_gs_agg       per axis: decayed sums over chunks of kGkL nodes of every
//   k_gs_carry     line (both directions), the values entering each chunk
//   k_gs_apply     from those, and the scans of the chunks from their
//                  entering values, corner pairs added as they are written
//   k_gs_rows      the contiguous axis when its lines are at most 1024 nodes:
//   (_mat)         one wavefront per line scans it in blocks of 64 nodes
//                  (steps composed across the lanes), both directions, in
//                  one pass
//   k_gk_combine   times the normalisation (density) or as a ratio
//                  (regression)
#include <vector>

#include "cells.hpp"
#include "common.hpp"
#include "radix.hpp"

namespace mecdf {

constexpr int kGkL = 16;  // nodes per scan chunk

struct GkGrid {
    int d;
    int64_t M[MECDF_MAX_DIM];      // nodes per axis
    int64_t off[MECDF_MAX_DIM];    // first node of each axis in the node array
    int64_t C[MECDF_MAX_DIM];      // cells per axis (M + 1)
    int64_t cst[MECDF_MAX_DIM];    // cell-key strides (C order)
    int64_t nst[MECDF_MAX_DIM];    // node-array strides (C order)
    int64_t nodes;                 // prod M
    int64_t cells;                 // prod C
    double z0[MECDF_MAX_DIM];      // first and last node of each axis and the
    double zl[MECDF_MAX_DIM];      // mesh-division scale (M - 1) / (zl - z0)
    double gs[MECDF_MAX_DIM];
};

struct GkH {
    double ih[MECDF_MAX_DIM];  // 1/h per axis
};

// Bandwidths handled by one launch (blockIdx.y picks one), each with its own
// arrays at a fixed stride.
constexpr int kGkGroup = 4;
struct GkHs {
    GkH h[kGkGroup];
};

constexpr int kGkLdsNodes = 4096;  // node tables up to this size searched in LDS

// cell c = #{nodes < x} on each axis (a mesh-division guess checked exactly
// against the nodes), key = C-order index of the cell vector.  One radix
// tile of points per workgroup, which also counts the tile's keys by the
// first radix digit (the low hbits bits): the counts the sort's first pass
// needs.
__global__ __launch_bounds__(256) void k_gk_keys(GkGrid g, const double *__restrict__ zn,
                                                 int64_t total, const double *__restrict__ x,
                                                 int64_t n, uint32_t dropped,
                                                 uint32_t *__restrict__ key,
                                                 uint32_t *__restrict__ idx,
                                                 uint32_t *__restrict__ hist, int hbits) {
    __shared__ double sn[kGkLdsNodes];
    __shared__ uint32_t h[kRadixMaxDigits];
    const bool lds = total <= kGkLdsNodes;
    const int R = 1 << hbits;
    for (int t = threadIdx.x; t < R; t += 256)
        h[t] = 0u;
    if (lds)
        for (int64_t t = threadIdx.x; t < total; t += 256)
            sn[t] = zn[t];
    __syncthreads();
    const double *zb = lds ? sn : zn;
    const int64_t base = (int64_t)blockIdx.x * kRadixTile;
    for (int q = 0; q < kRadixItems; ++q) {
        const int64_t i = base + (int64_t)q * 256 + threadIdx.x;
        if (i >= n)
            break;
        int64_t k = 0;
        bool nan = false;
        for (int a = 0; a < g.d; ++a) {
            const double v = x[(int64_t)a * n + i];
            nan = nan || v != v;
            k += (int64_t)cell_index(zb + g.off[a], (int)g.M[a], g.z0[a], g.zl[a], g.gs[a], v) *
                 g.cst[a];
        }
        const uint32_t kk = nan ? dropped : (uint32_t)k;
        key[i] = kk;
        idx[i] = (uint32_t)i;
        atomicAdd(&h[kk & (uint32_t)(R - 1)], 1u);
    }
    __syncthreads();
    for (int t = threadIdx.x; t < R; t += 256)
        hist[(int64_t)blockIdx.x * R + t] = h[t];
}

// coordinates and weights in sorted order
template <typename WT>
__global__ __launch_bounds__(256) void k_gk_gather(const uint32_t *__restrict__ idx, int64_t n,
                                                   int d, const double *__restrict__ x,
                                                   const WT *__restrict__ w,
                                                   double *__restrict__ xs,
                                                   double *__restrict__ ws) {
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= n)
        return;
    const int64_t i = idx[p];
    for (int a = 0; a < d; ++a)
        xs[(int64_t)a * n + p] = x[(int64_t)a * n + i];
    if (ws)
        ws[p] = (double)w[i];
}

// start[c] = first sorted position whose key is >= c, c = 0 .. cells: cell
// c holds the positions [start[c], start[c+1]); left-out points come after
__global__ __launch_bounds__(256) void k_gk_starts(const uint32_t *__restrict__ key, int64_t n,
                                                   int64_t cells, uint32_t *__restrict__ start) {
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (c > cells)
        return;
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if ((int64_t)key[mid] < c)
            lo = mid + 1;
        else
            hi = mid;
    }
    start[c] = (uint32_t)lo;
}

// Corners per thread: all 2^D up to D = 2, else 4 (axes 0 and 1 vary; the
// bits of the other axes are fixed by the thread's corner group).
template <int D> constexpr int gk_ncg() { return D <= 2 ? (1 << D) : 4; }

// Bandwidths of a launch group each thread sums (the cell's points are read
// once for all of them): as many as keep the sums of one thread to about 16
// values (NCG corners x NT slots x CH values each).
template <int D, int CH, int NT> constexpr int gk_nbw() {
    return gk_ncg<D>() * NT * CH <= 4 ? 4 : (gk_ncg<D>() * NT * CH <= 8 ? 2 : 1);
}

// Bin arrays: corner q, slot u (0: S; 1 + l: T_l, Matern only), value v
// (CH = 1: the weights w or 1; CH = 2: 1 and y), each of g.nodes doubles at
// ((q * NT + u) * CH + v) * g.nodes, for bandwidth b of the group at b *
// bins_stride.  The workgroups of grid row y take the bandwidths [y NBW,
// y NBW + NBW) of the nb in the group.
template <int D, int CH, int NT, int NBW>
__global__ __launch_bounds__(256) void k_gk_bins(GkGrid g, const double *__restrict__ zn,
                                                 const double *__restrict__ xs, int64_t n,
                                                 const uint32_t *__restrict__ start,
                                                 const double *__restrict__ w0,
                                                 const double *__restrict__ w1, GkHs hs, int nb,
                                                 double *__restrict__ bins_all,
                                                 int64_t bins_stride) {
    const int bb = (int)blockIdx.y * NBW;  // first bandwidth of this row
    constexpr int NCG = gk_ncg<D>();
    constexpr int NG = (1 << D) / NCG;
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= g.cells * NG)
        return;
    const int grp = (int)(t / g.cells);
    const int64_t cell = t - (int64_t)grp * g.cells;
    int64_t c[D];
    {
        int64_t rem = cell;
#pragma unroll
        for (int a = 0; a < D; ++a) {
            c[a] = rem / g.cst[a];
            rem -= c[a] * g.cst[a];
        }
    }
    const int qbase = grp * NCG;
    double s[NBW][NCG][NT][CH], e[NBW][NCG][NT][CH];
#pragma unroll
    for (int j = 0; j < NBW; ++j)
#pragma unroll
        for (int q = 0; q < NCG; ++q)
#pragma unroll
            for (int u = 0; u < NT; ++u)
#pragma unroll
                for (int v = 0; v < CH; ++v)
                    s[j][q][u][v] = e[j][q][u][v] = 0.0;
    const int64_t p0 = start[cell], p1 = start[cell + 1];
    // the next point's coordinates and weight are loaded while this one is
    // summed
    double nx[D], nw = 0.0;
    if (p0 < p1) {
#pragma unroll
        for (int a = 0; a < D; ++a)
            nx[a] = xs[(int64_t)a * n + p0];
        nw = CH == 1 ? (w0 ? w0[p0] : 1.0) : w1[p0];
    }
    for (int64_t p = p0; p < p1; ++p) {
        double cx[D];
#pragma unroll
        for (int a = 0; a < D; ++a)
            cx[a] = nx[a];
        const double cw = nw;
        if (p + 1 < p1) {
#pragma unroll
            for (int a = 0; a < D; ++a)
                nx[a] = xs[(int64_t)a * n + p + 1];
            nw = CH == 1 ? (w0 ? w0[p + 1] : 1.0) : w1[p + 1];
        }
        // distances to the cell's upper and lower node on each axis
        double ru[D], rd[D];
        bool hu[D], hd[D];
#pragma unroll
        for (int a = 0; a < D; ++a) {
            const double v = cx[a];
            const double *z = zn + g.off[a];
            hu[a] = c[a] < g.M[a];
            hd[a] = c[a] > 0;
            ru[a] = hu[a] ? z[c[a]] - v : 0.0;
            rd[a] = hd[a] ? v - z[c[a] - 1] : 0.0;
        }
        double wv[CH];
        if (CH == 1) {
            wv[0] = cw;
        } else {
            wv[0] = 1.0;
            wv[CH - 1] = cw;
        }
#pragma unroll
        for (int j = 0; j < NBW; ++j) {
            if (bb + j >= nb)
                break;
            const GkH &hb = hs.h[bb + j];
            double du[D], dd[D], fu[D], fd[D];
#pragma unroll
            for (int a = 0; a < D; ++a) {
                du[a] = ru[a] * hb.ih[a];
                dd[a] = rd[a] * hb.ih[a];
                // only the factors this thread's corners use
                const bool vary = D <= 2 || a < 2;
                const bool upb = ((qbase >> a) & 1) != 0;
                fu[a] = (hu[a] && (vary || upb)) ? exp(-du[a]) : 0.0;
                fd[a] = (hd[a] && (vary || !upb)) ? exp(-dd[a]) : 0.0;
            }
#pragma unroll
            for (int lq = 0; lq < NCG; ++lq) {
                const int q = qbase + lq;
                double f = 1.0;
#pragma unroll
                for (int a = 0; a < D; ++a)
                    f *= ((q >> a) & 1) ? fu[a] : fd[a];
#pragma unroll
                for (int u = 0; u < NT; ++u) {
                    const double fq =
                        u == 0 ? f : f * (((q >> (u - 1)) & 1) ? du[u - 1] : dd[u - 1]);
#pragma unroll
                    for (int v = 0; v < CH; ++v) {
                        double &sv = s[j][lq][u][v];
                        const double tv = fq * wv[v];
                        const double sm = sv + tv;
                        e[j][lq][u][v] +=
                            fabs(sv) >= fabs(tv) ? (sv - sm) + tv : (tv - sm) + sv;
                        sv = sm;
                    }
                }
            }
        }
    }
#pragma unroll
    for (int lq = 0; lq < NCG; ++lq) {
        const int q = qbase + lq;
        int64_t node = 0;
        bool inside = true;
#pragma unroll
        for (int a = 0; a < D; ++a) {
            const int64_t jn = ((q >> a) & 1) ? c[a] : c[a] - 1;
            inside = inside && jn >= 0 && jn < g.M[a];
            node += jn * g.nst[a];
        }
        if (!inside)
            continue;
#pragma unroll
        for (int j = 0; j < NBW; ++j) {
            if (bb + j >= nb)
                break;
            double *__restrict__ bins = bins_all + (int64_t)(bb + j) * bins_stride;
#pragma unroll
            for (int u = 0; u < NT; ++u)
#pragma unroll
                for (int v = 0; v < CH; ++v)
                    bins[((int64_t)(q * NT + u) * CH + v) * g.nodes + node] =
                        s[j][lq][u][v] + e[j][lq][u][v];
        }
    }
}

// decays between neighbouring nodes: dec[off_a + j] = exp(-(z_j - z_{j-1}) ih_a), j >= 1
__global__ void k_gk_decays(GkGrid g, const double *__restrict__ zn, GkHs hs, int64_t total,
                            double *__restrict__ dec_all) {
    const GkH &hb = hs.h[blockIdx.y];
    double *__restrict__ dec = dec_all + (int64_t)blockIdx.y * total;
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= total)
        return;
    int a = 0;
    while (a + 1 < g.d && t >= g.off[a + 1])
        ++a;
    const int64_t j = t - g.off[a];
    dec[t] = j == 0 ? 0.0 : exp(-(zn[t] - zn[t - 1]) * hb.ih[a]);
}

// ---- scans along one axis ------------------------------------------------
//
// Stage k scans axis k.  Its input holds 2^(d-k) corners (bit 0: axis k,
// bit 1: axis k+1, ...), its output 2^(d-k-1): output corner co is the sum of
// the forward scan of input corner 2co+1 (upper nodes on axis k) and the
// backward scan of input corner 2co.  Slots: 0 = S; Matern: 1 = R (at k = 0
// the channel T_0) and 1 + l = T_l for the axes l > k not yet scanned; the
// pair (S, T_k) takes the affine step, the others the plain decay, and the
// output's R is R + T_k.
struct GsArgs {
    const double *in;
    double *out;
    double *agg;        // [chunk][dir][nt][col]: chunk sums, then entering values
    const double *dec;  // decays of axis k (dec[0] unused)
    const double *z;    // nodes of axis k
    const double *span; // [dir][chunk][2]: the transfer of each chunk (P, G)
    double ih;
    int64_t M, inner, outer, nodes, nck, cols;
    int nco, k, nt;
};

struct GsBatch {
    GsArgs a[kGkGroup];
};

struct GsCol {
    int co, v;
    int64_t chunk, col, base;  // base: offset of this line's node 0 inside an array
};

template <int CH>
__device__ __forceinline__ GsCol gs_map(const GsArgs &a, int64_t t) {
    GsCol c;
    int64_t r, oi, ii;
    if (a.inner >= 16) {  // neighbouring threads on neighbouring lines
        ii = t % a.inner;
        r = t / a.inner;
        c.chunk = r % a.nck;
        r /= a.nck;
    } else {              // neighbouring threads on neighbouring chunks
        c.chunk = t % a.nck;
        r = t / a.nck;
        ii = r % a.inner;
        r /= a.inner;
    }
    oi = r % a.outer;
    r /= a.outer;
    c.v = (int)(r % CH);
    c.co = (int)(r / CH);
    c.col = (((int64_t)c.co * CH + c.v) * a.outer + oi) * a.inner + ii;
    c.base = oi * a.M * a.inner + ii;
    return c;
}

template <int CH>
__device__ __forceinline__ int64_t gs_arr(const GsArgs &a, int corner, int slot, int v) {
    return ((int64_t)(corner * a.nt + slot) * CH + v) * a.nodes;
}

// the chunk-sum slot of (column, chunk, direction, slot)
__device__ __forceinline__ int64_t gs_agg(const GsArgs &a, int64_t col, int64_t ch, int dir,
                                          int slot) {
    return ((ch * 2 + dir) * a.nt + slot) * a.cols + col;
}

// The transfer across each chunk, the same for every line of the axis:
// forward, from the node before chunk c to its last node; backward, from the
// node after it to its first node: P = exp(-span / h), G = span / h.
__global__ __launch_bounds__(256) void k_gs_spans(GsBatch gb) {
    const GsArgs &a = gb.a[blockIdx.y];
    const double *__restrict__ z = a.z;
    const int64_t M = a.M, nck = a.nck;
    const double ih = a.ih;
    double *__restrict__ span = const_cast<double *>(a.span);
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= 2 * nck)
        return;
    const int dir = (int)(t / nck);
    const int64_t ch = t - (int64_t)dir * nck;
    const int64_t j0 = ch * kGkL;
    const int64_t j1 = j0 + kGkL < M ? j0 + kGkL : M;
    double sp = 0.0;
    bool ok;
    if (dir == 0) {
        ok = ch > 0;
        if (ok)
            sp = z[j1 - 1] - z[j0 - 1];
    } else {
        ok = ch + 1 < nck;
        if (ok)
            sp = z[j1] - z[j0];
    }
    span[2 * t] = ok ? exp(-sp * ih) : 0.0;
    span[2 * t + 1] = sp * ih;
}

// Matern slots taking the plain decay at stage k: R (from the second stage
// on) and the T_l of the axes l > k
__device__ __forceinline__ bool gs_plain(const GsArgs &a, int slot) {
    if (slot == 1)
        return a.k >= 1;
    return slot - 1 > a.k;
}

template <int CH, bool MAT>
__global__ __launch_bounds__(256) void k_gs_agg(GsBatch gb, int64_t total) {
    const GsArgs &a = gb.a[blockIdx.y];
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= total)
        return;
    const GsCol c = gs_map<CH>(a, t);
    const int64_t j0 = c.chunk * kGkL;
    const int64_t j1 = j0 + kGkL < a.M ? j0 + kGkL : a.M;
    const int64_t st = a.inner;
    const int ps = 1 + a.k;  // the slot paired with S (Matern)
    for (int dir = 0; dir < 2; ++dir) {
        const int corner = 2 * c.co + (dir == 0 ? 1 : 0);  // forward: upper nodes
        const double *sI = a.in + gs_arr<CH>(a, corner, 0, c.v) + c.base;
        const double *tI = MAT ? a.in + gs_arr<CH>(a, corner, ps, c.v) + c.base : sI;
        double rs = 0.0, rt = 0.0;
        if (dir == 0) {
            for (int64_t j = j0; j < j1; ++j) {
                const double dk = j > j0 ? a.dec[j] : 0.0;
                if (MAT) {
                    const double gk = j > j0 ? (a.z[j] - a.z[j - 1]) * a.ih : 0.0;
                    rt = dk * (rt + gk * rs) + tI[j * st];
                }
                rs = dk * rs + sI[j * st];
            }
        } else {
            for (int64_t j = j1 - 1; j >= j0; --j) {
                const double dk = j + 1 < j1 ? a.dec[j + 1] : 0.0;
                if (MAT) {
                    const double gk = j + 1 < j1 ? (a.z[j + 1] - a.z[j]) * a.ih : 0.0;
                    rt = dk * (rt + gk * rs) + tI[j * st];
                }
                rs = dk * rs + sI[j * st];
            }
        }
        a.agg[gs_agg(a, c.col, c.chunk, dir, 0)] = rs;
        if (MAT) {
            a.agg[gs_agg(a, c.col, c.chunk, dir, ps)] = rt;
            for (int sl = 1; sl < a.nt; ++sl) {
                if (!gs_plain(a, sl))
                    continue;
                const double *pI = a.in + gs_arr<CH>(a, corner, sl, c.v) + c.base;
                double r = 0.0;
                if (dir == 0)
                    for (int64_t j = j0; j < j1; ++j)
                        r = (j > j0 ? a.dec[j] : 0.0) * r + pI[j * st];
                else
                    for (int64_t j = j1 - 1; j >= j0; --j)
                        r = (j + 1 < j1 ? a.dec[j + 1] : 0.0) * r + pI[j * st];
                a.agg[gs_agg(a, c.col, c.chunk, dir, sl)] = r;
            }
        }
    }
}

// One thread per (line, direction): the chunk sums become, in place, the
// values entering each chunk (forward: the scan at the node before the
// chunk; backward: at the node after it).  Neighbouring threads take
// neighbouring lines, whose chunk sums sit next to each other.
template <bool MAT>
__global__ __launch_bounds__(256) void k_gs_carry(GsBatch gb) {
    const GsArgs &a = gb.a[blockIdx.y];
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= 2 * a.cols)
        return;
    const int dir = (int)(t / a.cols);
    const int64_t col = t - (int64_t)dir * a.cols;
    const int ps = 1 + a.k;
    constexpr int kMaxSlots = 1 + MECDF_MAX_DIM;
    constexpr int kG = 16;  // chunk sums loaded together before the serial steps
    double cr[kMaxSlots];
    for (int sl = 0; sl < kMaxSlots; ++sl)
        cr[sl] = 0.0;
    const double *sp = a.span + (int64_t)dir * a.nck * 2;
    for (int64_t i0 = 0; i0 < a.nck; i0 += kG) {
        const int ng = (int)(a.nck - i0 < kG ? a.nck - i0 : kG);
        // S first: its values before each step feed the pair's update
        double s0[kG];
        {
            double v[kG];
#pragma unroll
            for (int g = 0; g < kG; ++g) {
                const int64_t i = i0 + g;
                const int64_t ch = dir == 0 ? i : a.nck - 1 - i;
                v[g] = g < ng ? a.agg[gs_agg(a, col, ch, dir, 0)] : 0.0;
            }
#pragma unroll
            for (int g = 0; g < kG; ++g) {
                if (g >= ng)
                    break;
                const int64_t i = i0 + g;
                const int64_t ch = dir == 0 ? i : a.nck - 1 - i;
                s0[g] = cr[0];
                a.agg[gs_agg(a, col, ch, dir, 0)] = cr[0];
                cr[0] = sp[2 * ch] * cr[0] + v[g];
            }
        }
        if (MAT) {
            for (int sl = 1; sl < a.nt; ++sl) {
                const bool pair = sl == ps;
                if (!pair && !gs_plain(a, sl))
                    continue;
                double v[kG];
#pragma unroll
                for (int g = 0; g < kG; ++g) {
                    const int64_t i = i0 + g;
                    const int64_t ch = dir == 0 ? i : a.nck - 1 - i;
                    v[g] = g < ng ? a.agg[gs_agg(a, col, ch, dir, sl)] : 0.0;
                }
#pragma unroll
                for (int g = 0; g < kG; ++g) {
                    if (g >= ng)
                        break;
                    const int64_t i = i0 + g;
                    const int64_t ch = dir == 0 ? i : a.nck - 1 - i;
                    const double P = sp[2 * ch], G = sp[2 * ch + 1];
                    const double old = cr[sl];
                    a.agg[gs_agg(a, col, ch, dir, sl)] = old;
                    cr[sl] = pair ? P * (old + G * s0[g]) + v[g] : P * old + v[g];
                }
            }
        }
    }
}

// A double from another lane by a DPP move: update (rows outside RM keep
// 0) or with bound_ctrl (lanes without a source lane get 0).
template <int CTRL, int RM> __device__ __forceinline__ double gs_dpp(double v) {
    union {
        double t;
        int i[2];
    } u;
    u.t = v;
    u.i[0] = __builtin_amdgcn_update_dpp(0, u.i[0], CTRL, RM, 0xf, false);
    u.i[1] = __builtin_amdgcn_update_dpp(0, u.i[1], CTRL, RM, 0xf, false);
    return u.t;
}
template <int CTRL> __device__ __forceinline__ double gs_dppz(double v) {
    union {
        double t;
        int i[2];
    } u;
    u.t = v;
    u.i[0] = __builtin_amdgcn_mov_dpp(u.i[0], CTRL, 0xf, 0xf, true);
    u.i[1] = __builtin_amdgcn_mov_dpp(u.i[1], CTRL, 0xf, 0xf, true);
    return u.t;
}

// The step y -> A y + B of each lane composed with those of the lanes before
// it: forward (dir 0: lanes 0..i) or backward (dir 1: lanes 63..i), so that
// lane i maps the value entering the wavefront's first lane in that order to
// its own.  A move from a lane outside the source range brings B = 0, which
// adds nothing; only A needs the choice.  DPP controls as in the kernel-sum
// scans: row_shr / row_shl 1, 2, 4, 8 (0x110 + n, 0x100 + n), row_bcast:15 /
// :31 (0x142, 0x143).
__device__ __forceinline__ void gs_wave_affine(int dir, double &A, double &B) {
    const int lane = threadIdx.x & 63;
    const int rl = lane & 15, row = lane >> 4;
#define MECDF_GS_STEP(MOVE, TAKE)                                                                 \
    {                                                                                             \
        const double Ao = MOVE(A), Bo = MOVE(B);                                                  \
        B = fma(A, Bo, B);                                                                        \
        A = (TAKE) ? A * Ao : A;                                                                  \
    }
    if (dir == 0) {
        MECDF_GS_STEP(gs_dppz<0x111>, rl >= 1)
        MECDF_GS_STEP(gs_dppz<0x112>, rl >= 2)
        MECDF_GS_STEP(gs_dppz<0x114>, rl >= 4)
        MECDF_GS_STEP(gs_dppz<0x118>, rl >= 8)
        MECDF_GS_STEP((gs_dpp<0x142, 0xa>), (row & 1) != 0)
        MECDF_GS_STEP((gs_dpp<0x143, 0xc>), row >= 2)
    } else {
        MECDF_GS_STEP(gs_dppz<0x101>, rl + 1 < 16)
        MECDF_GS_STEP(gs_dppz<0x102>, rl + 2 < 16)
        MECDF_GS_STEP(gs_dppz<0x104>, rl + 4 < 16)
        MECDF_GS_STEP(gs_dppz<0x108>, rl + 8 < 16)
        {
            // the first lane of the next row (rows 0 and 2), then lane 32
            // (rows 0 and 1); other lanes take nothing
            const bool t1 = (row & 1) == 0;
            const int src1 = (16 * (row + 1)) & 63;
            const double Ao = __shfl(A, src1), Bo = __shfl(B, src1);
            B = t1 ? fma(A, Bo, B) : B;
            A = t1 ? A * Ao : A;
            const bool t2 = row < 2;
            const double Ao2 = __shfl(A, 32), Bo2 = __shfl(B, 32);
            B = t2 ? fma(A, Bo2, B) : B;
            A = t2 ? A * Ao2 : A;
        }
    }
#undef MECDF_GS_STEP
}

// The Laplacian scan along the contiguous axis (inner == 1) when a line fits
// kGsRowBlocks blocks of 64 nodes: one wavefront per line and corner pair,
// 64 nodes at a time, each block's steps composed across the lanes and
// entered by the value the block before left (its last lane forward, first
// lane backward).  Loads and stores are whole 512-byte rows; the forward
// results wait in registers for the backward ones, and their sum is written
// once.  Replaces the chunk sums, carries and chunk scans of this axis.
constexpr int kGsRowBlocks = 16;
template <int CH>
__global__ __launch_bounds__(256) void k_gs_rows(GsBatch gb) {
    const GsArgs &a = gb.a[blockIdx.y];
    const int lane = threadIdx.x & 63;
    const int64_t col = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (col >= a.cols)
        return;  // whole wavefronts
    const int64_t oi = col % a.outer;
    const int64_t r = col / a.outer;
    const int v = (int)(r % CH), co = (int)(r / CH);
    const int64_t M = a.M, base = oi * M;
    const double *__restrict__ sU = a.in + gs_arr<CH>(a, 2 * co + 1, 0, v) + base;
    const double *__restrict__ sD = a.in + gs_arr<CH>(a, 2 * co, 0, v) + base;
    double *__restrict__ oS = a.out + gs_arr<CH>(a, co, 0, v) + base;
    const int nb = (int)((M + 63) >> 6);
    double fs[kGsRowBlocks];
    double carry = 0.0;
#pragma unroll
    for (int b = 0; b < kGsRowBlocks; ++b) {
        if (b < nb) {
            // forward into node j: the decay from node j - 1 (none before node 0)
            const int64_t j = (int64_t)b * 64 + lane;
            const bool ok = j < M;
            double A = (ok && j > 0) ? a.dec[j] : 0.0;
            double B = ok ? sU[j] : 0.0;
            gs_wave_affine(0, A, B);
            const double y = fma(A, carry, B);
            fs[b] = y;
            carry = __shfl(y, 63);
        }
    }
    carry = 0.0;
#pragma unroll
    for (int b = kGsRowBlocks - 1; b >= 0; --b) {
        if (b < nb) {
            // backward into node j: the decay from node j + 1 (none after the
            // last node, which also stops the lanes past the end)
            const int64_t j = (int64_t)b * 64 + lane;
            const bool ok = j < M;
            double A = (ok && j + 1 < M) ? a.dec[j + 1] : 0.0;
            double B = ok ? sD[j] : 0.0;
            gs_wave_affine(1, A, B);
            const double y = fma(A, carry, B);
            if (ok)
                oS[j] = fs[b] + y;
            carry = __shfl(y, 0);
        }
    }
}

// The Matern pair (S, T) of the scanned axis moves by (s, t) -> (d s + S_j,
// d (t + g s) + T_j): a map with parameters (a, c, bs, bt) standing for
// s -> a s + bs, t -> c s + a t + bt.  gs_wave_pair composes these maps across
// the lanes as gs_wave_affine does the plain ones (moves from outside the
// source range bring zeros: only a and c need the choice).
__device__ __forceinline__ void gs_pair_then(double Pa, double Pc, double Pbs, double Pbt,
                                             bool take, double &a, double &c, double &bs,
                                             double &bt) {
    // own map after P: bt uses the old c and a
    bt = fma(c, Pbs, fma(a, Pbt, bt));
    bs = fma(a, Pbs, bs);
    const double nc = fma(c, Pa, a * Pc);
    c = take ? nc : c;
    a = take ? a * Pa : a;
}
__device__ __forceinline__ void gs_wave_pair(int dir, double &a, double &c, double &bs,
                                             double &bt) {
    const int lane = threadIdx.x & 63;
    const int rl = lane & 15, row = lane >> 4;
#define MECDF_GS_PSTEP(MOVE, TAKE)                                                               \
    {                                                                                            \
        const double Pa = MOVE(a), Pc = MOVE(c), Pbs = MOVE(bs), Pbt = MOVE(bt);                 \
        gs_pair_then(Pa, Pc, Pbs, Pbt, (TAKE), a, c, bs, bt);                                    \
    }
    if (dir == 0) {
        MECDF_GS_PSTEP(gs_dppz<0x111>, rl >= 1)
        MECDF_GS_PSTEP(gs_dppz<0x112>, rl >= 2)
        MECDF_GS_PSTEP(gs_dppz<0x114>, rl >= 4)
        MECDF_GS_PSTEP(gs_dppz<0x118>, rl >= 8)
        MECDF_GS_PSTEP((gs_dpp<0x142, 0xa>), (row & 1) != 0)
        MECDF_GS_PSTEP((gs_dpp<0x143, 0xc>), row >= 2)
    } else {
        MECDF_GS_PSTEP(gs_dppz<0x101>, rl + 1 < 16)
        MECDF_GS_PSTEP(gs_dppz<0x102>, rl + 2 < 16)
        MECDF_GS_PSTEP(gs_dppz<0x104>, rl + 4 < 16)
        MECDF_GS_PSTEP(gs_dppz<0x108>, rl + 8 < 16)
        {
            // every lane takes part in each shuffle (a source lane must be
            // active); the lanes that take nothing then drop the sums
            const bool t1 = (row & 1) == 0;
            const int src1 = (16 * (row + 1)) & 63;
            const double Pa = __shfl(a, src1), Pc = __shfl(c, src1);
            const double Pbs = __shfl(bs, src1), Pbt = __shfl(bt, src1);
            gs_pair_then(Pa, Pc, t1 ? Pbs : 0.0, t1 ? Pbt : 0.0, t1, a, c, bs, bt);
            const bool t2 = row < 2;
            const double Qa = __shfl(a, 32), Qc = __shfl(c, 32);
            const double Qbs = __shfl(bs, 32), Qbt = __shfl(bt, 32);
            gs_pair_then(Qa, Qc, t2 ? Qbs : 0.0, t2 ? Qbt : 0.0, t2, a, c, bs, bt);
        }
    }
#undef MECDF_GS_PSTEP
}

// The Matern-3/2 form of k_gs_rows (the contiguous axis is the last one, so
// no T_l of a later axis is left): S and the axis's own T_k as pairs, R
// (slot 1, from the second axis on) by the plain steps; the output holds S
// and R' = T_k + R, both directions added.
template <int CH>
__global__ __launch_bounds__(256) void k_gs_rows_mat(GsBatch gb) {
    const GsArgs &a = gb.a[blockIdx.y];
    const int lane = threadIdx.x & 63;
    const int64_t col = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (col >= a.cols)
        return;  // whole wavefronts
    const int64_t oi = col % a.outer;
    const int64_t r = col / a.outer;
    const int v = (int)(r % CH), co = (int)(r / CH);
    const int64_t M = a.M, base = oi * M;
    const int ps = 1 + a.k;
    const bool hasR = a.k >= 1;
    const int up = 2 * co + 1, dn = 2 * co;
    const double *__restrict__ sU = a.in + gs_arr<CH>(a, up, 0, v) + base;
    const double *__restrict__ tU = a.in + gs_arr<CH>(a, up, ps, v) + base;
    const double *__restrict__ rU = a.in + gs_arr<CH>(a, up, 1, v) + base;
    const double *__restrict__ sD = a.in + gs_arr<CH>(a, dn, 0, v) + base;
    const double *__restrict__ tD = a.in + gs_arr<CH>(a, dn, ps, v) + base;
    const double *__restrict__ rD = a.in + gs_arr<CH>(a, dn, 1, v) + base;
    double *__restrict__ oS = a.out + gs_arr<CH>(a, co, 0, v) + base;
    double *__restrict__ oR = a.out + gs_arr<CH>(a, co, 1, v) + base;
    const int nb = (int)((M + 63) >> 6);
    double fs[kGsRowBlocks], ft[kGsRowBlocks];
    double cs = 0.0, ct = 0.0, cr = 0.0;
#pragma unroll
    for (int b = 0; b < kGsRowBlocks; ++b) {
        if (b < nb) {
            const int64_t j = (int64_t)b * 64 + lane;
            const bool ok = j < M;
            const bool st = ok && j > 0;
            const double dk = st ? a.dec[j] : 0.0;
            const double gk = st ? (a.z[j] - a.z[j - 1]) * a.ih : 0.0;
            double pa = dk, pc = dk * gk, bs = ok ? sU[j] : 0.0, bt = ok ? tU[j] : 0.0;
            gs_wave_pair(0, pa, pc, bs, bt);
            const double ys = fma(pa, cs, bs);
            const double yt = fma(pc, cs, fma(pa, ct, bt));
            fs[b] = ys;
            ft[b] = yt;
            cs = __shfl(ys, 63);
            ct = __shfl(yt, 63);
            if (hasR) {
                double A = dk, B = ok ? rU[j] : 0.0;
                gs_wave_affine(0, A, B);
                const double yr = fma(A, cr, B);
                ft[b] += yr;
                cr = __shfl(yr, 63);
            }
        }
    }
    cs = ct = cr = 0.0;
#pragma unroll
    for (int b = kGsRowBlocks - 1; b >= 0; --b) {
        if (b < nb) {
            const int64_t j = (int64_t)b * 64 + lane;
            const bool ok = j < M;
            const bool st = ok && j + 1 < M;
            const double dk = st ? a.dec[j + 1] : 0.0;
            const double gk = st ? (a.z[j + 1] - a.z[j]) * a.ih : 0.0;
            double pa = dk, pc = dk * gk, bs = ok ? sD[j] : 0.0, bt = ok ? tD[j] : 0.0;
            gs_wave_pair(1, pa, pc, bs, bt);
            const double ys = fma(pa, cs, bs);
            const double yt = fma(pc, cs, fma(pa, ct, bt));
            cs = __shfl(ys, 0);
            ct = __shfl(yt, 0);
            double tot = ft[b] + yt;
            if (hasR) {
                double A = dk, B = ok ? rD[j] : 0.0;
                gs_wave_affine(1, A, B);
                const double yr = fma(A, cr, B);
                tot += yr;
                cr = __shfl(yr, 0);
            }
            if (ok) {
                oS[j] = fs[b] + ys;
                oR[j] = tot;
            }
        }
    }
}

template <int CH, bool MAT>
__global__ __launch_bounds__(256) void k_gs_apply(GsBatch gb, int64_t total) {
    const GsArgs &a = gb.a[blockIdx.y];
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= total)
        return;
    const GsCol c = gs_map<CH>(a, t);
    const int64_t j0 = c.chunk * kGkL;
    const int n = (int)((j0 + kGkL < a.M ? j0 + kGkL : a.M) - j0);
    const double *ag = a.agg;
    const int ps = 1 + a.k;
    auto entering = [&](int dir, int slot) { return ag[gs_agg(a, c.col, c.chunk, dir, slot)]; };
    // dk[i], gk[i]: the step between nodes j0+i-1 and j0+i (forward into
    // j0+i, backward out of it); i = n is the step from the next chunk
    double dk[kGkL + 1], gk[kGkL + 1];
#pragma unroll
    for (int i = 0; i <= kGkL; ++i) {
        const int64_t j = j0 + i;
        const bool ok = i <= n && j > 0 && j < a.M;
        dk[i] = ok ? a.dec[j] : 0.0;
        gk[i] = (MAT && ok) ? (a.z[j] - a.z[j - 1]) * a.ih : 0.0;
    }
    const int64_t st = a.inner;
    const int64_t off = c.base + j0 * st;
    const int up = 2 * c.co + 1, dn = 2 * c.co;
    double fs[kGkL], ft[kGkL];
    {
        const double *sU = a.in + gs_arr<CH>(a, up, 0, c.v) + off;
        const double *sD = a.in + gs_arr<CH>(a, dn, 0, c.v) + off;
        const double *tU = MAT ? a.in + gs_arr<CH>(a, up, ps, c.v) + off : sU;
        const double *tD = MAT ? a.in + gs_arr<CH>(a, dn, ps, c.v) + off : sD;
        double *oS = a.out + gs_arr<CH>(a, c.co, 0, c.v) + off;
        double rs = entering(0, 0), rt = MAT ? entering(0, ps) : 0.0;
#pragma unroll
        for (int i = 0; i < kGkL; ++i) {
            if (i < n) {
                if (MAT)
                    rt = dk[i] * (rt + gk[i] * rs) + tU[i * st];
                rs = dk[i] * rs + sU[i * st];
            }
            fs[i] = rs;
            ft[i] = rt;
        }
        rs = entering(1, 0);
        rt = MAT ? entering(1, ps) : 0.0;
#pragma unroll
        for (int i = kGkL - 1; i >= 0; --i) {
            if (i < n) {
                if (MAT)
                    rt = dk[i + 1] * (rt + gk[i + 1] * rs) + tD[i * st];
                rs = dk[i + 1] * rs + sD[i * st];
                oS[i * st] = fs[i] + rs;
                ft[i] += rt;
            }
        }
    }
    if constexpr (MAT) {
        // R' = T_k + R (R from the second stage on)
        double *oR = a.out + gs_arr<CH>(a, c.co, 1, c.v) + off;
        if (a.k >= 1) {
            const double *rU = a.in + gs_arr<CH>(a, up, 1, c.v) + off;
            const double *rD = a.in + gs_arr<CH>(a, dn, 1, c.v) + off;
            double r = entering(0, 1);
#pragma unroll
            for (int i = 0; i < kGkL; ++i) {
                if (i < n)
                    r = dk[i] * r + rU[i * st];
                ft[i] += r;
            }
            r = entering(1, 1);
#pragma unroll
            for (int i = kGkL - 1; i >= 0; --i) {
                if (i < n) {
                    r = dk[i + 1] * r + rD[i * st];
                    oR[i * st] = ft[i] + r;
                }
            }
        } else {
#pragma unroll
            for (int i = 0; i < kGkL; ++i)
                if (i < n)
                    oR[i * st] = ft[i];
        }
        // the T_l of the axes not yet scanned
        for (int sl = 2 + a.k; sl < a.nt; ++sl) {
            const double *pU = a.in + gs_arr<CH>(a, up, sl, c.v) + off;
            const double *pD = a.in + gs_arr<CH>(a, dn, sl, c.v) + off;
            double *oP = a.out + gs_arr<CH>(a, c.co, sl, c.v) + off;
            double r = entering(0, sl);
#pragma unroll
            for (int i = 0; i < kGkL; ++i) {
                if (i < n)
                    r = dk[i] * r + pU[i * st];
                fs[i] = r;
            }
            r = entering(1, sl);
#pragma unroll
            for (int i = kGkL - 1; i >= 0; --i) {
                if (i < n) {
                    r = dk[i + 1] * r + pD[i * st];
                    oP[i * st] = fs[i] + r;
                }
            }
        }
    }
}

// out[node] = norm * (S + R) (CH = 1), or the ratio of the second value's to
// the first value's S + R (CH = 2); R only for the Matern kernel
struct GkNorms {
    double v[kGkGroup];
};

template <int CH, typename OutT>
__global__ __launch_bounds__(256) void k_gk_combine(GkGrid g, const double *__restrict__ fin_all,
                                                    int64_t fin_stride, int matern, GkNorms nm,
                                                    OutT *__restrict__ out_all) {
    const double *__restrict__ fin = fin_all + (int64_t)blockIdx.y * fin_stride;
    OutT *__restrict__ out = out_all + (int64_t)blockIdx.y * g.nodes;
    const double norm = nm.v[blockIdx.y];
    const int64_t node = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (node >= g.nodes)
        return;
    double s[CH];
#pragma unroll
    for (int v = 0; v < CH; ++v) {
        s[v] = fin[(int64_t)v * g.nodes + node];
        if (matern)
            s[v] += fin[(int64_t)(CH + v) * g.nodes + node];
    }
    out[node] = CH == 1 ? (OutT)(s[0] * norm) : (OutT)(s[CH - 1] / s[0]);
}

// the bandwidths of a group share every size; only pointers and 1/h differ
template <int CH, bool MAT>
static void gs_launch(const GsBatch &gb, int nb, hipStream_t s) {
    const GsArgs &ga = gb.a[0];
    const int64_t tot = ga.cols * ga.nck;
    hipLaunchKernelGGL(k_gs_spans, dim3((unsigned)ceil_div(2 * ga.nck, 256), nb), dim3(256), 0,
                       s, gb);
    hipLaunchKernelGGL((k_gs_agg<CH, MAT>), dim3((unsigned)ceil_div(tot, 256), nb), dim3(256), 0,
                       s, gb, tot);
    hipLaunchKernelGGL(k_gs_carry<MAT>, dim3((unsigned)ceil_div(2 * ga.cols, 256), nb),
                       dim3(256), 0, s, gb);
    hipLaunchKernelGGL((k_gs_apply<CH, MAT>), dim3((unsigned)ceil_div(tot, 256), nb), dim3(256),
                       0, s, gb, tot);
}

template <int CH, typename WT, typename OutT>
static int gridkde_t(int d, int64_t N, const double *x, const WT *w, const int64_t *M,
                     const double *z, int nh, const double *h, OutT *out, int matern,
                     hipStream_t s) {
    GkGrid g{};
    g.d = d;
    int64_t total = 0;
    for (int a = 0; a < d; ++a) {
        g.M[a] = M[a];
        g.C[a] = M[a] + 1;
        g.off[a] = total;
        g.z0[a] = z[total];
        g.zl[a] = z[total + M[a] - 1];
        g.gs[a] = g.zl[a] > g.z0[a] ? (double)(M[a] - 1) / (g.zl[a] - g.z0[a]) : 0.0;
        total += M[a];
    }
    int64_t cs = 1, ns = 1;
    for (int a = d - 1; a >= 0; --a) {
        g.cst[a] = cs;
        g.nst[a] = ns;
        cs *= g.C[a];
        ns *= g.M[a];
    }
    g.nodes = ns;
    g.cells = cs;
    const int nch = 1 << d;
    const int NT = matern ? 1 + d : 1;
    const int64_t nA = (int64_t)nch * NT * CH * g.nodes;
    const int64_t nB = (int64_t)(nch / 2) * NT * CH * g.nodes;
    int64_t nagg = 0, nspan = 0;
    for (int a = 0; a < d; ++a) {
        const int64_t cols = (int64_t)(nch >> (a + 1)) * CH * (g.nodes / g.M[a]);
        nagg = std::max(nagg, cols * ceil_div(g.M[a], kGkL) * 2 * NT);
        nspan = std::max(nspan, ceil_div(g.M[a], kGkL) * 4);
    }
    const bool has_w = CH == 2 || w != nullptr;
    // bandwidths per launch group: up to kGkGroup, fewer where the arrays of
    // one bandwidth are large (about 16 GB for a group at most)
    const double per_bw = 8.0 * (double)(nA + nB + nagg + nspan + total);
    int G = (int)std::min<double>((double)kGkGroup, std::max(1.0, 16e9 / per_bw));
    G = std::min(G, nh);
    ArenaPlan pl;
    pl.add<double>((size_t)total);          // nodes
    pl.add<double>((size_t)total * G);      // decays
    for (int q = 0; q < 3; ++q)
        pl.add<uint32_t>((size_t)N);        // keys
    for (int q = 0; q < 3; ++q)
        pl.add<uint32_t>((size_t)N);        // point indices
    pl.add<double>((size_t)N * d);          // coordinates in cell order
    if (has_w)
        pl.add<double>((size_t)N);          // weights / responses in cell order
    pl.add<uint32_t>((size_t)g.cells + 1);  // cell starts
    pl.add<double>((size_t)nA * G);
    pl.add<double>((size_t)nB * G);
    pl.add<double>((size_t)nagg * G);
    pl.add<double>((size_t)nspan * G);
    radix_plan(pl, N);
    void *wsb = nullptr;
    MECDF_TRY(workspace_reserve(pl.used, &wsb));
    Arena ar;
    ar.base = (char *)wsb;
    double *zn = ar.take<double>((size_t)total);
    double *dec = ar.take<double>((size_t)total * G);
    uint32_t *k0 = ar.take<uint32_t>((size_t)N), *k1 = ar.take<uint32_t>((size_t)N),
             *k2 = ar.take<uint32_t>((size_t)N);
    uint32_t *i0 = ar.take<uint32_t>((size_t)N), *i1 = ar.take<uint32_t>((size_t)N),
             *i2 = ar.take<uint32_t>((size_t)N);
    double *xs = ar.take<double>((size_t)N * d);
    double *ws = has_w ? ar.take<double>((size_t)N) : nullptr;
    uint32_t *cstart = ar.take<uint32_t>((size_t)g.cells + 1);
    double *bufA = ar.take<double>((size_t)nA * G);
    double *bufB = ar.take<double>((size_t)nB * G);
    double *agg = ar.take<double>((size_t)nagg * G);
    double *span = ar.take<double>((size_t)nspan * G);
    RadixScratch rs = radix_take(ar, N);
    MECDF_TRY(upload_small(z, sizeof(double) * (size_t)total, zn, s));
    const unsigned nbN = (unsigned)ceil_div(N, 256);
    // cell keys 0 .. cells-1, the value `cells` for points left out
    const uint32_t dropped = (uint32_t)cs;
    const int kbits = bits_for((uint64_t)cs);
    {
        ProfScope prof("gridkde_sort", s);
        const int hbits = std::min(kRadixMaxBits, kbits);
        hipLaunchKernelGGL(k_gk_keys, dim3((unsigned)ceil_div(N, kRadixTile)), dim3(256), 0, s, g,
                           zn, total, x, N, dropped, k0, i0, rs.hist, hbits);
        int which = 0;
        MECDF_TRY((radix_sort_bits<uint32_t, uint32_t>(k0, i0, k1, i1, k2, i2, N, 0, kbits, rs,
                                                       s, &which, true)));
        const uint32_t *ks = which == 1 ? k1 : (which == 2 ? k2 : k0);
        const uint32_t *is = which == 1 ? i1 : (which == 2 ? i2 : i0);
        hipLaunchKernelGGL((k_gk_gather<WT>), dim3(nbN), dim3(256), 0, s, is, N, d, x,
                           has_w ? w : (const WT *)nullptr, xs, ws);
        hipLaunchKernelGGL(k_gk_starts, dim3((unsigned)ceil_div(g.cells + 1, 256)), dim3(256), 0,
                           s, ks, N, g.cells, cstart);
        MECDF_LAUNCH_CHECK();
    }
    for (int b0 = 0; b0 < nh; b0 += G) {
        const int nb = std::min(G, nh - b0);
        GkHs hs{};
        GkNorms nm{};
        for (int j = 0; j < nb; ++j) {
            double prod = 1.0;
            for (int a = 0; a < d; ++a) {
                hs.h[j].ih[a] = 1.0 / h[(size_t)(b0 + j) * d + a];
                prod *= h[(size_t)(b0 + j) * d + a];
            }
            nm.v[j] = 1.0 / ((double)nch * (matern ? (double)(1 + d) : 1.0) * (double)N * prod);
        }
        {
            ProfScope prof("gridkde_bins", s);
            hipLaunchKernelGGL(k_gk_decays, dim3((unsigned)ceil_div(total, 256), nb), dim3(256), 0,
                               s, g, zn, hs, total, dec);
            const double *w0 = CH == 1 ? ws : nullptr;
            const double *w1 = CH == 2 ? ws : nullptr;
            const int ng = d <= 2 ? 1 : nch / 4;
            const unsigned nbc = (unsigned)ceil_div(g.cells * ng, 256);
#define MECDF_GKB(D, NTV)                                                                   \
    hipLaunchKernelGGL((k_gk_bins<D, CH, NTV, gk_nbw<D, CH, NTV>()>),                       \
                       dim3(nbc, (unsigned)ceil_div(nb, gk_nbw<D, CH, NTV>())), dim3(256), 0, s, \
                       g, zn, xs, N, cstart, w0, w1, hs, nb, bufA, nA)
            if (!matern) {
                switch (d) {
                case 1: MECDF_GKB(1, 1); break;
                case 2: MECDF_GKB(2, 1); break;
                case 3: MECDF_GKB(3, 1); break;
                case 4: MECDF_GKB(4, 1); break;
                case 5: MECDF_GKB(5, 1); break;
                default: MECDF_GKB(6, 1); break;
                }
            } else {
                switch (d) {
                case 1: MECDF_GKB(1, 2); break;
                case 2: MECDF_GKB(2, 3); break;
                case 3: MECDF_GKB(3, 4); break;
                case 4: MECDF_GKB(4, 5); break;
                case 5: MECDF_GKB(5, 6); break;
                default: MECDF_GKB(6, 7); break;
                }
            }
#undef MECDF_GKB
            MECDF_LAUNCH_CHECK();
        }
        {
            ProfScope prof("gridkde_scan", s);
            double *in = bufA, *outb = bufB;
            int64_t in_st = nA, out_st = nB;
            for (int a = 0; a < d; ++a) {
                GsBatch gb{};
                for (int j = 0; j < nb; ++j) {
                    GsArgs &ga = gb.a[j];
                    ga.in = in + (int64_t)j * in_st;
                    ga.out = outb + (int64_t)j * out_st;
                    ga.agg = agg + (int64_t)j * nagg;
                    ga.dec = dec + (int64_t)j * total + g.off[a];
                    ga.z = zn + g.off[a];
                    ga.span = span + (int64_t)j * nspan;
                    ga.ih = hs.h[j].ih[a];
                    ga.M = g.M[a];
                    ga.inner = g.nst[a];
                    ga.outer = g.nodes / (g.M[a] * g.nst[a]);
                    ga.nodes = g.nodes;
                    ga.nck = ceil_div(g.M[a], kGkL);
                    ga.nco = nch >> (a + 1);
                    ga.k = a;
                    ga.nt = NT;
                    ga.cols = (int64_t)ga.nco * CH * ga.outer * ga.inner;
                }
                const bool rows = gb.a[0].inner == 1 && gb.a[0].M <= 64 * kGsRowBlocks;
                if (matern && rows)
                    hipLaunchKernelGGL((k_gs_rows_mat<CH>),
                                       dim3((unsigned)ceil_div(gb.a[0].cols, 4), nb), dim3(256), 0,
                                       s, gb);
                else if (matern)
                    gs_launch<CH, true>(gb, nb, s);
                else if (rows)
                    hipLaunchKernelGGL((k_gs_rows<CH>),
                                       dim3((unsigned)ceil_div(gb.a[0].cols, 4), nb), dim3(256), 0,
                                       s, gb);
                else
                    gs_launch<CH, false>(gb, nb, s);
                MECDF_LAUNCH_CHECK();
                std::swap(in, outb);
                std::swap(in_st, out_st);
            }
            hipLaunchKernelGGL((k_gk_combine<CH, OutT>),
                               dim3((unsigned)ceil_div(g.nodes, 256), nb), dim3(256), 0, s, g, in,
                               in_st, matern, nm, out + (int64_t)b0 * g.nodes);
            MECDF_LAUNCH_CHECK();
        }
    }
    return MECDF_OK;
}

int gridkde_run(int d, int64_t N, const double *x, const void *w, const int64_t *M,
                const double *z, int nh, const double *h, void *out, int regression,
                int matern, int prec, hipStream_t s) {
    if (!regression) {
        if (prec == MECDF_F64)
            return gridkde_t<1, double, double>(d, N, x, (const double *)w, M, z, nh, h,
                                                (double *)out, matern, s);
        return gridkde_t<1, float, float>(d, N, x, (const float *)w, M, z, nh, h, (float *)out,
                                          matern, s);
    }
    if (prec == MECDF_F64)
        return gridkde_t<2, double, double>(d, N, x, (const double *)w, M, z, nh, h,
                                            (double *)out, matern, s);
    return gridkde_t<2, float, float>(d, N, x, (const float *)w, M, z, nh, h, (float *)out,
                                      matern, s);
}

}  // namespace mecdf
