// Laplacian kernel sums at the nodes of a rectilinear grid: the "fast
// summation" kernel density estimate and Nadaraya-Watson regression of
// Section 3 (eq. (Laplacian_kde_nD) evaluated through the decomposition of
// eq. (Laplacian_decomposition_nD) on the grid of Section 2.1), in Langrene &
// Warin, arXiv 2005.03246.
//
// Along one axis, a point x in cell c (z_{c-1} < x <= z_c) reaches the nodes
// j >= c through exp(-(z_j - x)/h) = exp(-(z_j - z_c)/h) exp(-(z_c - x)/h)
// and the nodes j <= c-1 through exp(-(x - z_{c-1})/h) = exp(-(z_{c-1} -
// z_j)/h) exp(-(x - z_{c-1})/h).  So each point puts, for every choice delta
// in {up, down}^d, the weight w prod_k (its factor to the cell's upper or
// lower node on axis k) into the bin of that corner node, and each of the
// 2^d bin arrays is scanned along every axis with the decays between
// neighbouring nodes: forward where delta_k = up, backward where down.  The
// estimate at a node is the sum of the 2^d scanned arrays.  Every factor is
// at most 1: nothing overflows.
//
//   k_gk_keys      the cell of every point (exact comparisons with the nodes),
//                  one linear key per cell; points with a NaN coordinate are
//                  left out
//   radix sort     stable, so each cell's points are contiguous, in input order
//   k_gk_bins      per cell, one thread adds its points' corner weights in
//                  input order (float64, Neumaier) and writes one bin per
//                  channel: no two cells share a bin of one channel
//   k_gk_scan      the decayed prefix / suffix of one channel along one axis,
//                  one thread per line, coalesced over the trailing axes
//   k_gk_combine   the 2^d channels summed at each node, times the
//                  normalisation (density) or as a ratio (regression)
#include <vector>

#include "common.hpp"
#include "radix.hpp"

namespace mecdf {

struct GkGrid {
    int d;
    int64_t M[MECDF_MAX_DIM];      // nodes per axis
    int64_t off[MECDF_MAX_DIM];    // first node of each axis in the node array
    int64_t C[MECDF_MAX_DIM];      // cells per axis (M + 1)
    int64_t cst[MECDF_MAX_DIM];    // cell-key strides (C order)
    int64_t nst[MECDF_MAX_DIM];    // node-array strides (C order)
    int64_t nodes;                 // prod M
};

struct GkH {
    double ih[MECDF_MAX_DIM];  // 1/h per axis
};

// cell c = #{nodes < x} on each axis; key = C-order index of the cell vector
__global__ __launch_bounds__(256) void k_gk_keys(GkGrid g, const double *__restrict__ zn,
                                                 const double *__restrict__ x, int64_t n,
                                                 uint32_t dropped, uint32_t *__restrict__ key,
                                                 uint32_t *__restrict__ idx) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n)
        return;
    int64_t k = 0;
    bool nan = false;
    for (int a = 0; a < g.d; ++a) {
        const double v = x[(int64_t)a * n + i];
        nan = nan || v != v;
        const double *z = zn + g.off[a];
        int64_t lo = 0, hi = g.M[a];  // count of nodes < v in [lo, hi]
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (z[mid] < v)
                lo = mid + 1;
            else
                hi = mid;
        }
        k += lo * g.cst[a];
    }
    key[i] = nan ? dropped : (uint32_t)k;
    idx[i] = (uint32_t)i;
}

// One thread per sorted position that starts a run of equal keys: the run's
// points (input order) give, for each channel delta (bit a set: the point's
// upper node on axis a; clear: its lower node), the sum of
// w_i prod_a (factor of point i to that node), written to the channel's bin
// at the corner node; corners outside the node range are skipped.
// CH = 1: weights w (or 1); CH = 2: channel pairs (1, y).
template <int D, int CH, typename WT>
__global__ __launch_bounds__(256) void k_gk_bins(GkGrid g, const double *__restrict__ zn,
                                                 const double *__restrict__ x, int64_t n,
                                                 uint32_t dropped,
                                                 const uint32_t *__restrict__ key,
                                                 const uint32_t *__restrict__ idx,
                                                 const WT *__restrict__ w, GkH hb,
                                                 double *__restrict__ bins) {
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= n)
        return;
    const uint32_t kk = key[p];
    if (kk == dropped || (p > 0 && key[p - 1] == kk))
        return;
    // the cell vector of this run
    int64_t c[D];
    int64_t rem = kk;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        c[a] = rem / g.cst[a];
        rem -= c[a] * g.cst[a];
    }
    constexpr int nch = 1 << D;
    // Neumaier pairs per channel and value
    double s[nch][CH], e[nch][CH];
#pragma unroll
    for (int q = 0; q < nch; ++q)
#pragma unroll
        for (int v = 0; v < CH; ++v)
            s[q][v] = e[q][v] = 0.0;
    for (int64_t r = p; r < n && key[r] == kk; ++r) {
        const int64_t i = idx[r];
        double up[D], dn[D];
#pragma unroll
        for (int a = 0; a < D; ++a) {
            const double v = x[(int64_t)a * n + i];
            const double *z = zn + g.off[a];
            up[a] = c[a] < g.M[a] ? exp(-(z[c[a]] - v) * hb.ih[a]) : 0.0;
            dn[a] = c[a] > 0 ? exp(-(v - z[c[a] - 1]) * hb.ih[a]) : 0.0;
        }
        double wv[CH];
        if (CH == 1) {
            wv[0] = w ? (double)w[i] : 1.0;
        } else {
            wv[0] = 1.0;
            wv[CH - 1] = (double)w[i];
        }
#pragma unroll
        for (int q = 0; q < nch; ++q) {
            double f = 1.0;
#pragma unroll
            for (int a = 0; a < D; ++a)
                f *= ((q >> a) & 1) ? up[a] : dn[a];
#pragma unroll
            for (int v = 0; v < CH; ++v) {
                const double t = f * wv[v];
                const double u = s[q][v] + t;
                e[q][v] += fabs(s[q][v]) >= fabs(t) ? (s[q][v] - u) + t : (t - u) + s[q][v];
                s[q][v] = u;
            }
        }
    }
#pragma unroll
    for (int q = 0; q < nch; ++q) {
        int64_t node = 0;
        bool inside = true;
#pragma unroll
        for (int a = 0; a < D; ++a) {
            const int64_t j = ((q >> a) & 1) ? c[a] : c[a] - 1;
            inside = inside && j >= 0 && j < g.M[a];
            node += j * g.nst[a];
        }
        if (!inside)
            continue;
#pragma unroll
        for (int v = 0; v < CH; ++v)
            bins[((int64_t)q * CH + v) * g.nodes + node] = s[q][v] + e[q][v];
    }
}

__global__ void k_gk_zero(double *a, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n)
        a[i] = 0.0;
}

// decays between neighbouring nodes: dec[off_a + j] = exp(-(z_j - z_{j-1}) ih_a), j >= 1
__global__ void k_gk_decays(GkGrid g, const double *__restrict__ zn, GkH hb, int64_t total,
                            double *__restrict__ dec) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= total)
        return;
    int a = 0;
    while (a + 1 < g.d && t >= g.off[a + 1])
        ++a;
    const int64_t j = t - g.off[a];
    dec[t] = j == 0 ? 0.0 : exp(-(zn[t] - zn[t - 1]) * hb.ih[a]);
}

// Decayed scan of each array of the batch (count arrays of g.nodes values)
// along axis a: forward S_j = dec_j S_{j-1} + B_j (dir 0) or backward
// S_j = dec_{j+1} S_{j+1} + B_j (dir 1), in place.  Thread per line.
__global__ __launch_bounds__(256) void k_gk_scan(GkGrid g, int a, int dir,
                                                 const double *__restrict__ dec,
                                                 double *__restrict__ arr, int count) {
    const int64_t lines = g.nodes / g.M[a];
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= lines * count)
        return;
    const int which = (int)(t / lines);
    const int64_t l = t - (int64_t)which * lines;
    // l enumerates the other axes in C order: split around axis a
    const int64_t inner = g.nst[a];  // product of the sizes after axis a
    const int64_t outer_i = l / inner, inner_i = l - outer_i * inner;
    double *col = arr + (int64_t)which * g.nodes + outer_i * inner * g.M[a] + inner_i;
    const double *dz = dec + g.off[a];
    const int64_t M = g.M[a];
    double run = 0.0;
    if (dir == 0) {
        for (int64_t j = 0; j < M; ++j) {
            run = dz[j] * run + col[j * inner];
            col[j * inner] = run;
        }
    } else {
        for (int64_t j = M - 1; j >= 0; --j) {
            run = (j + 1 < M ? dz[j + 1] : 0.0) * run + col[j * inner];
            col[j * inner] = run;
        }
    }
}

// out[node] = norm * sum of the 2^d channels (CH = 1), or the ratio of the
// summed second to the summed first values (CH = 2), channels in order
template <int CH, typename OutT>
__global__ __launch_bounds__(256) void k_gk_combine(GkGrid g, const double *__restrict__ bins,
                                                    double norm, OutT *__restrict__ out) {
    const int64_t node = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (node >= g.nodes)
        return;
    const int nch = 1 << g.d;
    double s[CH];
    for (int v = 0; v < CH; ++v)
        s[v] = 0.0;
    for (int q = 0; q < nch; ++q)
        for (int v = 0; v < CH; ++v)
            s[v] += bins[((int64_t)q * CH + v) * g.nodes + node];
    out[node] = CH == 1 ? (OutT)(s[0] * norm) : (OutT)(s[CH - 1] / s[0]);
}

template <int CH, typename WT, typename OutT>
static int gridkde_t(int d, int64_t N, const double *x, const WT *w, const int64_t *M,
                     const double *z, int nh, const double *h, OutT *out, hipStream_t s) {
    GkGrid g{};
    g.d = d;
    int64_t total = 0;
    for (int a = 0; a < d; ++a) {
        g.M[a] = M[a];
        g.C[a] = M[a] + 1;
        g.off[a] = total;
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
    const int nch = 1 << d;
    const int64_t nbins = (int64_t)nch * CH * g.nodes;
    ArenaPlan pl;
    pl.add<double>((size_t)total);          // nodes
    pl.add<double>((size_t)total);          // decays
    for (int q = 0; q < 3; ++q)
        pl.add<uint32_t>((size_t)N);        // keys
    for (int q = 0; q < 3; ++q)
        pl.add<uint32_t>((size_t)N);        // point indices
    pl.add<double>((size_t)nbins);
    radix_plan(pl, N);
    void *wsb = nullptr;
    MECDF_TRY(workspace_reserve(pl.used, &wsb));
    Arena ar;
    ar.base = (char *)wsb;
    double *zn = ar.take<double>((size_t)total);
    double *dec = ar.take<double>((size_t)total);
    uint32_t *k0 = ar.take<uint32_t>((size_t)N), *k1 = ar.take<uint32_t>((size_t)N),
             *k2 = ar.take<uint32_t>((size_t)N);
    uint32_t *i0 = ar.take<uint32_t>((size_t)N), *i1 = ar.take<uint32_t>((size_t)N),
             *i2 = ar.take<uint32_t>((size_t)N);
    double *bins = ar.take<double>((size_t)nbins);
    RadixScratch rs = radix_take(ar, N);
    MECDF_TRY(upload_small(z, sizeof(double) * (size_t)total, zn, s));
    const unsigned nbN = (unsigned)ceil_div(N, 256);
    const uint32_t *ks = k0, *is = i0;
    // cell keys 0 .. cells-1, the value `cells` for points left out
    const uint32_t dropped = (uint32_t)cs;
    const int kbits = bits_for((uint64_t)cs);
    {
        ProfScope prof("gridkde_sort", s);
        hipLaunchKernelGGL(k_gk_keys, dim3(nbN), dim3(256), 0, s, g, zn, x, N, dropped, k0, i0);
        int which = 0;
        MECDF_TRY((radix_sort_bits<uint32_t, uint32_t>(k0, i0, k1, i1, k2, i2, N, 0, kbits, rs,
                                                       s, &which)));
        ks = which == 1 ? k1 : (which == 2 ? k2 : k0);
        is = which == 1 ? i1 : (which == 2 ? i2 : i0);
        MECDF_LAUNCH_CHECK();
    }
    for (int b = 0; b < nh; ++b) {
        GkH hb{};
        double prod = 1.0;
        for (int a = 0; a < d; ++a) {
            hb.ih[a] = 1.0 / h[(size_t)b * d + a];
            prod *= h[(size_t)b * d + a];
        }
        ProfScope prof("gridkde_bandwidth", s);
        hipLaunchKernelGGL(k_gk_zero, dim3((unsigned)ceil_div(nbins, 256)), dim3(256), 0, s,
                           bins, nbins);
        hipLaunchKernelGGL(k_gk_decays, dim3((unsigned)ceil_div(total, 256)), dim3(256), 0, s, g,
                           zn, hb, total, dec);
        switch (d) {
#define MECDF_GKB(D)                                                                           \
    hipLaunchKernelGGL((k_gk_bins<D, CH, WT>), dim3(nbN), dim3(256), 0, s, g, zn, x, N, dropped, \
                       ks, is, w, hb, bins)
        case 1: MECDF_GKB(1); break;
        case 2: MECDF_GKB(2); break;
        case 3: MECDF_GKB(3); break;
        case 4: MECDF_GKB(4); break;
        case 5: MECDF_GKB(5); break;
        default: MECDF_GKB(6); break;
#undef MECDF_GKB
        }
        // every channel along every axis, forward where the channel takes the
        // upper node on that axis
        for (int q = 0; q < nch; ++q)
            for (int a = 0; a < d; ++a) {
                const int64_t lines = g.nodes / g.M[a];
                hipLaunchKernelGGL(k_gk_scan, dim3((unsigned)ceil_div(lines * CH, 256)),
                                   dim3(256), 0, s, g, a, ((q >> a) & 1) ? 0 : 1, dec,
                                   bins + (int64_t)q * CH * g.nodes, CH);
            }
        const double norm = 1.0 / ((double)nch * (double)N * prod);
        hipLaunchKernelGGL((k_gk_combine<CH, OutT>), dim3((unsigned)ceil_div(g.nodes, 256)),
                           dim3(256), 0, s, g, bins, norm, out + (int64_t)b * g.nodes);
        MECDF_LAUNCH_CHECK();
    }
    return MECDF_OK;
}

int gridkde_run(int d, int64_t N, const double *x, const void *w, const int64_t *M,
                const double *z, int nh, const double *h, void *out, int regression, int prec,
                hipStream_t s) {
    if (!regression) {
        if (prec == MECDF_F64)
            return gridkde_t<1, double, double>(d, N, x, (const double *)w, M, z, nh, h,
                                                (double *)out, s);
        return gridkde_t<1, float, float>(d, N, x, (const float *)w, M, z, nh, h, (float *)out,
                                          s);
    }
    if (prec == MECDF_F64)
        return gridkde_t<2, double, double>(d, N, x, (const double *)w, M, z, nh, h,
                                            (double *)out, s);
    return gridkde_t<2, float, float>(d, N, x, (const float *)w, M, z, nh, h, (float *)out, s);
}

}  // namespace mecdf
