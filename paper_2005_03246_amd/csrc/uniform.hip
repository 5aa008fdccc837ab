// The uniform-kernel density estimate of Section 3.2 (eq. (uniform_kde_nD))
// at arbitrary points, through its CDF decomposition eq.
// (uniform_decomposition_nD) in Langrene & Warin, arXiv 2005.03246: the
// weight of the points in the closed box [z - h, z + h] is the signed sum,
// over the 2^d sign patterns delta, of the generalized ECDF of eq.
// (ECDFdelta) at the corner z + delta h, with <= on the axes where delta_k =
// +1 and < where delta_k = -1.  The corner coordinates are rounded to
// doubles once (z_k + h_k and z_k - h_k), so the box is the one those
// rounded ends bound, and all corners of one bandwidth go through one run of
// the points recursion with per-query patterns.
//
//   k_uni_corners   the 2^d Q corner queries and their delta masks
//   recursion       eq. (ECDFdelta) at every corner (points.hip); at the
//                   sample points themselves (z is x) the corners' ranks come
//                   from the points' own ranks and no corner is formed here
//   k_uni_combine   the signed sum per point, times 1/(2^d N prod h): exact
//                   integer arithmetic for counts, float64 for weights
#include "common.hpp"

namespace mecdf {

int points_delta_run(int d, int64_t N, const double *x, const void *y, int64_t Q,
                     const double *z, const uint8_t *delta, void *F, int prec, hipStream_t s);
int points_corners_run(int d, int64_t N, const double *x, const void *y, const double *h,
                       void *F, int prec, hipStream_t s);

struct UniH {
    double h[MECDF_MAX_DIM];
};

// corner c of point q: query slot c*Q + q, bit k of c set for delta_k = -1
__global__ __launch_bounds__(256) void k_uni_corners(const double *__restrict__ z, int64_t Q,
                                                     int d, UniH hb, double *__restrict__ zc,
                                                     uint8_t *__restrict__ dl) {
    const int64_t nq = Q << d;
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= nq)
        return;
    const int c = (int)(t / Q);
    const int64_t q = t - (int64_t)c * Q;
    for (int k = 0; k < d; ++k) {
        const double v = z[(int64_t)k * Q + q];
        zc[(int64_t)k * nq + t] = ((c >> k) & 1) ? v - hb.h[k] : v + hb.h[k];
    }
    dl[t] = (uint8_t)c;
}

// f[q] = norm * sum_c (-1)^{|c|} G[c*Q + q], corners in order
template <typename GT, typename OutT>
__global__ __launch_bounds__(256) void k_uni_combine(const GT *__restrict__ G, int64_t Q, int d,
                                                     double norm, OutT *__restrict__ f) {
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= Q)
        return;
    GT acc = GT(0);
    for (int c = 0; c < (1 << d); ++c) {
        const GT v = G[(int64_t)c * Q + q];
        acc = (__builtin_popcount((unsigned)c) & 1) ? acc - v : acc + v;
    }
    f[q] = (OutT)((double)acc * norm);
}

__global__ __launch_bounds__(256) void k_uni_f64(const float *__restrict__ a, int64_t n,
                                                 double *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n)
        out[i] = (double)a[i];
}

int kde_uniform_run(int d, int64_t N, const double *x, const void *w, int64_t Q,
                    const double *z, int nh, const double *h, void *f, int prec,
                    hipStream_t s) {
    if (Q == 0)
        return MECDF_OK;
    const int64_t nq = Q << d;
    const bool weighted = w != nullptr;
    const bool at_points = z == x && Q == N;
    // working memory of one recursion over all corners (the weights go in as
    // float64: float32 weights are converted first)
    size_t inner = 0;
    set_workspace_sizing(&inner);
    const double hs[MECDF_MAX_DIM] = {1.0, 1.0, 1.0, 1.0, 1.0, 1.0};
    const void *ys = weighted ? (const void *)x : nullptr;
    const int rs = at_points ? points_corners_run(d, N, x, ys, hs, nullptr, MECDF_F64, s)
                             : points_delta_run(d, N, x, ys, nq, nullptr, nullptr, nullptr,
                                                MECDF_F64, s);
    set_workspace_sizing(nullptr);
    if (rs != kSizingOnly)
        return rs == MECDF_OK ? MECDF_EDEVICE : rs;
    const bool conv = weighted && prec != MECDF_F64;
    ArenaPlan pl;
    if (!at_points) {
        pl.add<double>((size_t)nq * d);  // corner coordinates
        pl.add<uint8_t>((size_t)nq);     // corner masks
    }
    pl.add<int64_t>((size_t)nq);      // corner ECDFs (int64 counts or doubles)
    if (conv)
        pl.add<double>((size_t)N);    // float64 weights
    const size_t mine = (pl.used + 255) & ~size_t(255);
    void *wsb = nullptr;
    MECDF_TRY(workspace_reserve(mine + inner, &wsb));
    Arena ar;
    ar.base = (char *)wsb;
    double *zc = at_points ? nullptr : ar.take<double>((size_t)nq * d);
    uint8_t *dl = at_points ? nullptr : ar.take<uint8_t>((size_t)nq);
    void *G = ar.take<int64_t>((size_t)nq);
    double *wd = conv ? ar.take<double>((size_t)N) : nullptr;
    FixedWorkspace fixed((char *)wsb + mine, inner);
    const void *wv = w;
    if (conv) {
        hipLaunchKernelGGL(k_uni_f64, dim3((unsigned)ceil_div(N, 256)), dim3(256), 0, s,
                           (const float *)w, N, wd);
        MECDF_LAUNCH_CHECK();
        wv = wd;
    }
    const size_t osz = prec == MECDF_F64 ? sizeof(double) : sizeof(float);
    for (int b = 0; b < nh; ++b) {
        UniH hb{};
        double prod = 1.0;
        for (int k = 0; k < d; ++k) {
            hb.h[k] = h[(size_t)b * d + k];
            prod *= hb.h[k];
        }
        if (at_points) {
            MECDF_TRY(points_corners_run(d, N, x, wv, hb.h, G, MECDF_F64, s));
        } else {
            {
                ProfScope prof("uniform_corners", s);
                hipLaunchKernelGGL(k_uni_corners, dim3((unsigned)ceil_div(nq, 256)), dim3(256), 0,
                                   s, z, Q, d, hb, zc, dl);
                MECDF_LAUNCH_CHECK();
            }
            MECDF_TRY(points_delta_run(d, N, x, wv, nq, zc, dl, G, MECDF_F64, s));
        }
        // counts come back raw, weighted sums as F_N (already over N)
        const double norm = 1.0 / ((double)(1 << d) * prod * (weighted ? 1.0 : (double)N));
        void *fb = (char *)f + (size_t)b * Q * osz;
        const unsigned nb = (unsigned)ceil_div(Q, 256);
        ProfScope prof("uniform_combine", s);
        if (!weighted && prec == MECDF_F64)
            hipLaunchKernelGGL((k_uni_combine<int64_t, double>), dim3(nb), dim3(256), 0, s,
                               (const int64_t *)G, Q, d, norm, (double *)fb);
        else if (!weighted)
            hipLaunchKernelGGL((k_uni_combine<int64_t, float>), dim3(nb), dim3(256), 0, s,
                               (const int64_t *)G, Q, d, norm, (float *)fb);
        else if (prec == MECDF_F64)
            hipLaunchKernelGGL((k_uni_combine<double, double>), dim3(nb), dim3(256), 0, s,
                               (const double *)G, Q, d, norm, (double *)fb);
        else
            hipLaunchKernelGGL((k_uni_combine<double, float>), dim3(nb), dim3(256), 0, s,
                               (const double *)G, Q, d, norm, (float *)fb);
        MECDF_LAUNCH_CHECK();
    }
    return MECDF_OK;
}

}  // namespace mecdf
