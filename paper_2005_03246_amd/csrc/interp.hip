// Grid values at arbitrary points by multilinear interpolation: the step
// that turns the grid path's ECDF (or grid-mode kernel sums) into values at
// the sample points (Section 4.1 and 4.2 of Langrene & Warin, arXiv
// 2005.03246, study the error of exactly this against the divide-and-conquer
// values at the points).
//
// One thread per query point.  Along each axis the query's interval
// [z_j, z_{j+1}] is found by binary search of the nodes (staged in LDS when
// they fit) and the weight t = (q - z_j) / (z_{j+1} - z_j); a query outside
// the nodes is clamped to the nearest end node, an axis with one node is
// constant.  The 2^d corner values are combined in a fixed order.
#include "common.hpp"

namespace mecdf {

constexpr int kInterpLdsNodes = 8192;

struct InterpInfo {
    int d;
    int64_t M[MECDF_MAX_DIM];
    int64_t off[MECDF_MAX_DIM];     // first node of each axis in the node array
    int64_t stride[MECDF_MAX_DIM];  // C-order strides of the value array
};

template <typename VT>
__global__ __launch_bounds__(256) void k_interp(InterpInfo g, const double *__restrict__ nodes,
                                                int64_t total_nodes, const VT *__restrict__ G,
                                                int64_t Q, const double *__restrict__ q,
                                                VT *__restrict__ out) {
    __shared__ double sn[kInterpLdsNodes];
    const bool lds = total_nodes <= kInterpLdsNodes;
    if (lds) {
        for (int64_t i = threadIdx.x; i < total_nodes; i += 256)
            sn[i] = nodes[i];
        __syncthreads();
    }
    const double *zn = lds ? sn : nodes;
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= Q)
        return;
    int64_t j[MECDF_MAX_DIM];
    double t[MECDF_MAX_DIM];
    bool nan = false;
#pragma unroll
    for (int k = 0; k < MECDF_MAX_DIM; ++k) {
        j[k] = 0;
        t[k] = 0.0;
        if (k >= g.d)
            continue;
        const double v = q[(int64_t)k * Q + p];
        const double *z = zn + g.off[k];
        const int64_t M = g.M[k];
        if (v != v) {
            nan = true;
        } else if (M == 1 || v <= z[0]) {
            j[k] = 0;
            t[k] = 0.0;
        } else if (v >= z[M - 1]) {
            j[k] = M - 2;
            t[k] = 1.0;
        } else {
            // the last node <= v (z[0] < v < z[M-1])
            int64_t lo = 0, hi = M - 1;
            while (hi - lo > 1) {
                const int64_t mid = (lo + hi) >> 1;
                if (z[mid] <= v)
                    lo = mid;
                else
                    hi = mid;
            }
            j[k] = lo;
            t[k] = (v - z[lo]) / (z[lo + 1] - z[lo]);
        }
    }
    if (nan) {
        out[p] = (VT)__builtin_nan("");
        return;
    }
    int64_t base = 0;
    for (int k = 0; k < g.d; ++k)
        base += j[k] * g.stride[k];
    // corners in the order of their bit patterns (bit k: upper node on axis k)
    double acc = 0.0;
    const int nc = 1 << g.d;
    for (int c = 0; c < nc; ++c) {
        double wgt = 1.0;
        int64_t idx = base;
        for (int k = 0; k < g.d; ++k) {
            const bool up = (c >> k) & 1;
            const bool single = g.M[k] == 1;
            wgt *= up ? t[k] : 1.0 - t[k];
            if (up && !single)
                idx += g.stride[k];
        }
        if (wgt != 0.0)
            acc += wgt * (double)G[idx];
    }
    out[p] = (VT)acc;
}

int grid_interp(int d, const int64_t *M, const double *z, const void *G, int64_t Q,
                const double *q, void *out, int prec, hipStream_t s) {
    InterpInfo g{};
    g.d = d;
    int64_t total = 0;
    for (int k = 0; k < d; ++k) {
        g.M[k] = M[k];
        g.off[k] = total;
        total += M[k];
    }
    int64_t st = 1;
    for (int k = d - 1; k >= 0; --k) {
        g.stride[k] = st;
        st *= M[k];
    }
    void *wsb = nullptr;
    MECDF_TRY(workspace_reserve(sizeof(double) * (size_t)total, &wsb));
    MECDF_TRY(upload_small(z, sizeof(double) * (size_t)total, wsb, s));
    if (Q == 0)
        return MECDF_OK;
    ProfScope prof("grid_interp", s);
    const unsigned nb = (unsigned)ceil_div(Q, 256);
    if (prec == MECDF_F64)
        hipLaunchKernelGGL(k_interp<double>, dim3(nb), dim3(256), 0, s, g, (const double *)wsb,
                           total, (const double *)G, Q, q, (double *)out);
    else
        hipLaunchKernelGGL(k_interp<float>, dim3(nb), dim3(256), 0, s, g, (const double *)wsb,
                           total, (const float *)G, Q, q, (float *)out);
    MECDF_LAUNCH_CHECK();
    return MECDF_OK;
}

}  // namespace mecdf
