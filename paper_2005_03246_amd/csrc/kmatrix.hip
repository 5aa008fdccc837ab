// Two uses of the Laplacian kernel sums beyond a diagonal bandwidth and a
// local constant fit (Langrene & Warin, arXiv 2005.03246):
//
// * General matrix bandwidth (Appendix B, eq. (kde_nD_H)): with the
//   eigendecomposition H = R Delta^2 R^T, the estimator is the diagonal-
//   bandwidth one (eq. (kde_nD)) in the coordinates R^T x with h = diag(Delta):
//   the points are rotated on the device and the kernel sums run unchanged.
//
// * Local-linear regression: the weighted least-squares fit of
//   y ~ a + b^T (x - x_j) with weights K(x_i - x_j) at every sample point;
//   its moments sum_i K (x_i - x_j)^p (y_i) are expanded into kernel sums with
//   the weights 1, x_l, x_l x_m, y and y x_l (the paper's moment weights for
//   local polynomial fits), each one call of the kernel-sum path, and a
//   (d+1) x (d+1) system is solved per point.
#include <cmath>
#include <vector>

#include "common.hpp"

namespace mecdf {

int kde_run(int d, int64_t N, const double *x, const void *w, int nh, const double *h,
            void *f, double *score, int regression, int prec, hipStream_t s);

// ------------------------------------------------------------ eigenvectors
// Cyclic Jacobi rotations on a symmetric d x d matrix (row-major): on return
// the diagonal of A holds the eigenvalues and the columns of V the
// eigenvectors.  Returns false when the sweeps do not converge.
static bool jacobi_eigen(int d, std::vector<double> &A, std::vector<double> &V) {
    V.assign((size_t)d * d, 0.0);
    for (int i = 0; i < d; ++i)
        V[(size_t)i * d + i] = 1.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, diag = 0.0;
        for (int i = 0; i < d; ++i)
            for (int j = 0; j < d; ++j)
                (i == j ? diag : off) += A[(size_t)i * d + j] * A[(size_t)i * d + j];
        if (off <= 1e-28 * diag)  // off-diagonal mass below 1e-14 of the diagonal
            return true;
        for (int p = 0; p < d; ++p)
            for (int q = p + 1; q < d; ++q) {
                const double apq = A[(size_t)p * d + q];
                if (apq == 0.0)
                    continue;
                const double app = A[(size_t)p * d + p], aqq = A[(size_t)q * d + q];
                const double theta = (aqq - app) / (2.0 * apq);
                const double t = (theta >= 0 ? 1.0 : -1.0) /
                                 (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), sn = t * c;
                for (int k = 0; k < d; ++k) {  // A <- A J
                    const double akp = A[(size_t)k * d + p], akq = A[(size_t)k * d + q];
                    A[(size_t)k * d + p] = c * akp - sn * akq;
                    A[(size_t)k * d + q] = sn * akp + c * akq;
                }
                for (int k = 0; k < d; ++k) {  // A <- J^T A
                    const double apk = A[(size_t)p * d + k], aqk = A[(size_t)q * d + k];
                    A[(size_t)p * d + k] = c * apk - sn * aqk;
                    A[(size_t)q * d + k] = sn * apk + c * aqk;
                }
                for (int k = 0; k < d; ++k) {  // V <- V J
                    const double vkp = V[(size_t)k * d + p], vkq = V[(size_t)k * d + q];
                    V[(size_t)k * d + p] = c * vkp - sn * vkq;
                    V[(size_t)k * d + q] = sn * vkp + c * vkq;
                }
            }
    }
    return false;
}

struct Rot {
    double r[MECDF_MAX_DIM][MECDF_MAX_DIM];  // x'_k = sum_l r[k][l] x_l  (R^T)
};

__global__ __launch_bounds__(256) void k_rotate(const double *__restrict__ x, int d, int64_t n,
                                                Rot R, double *__restrict__ xr) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n)
        return;
    double v[MECDF_MAX_DIM];
    for (int l = 0; l < d; ++l)
        v[l] = x[(int64_t)l * n + i];
    for (int k = 0; k < d; ++k) {
        double s = 0.0;
        for (int l = 0; l < d; ++l)
            s += R.r[k][l] * v[l];
        xr[(int64_t)k * n + i] = s;
    }
}

// The rotation R^T and the diagonal bandwidth sqrt(eigenvalues) of H
// (row-major, symmetric positive definite); MECDF_EINVAL otherwise.
// A matrix whose two triangles differ by more than 1e-12 of its largest entry
// is refused; otherwise its symmetric part is used.
static int matrix_bandwidth(int d, const double *H, Rot &R, double *h) {
    std::vector<double> A((size_t)d * d), V;
    double amax = 0.0;
    for (int i = 0; i < d * d; ++i) {
        if (!std::isfinite(H[i]))
            return MECDF_EINVAL;
        amax = std::fmax(amax, std::fabs(H[i]));
    }
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) {
            const double a = H[(size_t)i * d + j], b = H[(size_t)j * d + i];
            if (std::fabs(a - b) > 1e-12 * amax)
                return MECDF_EINVAL;
            A[(size_t)i * d + j] = 0.5 * (a + b);
        }
    if (!jacobi_eigen(d, A, V))
        return MECDF_EINVAL;
    for (int k = 0; k < d; ++k) {
        const double ev = A[(size_t)k * d + k];
        if (!(ev > 0.0))
            return MECDF_EINVAL;
        h[k] = std::sqrt(ev);
        for (int l = 0; l < d; ++l)
            R.r[k][l] = V[(size_t)l * d + k];
    }
    return MECDF_OK;
}

// Kernel sums with matrix bandwidths H[b] (one call of the kernel-sum path
// per bandwidth, in the rotated coordinates).  The rotated points sit at the
// start of the working memory; the kernel sums get the rest.
int kde_matrix_run(int d, int64_t N, const double *x, const void *w, int nh, const double *H,
                   void *f, double *score, int regression, int prec, hipStream_t s) {
    std::vector<Rot> rots((size_t)nh);
    std::vector<double> hd((size_t)nh * d);
    for (int b = 0; b < nh; ++b)
        if (matrix_bandwidth(d, H + (size_t)b * d * d, rots[b], hd.data() + (size_t)b * d) !=
            MECDF_OK) {
            set_error("bandwidth matrices must be symmetric positive definite");
            return MECDF_EINVAL;
        }
    size_t inner = 0;
    set_workspace_sizing(&inner);
    const int rs = kde_run(d, N, x, w, 1, hd.data(), f, score, regression, prec, s);
    set_workspace_sizing(nullptr);
    if (rs != kSizingOnly)
        return rs == MECDF_OK ? MECDF_EDEVICE : rs;
    const size_t xb = (((size_t)d * N * sizeof(double)) + 255) & ~size_t(255);
    void *wsb = nullptr;
    MECDF_TRY(workspace_reserve(xb + inner, &wsb));
    double *xr = (double *)wsb;
    FixedWorkspace fixed((char *)wsb + xb, inner);
    const size_t osz = prec == MECDF_F64 ? sizeof(double) : sizeof(float);
    for (int b = 0; b < nh; ++b) {
        hipLaunchKernelGGL(k_rotate, dim3((unsigned)ceil_div(N, 256)), dim3(256), 0, s, x, d, N,
                           rots[b], xr);
        MECDF_LAUNCH_CHECK();
        MECDF_TRY(kde_run(d, N, xr, w, 1, hd.data() + (size_t)b * d,
                          f ? (void *)((char *)f + (size_t)b * N * osz) : nullptr,
                          score ? score + b : nullptr, regression, prec, s));
    }
    return MECDF_OK;
}

// ------------------------------------------------------------ local linear
template <typename YT>
__global__ void k_to_f64(const YT *__restrict__ a, int64_t n, double *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n)
        out[i] = (double)a[i];
}

// weights of the moment sums: column c (stride ld) of the array
//   0: 1   1..d: x_l   then x_l x_m (l <= m)   then y   then y x_l
__global__ __launch_bounds__(256) void k_moment_weights(const double *__restrict__ x, int d,
                                                        int64_t n, const double *__restrict__ y,
                                                        double *__restrict__ W, int64_t ld) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n)
        return;
    double v[MECDF_MAX_DIM];
    for (int l = 0; l < d; ++l)
        v[l] = x[(int64_t)l * n + i];
    const double yi = y[i];
    int c = 0;
    W[(int64_t)c++ * ld + i] = 1.0;
    for (int l = 0; l < d; ++l)
        W[(int64_t)c++ * ld + i] = v[l];
    for (int l = 0; l < d; ++l)
        for (int m = l; m < d; ++m)
            W[(int64_t)c++ * ld + i] = v[l] * v[m];
    W[(int64_t)c++ * ld + i] = yi;
    for (int l = 0; l < d; ++l)
        W[(int64_t)c++ * ld + i] = yi * v[l];
}

// Per point j: the moments about x_j from the sums, the (d+1)^2 system of the
// local-linear fit, solved by Gaussian elimination with partial pivoting; the
// intercept is the estimate.  A pivot below 1e-10 of the largest diagonal
// entry (only the point itself, or points on a lower-dimensional set, carry
// weight) gives the local constant (Nadaraya-Watson) estimate instead.
template <typename OutT>
__global__ __launch_bounds__(256) void k_loclin_solve(const double *__restrict__ x, int d,
                                                      int64_t n, const double *__restrict__ S,
                                                      int64_t ld, OutT *__restrict__ out) {
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= n)
        return;
    double xj[MECDF_MAX_DIM];
    for (int l = 0; l < d; ++l)
        xj[l] = x[(int64_t)l * n + j];
    auto sum = [&](int c) { return S[(int64_t)c * ld + j]; };
    const int c1 = 1, c2 = 1 + d, cy = c2 + d * (d + 1) / 2, cy1 = cy + 1;
    const double s0 = sum(0);
    double s1[MECDF_MAX_DIM], t1[MECDF_MAX_DIM];
    double A[MECDF_MAX_DIM + 1][MECDF_MAX_DIM + 2];
    const double t0 = sum(cy);
    for (int l = 0; l < d; ++l) {
        s1[l] = sum(c1 + l) - xj[l] * s0;
        t1[l] = sum(cy1 + l) - xj[l] * t0;
    }
    A[0][0] = s0;
    A[0][d + 1] = t0;
    for (int l = 0; l < d; ++l) {
        A[0][l + 1] = s1[l];
        A[l + 1][0] = s1[l];
        A[l + 1][d + 1] = t1[l];
    }
    int c = c2;
    for (int l = 0; l < d; ++l)
        for (int m = l; m < d; ++m, ++c) {
            const double v = sum(c) - xj[l] * sum(c1 + m) - xj[m] * sum(c1 + l) +
                             xj[l] * xj[m] * s0;
            A[l + 1][m + 1] = v;
            A[m + 1][l + 1] = v;
        }
    const int k = d + 1;
    double dmax = 0.0;
    for (int r = 0; r < k; ++r)
        dmax = fmax(dmax, fabs(A[r][r]));
    bool ok = dmax > 0.0;
    for (int col = 0; col < k && ok; ++col) {
        int piv = col;
        for (int r = col + 1; r < k; ++r)
            if (fabs(A[r][col]) > fabs(A[piv][col]))
                piv = r;
        if (!(fabs(A[piv][col]) > 1e-10 * dmax)) {
            ok = false;
            break;
        }
        if (piv != col)
            for (int q = 0; q <= k; ++q) {
                const double t = A[col][q];
                A[col][q] = A[piv][q];
                A[piv][q] = t;
            }
        for (int r = col + 1; r < k; ++r) {
            const double fct = A[r][col] / A[col][col];
            for (int q = col; q <= k; ++q)
                A[r][q] -= fct * A[col][q];
        }
    }
    double est;
    if (ok) {
        double sol[MECDF_MAX_DIM + 1];
        for (int r = k - 1; r >= 0; --r) {
            double v = A[r][k];
            for (int q = r + 1; q < k; ++q)
                v -= A[r][q] * sol[q];
            sol[r] = v / A[r][r];
        }
        est = sol[0];
    } else {
        est = t0 / s0;
    }
    out[j] = (OutT)est;
}

template <typename YT, typename OutT>
static int loclin_t(int d, int64_t N, const double *x, const YT *y, int nh, const double *h,
                    OutT *m, hipStream_t s) {
    const int nmom = 1 + d + d * (d + 1) / 2 + 1 + d;
    size_t inner = 0;
    set_workspace_sizing(&inner);
    const int rs = kde_run(d, N, x, nullptr, nh, h, m, nullptr, 0, MECDF_F64, s);
    set_workspace_sizing(nullptr);
    if (rs != kSizingOnly)
        return rs == MECDF_OK ? MECDF_EDEVICE : rs;
    const size_t colb = (((size_t)N * sizeof(double)) + 255) & ~size_t(255);
    const int64_t ld = (int64_t)(colb / sizeof(double));  // column stride
    void *wsb = nullptr;
    // the float64 response, the moment weights, the sums of one bandwidth
    MECDF_TRY(workspace_reserve(colb + 2 * colb * nmom + inner, &wsb));
    double *yd = (double *)wsb;
    double *W = (double *)((char *)wsb + colb);
    double *S = (double *)((char *)wsb + colb + colb * nmom);
    FixedWorkspace fixed((char *)wsb + colb + 2 * colb * nmom, inner);
    const unsigned nb = (unsigned)ceil_div(N, 256);
    hipLaunchKernelGGL(k_to_f64<YT>, dim3(nb), dim3(256), 0, s, y, N, yd);
    hipLaunchKernelGGL(k_moment_weights, dim3(nb), dim3(256), 0, s, x, d, N, yd, W, ld);
    MECDF_LAUNCH_CHECK();
    for (int b = 0; b < nh; ++b) {
        for (int c = 0; c < nmom; ++c)
            MECDF_TRY(kde_run(d, N, x, W + (size_t)c * ld, 1, h + (size_t)b * d,
                              S + (size_t)c * ld, nullptr, 0, MECDF_F64, s));
        hipLaunchKernelGGL(k_loclin_solve<OutT>, dim3(nb), dim3(256), 0, s, x, d, N, S, ld,
                           m + (size_t)b * N);
        MECDF_LAUNCH_CHECK();
    }
    return MECDF_OK;
}

int loclin_run(int d, int64_t N, const double *x, const void *y, int nh, const double *h,
               void *m, int prec, hipStream_t s) {
    if (prec == MECDF_F64)
        return loclin_t<double, double>(d, N, x, (const double *)y, nh, h, (double *)m, s);
    return loclin_t<float, float>(d, N, x, (const float *)y, nh, h, (float *)m, s);
}

}  // namespace mecdf
