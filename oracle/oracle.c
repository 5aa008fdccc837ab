/*
 * Brute-force CPU oracle for the generalized multivariate ECDF / ESF and the
 * Laplacian-kernel sums of Langrene & Warin, "Fast multivariate empirical
 * cumulative distribution function with connection to kernel density
 * estimation" (arXiv 2005.03246).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain definition written out:
 * a double loop over (query, data point) with no sorting, no blocking, no
 * decomposition.  Only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg may load it; the GPU library never does, and the two share
 * no code.
 *
 * Floating-point sums use Neumaier's compensated summation (a textbook
 * refinement of Kahan's) so that the oracle's own rounding error stays near
 * one ulp of the result even for 2^24 terms.  Every weighted sum is returned
 * together with the same sum taken over |weight|, which is the scale that
 * GPU-vs-oracle errors are normalised by.
 *
 * Build: gcc -O2 -fopenmp -fPIC -shared oracle.c -o liboracle.so -lm
 * (no -ffast-math: the compensated sums rely on IEEE evaluation order).
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    double s; /* running sum          */
    double c; /* running compensation */
} nsum_t;

static inline void nsum_add(nsum_t *a, double v)
{
    double t = a->s + v;
    if (fabs(a->s) >= fabs(v))
        a->c += (a->s - t) + v;
    else
        a->c += (v - t) + a->s;
    a->s = t;
}

static inline double nsum_get(const nsum_t *a) { return a->s + a->c; }

/* nthreads > 0: that many threads; 0: the OpenMP default of the process
 * (OMP_NUM_THREADS, else all processors), restored on every call so that a
 * one-thread call does not leave later calls on one thread.  Every query's
 * sum runs on one thread in a fixed order, so results do not depend on it. */
static int default_threads(void)
{
#ifdef _OPENMP
    static int n = 0;
    if (n == 0)
        n = omp_get_max_threads();
    return n;
#else
    return 1;
#endif
}

static void set_threads(int nthreads)
{
#ifdef _OPENMP
    omp_set_num_threads(nthreads > 0 ? nthreads : default_threads());
#else
    (void)nthreads;
#endif
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return default_threads();
#else
    return 1;
#endif
}

/*
 * Weighted dominance sums, the sums inside eq. (ECDF) and eq. (ESF) of
 * Section 1 without the 1/N factor (the caller divides, as Remark 2.1
 * suggests, so that integer weights give exact results).
 *
 *   survival == 0 :  S_q = sum_i y_i * prod_k [ x_{k,i} <= z_{k,q} ]   (ECDF)
 *   survival != 0 :  S_q = sum_i y_i * prod_k [ x_{k,i} >  z_{k,q} ]   (ESF)
 *
 * Layout: x[k*N + i] (d x N), z[k*Q + q] (d x Q).  Comparisons are IEEE:
 * a NaN coordinate makes both <= and > false.
 *
 * y == NULL : y_i = 1 and the integer count goes to out_cnt[q].
 * y != NULL : out_sum[q] = compensated S_q, out_abs[q] = same with |y_i|.
 */
int oracle_dominance(int d, int64_t N, const double *x, const double *y,
                     int64_t Q, const double *z, int survival,
                     int64_t *out_cnt, double *out_sum, double *out_abs,
                     int nthreads)
{
    if (d < 1 || N < 0 || Q < 0 || !x || !z)
        return -1;
    if (!y && !out_cnt)
        return -1;
    if (y && (!out_sum || !out_abs))
        return -1;
    set_threads(nthreads);

#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t q = 0; q < Q; ++q) {
        int64_t cnt = 0;
        nsum_t s = {0.0, 0.0}, a = {0.0, 0.0};
        for (int64_t i = 0; i < N; ++i) {
            int inside = 1;
            for (int k = 0; k < d && inside; ++k) {
                double xi = x[(int64_t)k * N + i];
                double zq = z[(int64_t)k * Q + q];
                inside = survival ? (xi > zq) : (xi <= zq);
            }
            if (!inside)
                continue;
            if (y) {
                nsum_add(&s, y[i]);
                nsum_add(&a, fabs(y[i]));
            } else {
                ++cnt;
            }
        }
        if (y) {
            out_sum[q] = nsum_get(&s);
            out_abs[q] = nsum_get(&a);
        } else {
            out_cnt[q] = cnt;
        }
    }
    return 0;
}

/*
 * Laplacian kernel sums, the sum inside eq. (Laplacian_kde_nD) of Section 3.1
 * without its normalising constant 1/(2^d N prod_k h_k):
 *
 *   S[c][b][q] = sum_{i != skip[q]} w_c,i * exp( - sum_k |x_{k,i} - z_{k,q}| / h_{b,k} )
 *   A[c][b][q] = same with |w_c,i|
 *
 * for nw weight channels w[c*N + i] (w == NULL: one channel of ones) and nh
 * bandwidth vectors h[b*d + k].  skip == NULL excludes nothing; skip[q] = i
 * leaves data point i out of query q (leave-one-out at the sample points).
 * Output index: (c*nh + b)*Q + q.
 */
int oracle_laplace_sums(int d, int64_t N, const double *x, int nw,
                        const double *w, int64_t Q, const double *z, int nh,
                        const double *h, const int64_t *skip,
                        double *out_sum, double *out_abs, int nthreads)
{
    if (d < 1 || N < 0 || Q < 0 || nh < 1 || !x || !z || !h || !out_sum ||
        !out_abs)
        return -1;
    if (w == NULL)
        nw = 1;
    if (nw < 1 || nw > 8 || nh > 4096)
        return -1;
    for (int b = 0; b < nh; ++b)
        for (int k = 0; k < d; ++k)
            if (!(h[b * d + k] > 0.0))
                return -1;
    set_threads(nthreads);

#pragma omp parallel
    {
        /* per-thread accumulators: nw * nh of them */
        nsum_t acc_s[8 * 64], acc_a[8 * 64];
        for (int b0 = 0; b0 < nh; b0 += 64) {
            int nb = nh - b0 < 64 ? nh - b0 : 64;
#pragma omp for schedule(dynamic, 8)
            for (int64_t q = 0; q < Q; ++q) {
                for (int t = 0; t < nw * nb; ++t) {
                    acc_s[t].s = acc_s[t].c = 0.0;
                    acc_a[t].s = acc_a[t].c = 0.0;
                }
                int64_t sk = skip ? skip[q] : -1;
                for (int64_t i = 0; i < N; ++i) {
                    if (i == sk)
                        continue;
                    for (int b = 0; b < nb; ++b) {
                        double e = 0.0;
                        for (int k = 0; k < d; ++k)
                            e += fabs(x[(int64_t)k * N + i] -
                                      z[(int64_t)k * Q + q]) /
                                 h[(b0 + b) * d + k];
                        double kv = exp(-e);
                        for (int c = 0; c < nw; ++c) {
                            double wc = w ? w[(int64_t)c * N + i] : 1.0;
                            nsum_add(&acc_s[c * nb + b], wc * kv);
                            nsum_add(&acc_a[c * nb + b], fabs(wc) * kv);
                        }
                    }
                }
                for (int c = 0; c < nw; ++c)
                    for (int b = 0; b < nb; ++b) {
                        int64_t o = ((int64_t)c * nh + b0 + b) * Q + q;
                        out_sum[o] = nsum_get(&acc_s[c * nb + b]);
                        out_abs[o] = nsum_get(&acc_a[c * nb + b]);
                    }
            }
        }
    }
    return 0;
}

/*
 * Leave-one-out Laplacian kernel sums at the sample points with the largest
 * term factored out (a max-shifted log-sum-exp), for the likelihood and
 * squared-error cross-validation scores built on eq. (Laplacian_kde_nD).
 *
 * For query point j and bandwidth vector b, with e_i = sum_k |x_{k,i} - x_{k,j}| / h_{b,k}
 * over the data points i != j:
 *
 *   out_min[b*N + j]          = m = min_{i != j} e_i
 *   out_sum[(c*nh + b)*N + j] = sum_{i != j} w_c,i exp(-(e_i - m))
 *   out_abs[(c*nh + b)*N + j] = same with |w_c,i|
 *
 * so that sum_{i != j} w_c,i exp(-e_i) = exp(-m) * out_sum, and the logarithm
 * of the leave-one-out sum is -m + log(out_sum) even where every exp(-e_i)
 * underflows.  The nearest point (e_i = m) contributes exp(0) = 1, so
 * out_sum >= min_i w_0,i > 0 for positive weights.  N >= 2.
 */
int oracle_laplace_loo_shifted(int d, int64_t N, const double *x, int nw,
                               const double *w, int nh, const double *h,
                               double *out_min, double *out_sum,
                               double *out_abs, int nthreads)
{
    if (d < 1 || N < 2 || nh < 1 || !x || !h || !out_min || !out_sum ||
        !out_abs)
        return -1;
    if (w == NULL)
        nw = 1;
    if (nw < 1 || nw > 8)
        return -1;
    for (int b = 0; b < nh; ++b)
        for (int k = 0; k < d; ++k)
            if (!(h[b * d + k] > 0.0))
                return -1;
    set_threads(nthreads);

#pragma omp parallel for schedule(dynamic, 8) collapse(2)
    for (int b = 0; b < nh; ++b)
        for (int64_t j = 0; j < N; ++j) {
            /* first pass: the smallest scaled distance to another point */
            double m = INFINITY;
            for (int64_t i = 0; i < N; ++i) {
                if (i == j)
                    continue;
                double e = 0.0;
                for (int k = 0; k < d; ++k)
                    e += fabs(x[(int64_t)k * N + i] - x[(int64_t)k * N + j]) /
                         h[b * d + k];
                if (e < m)
                    m = e;
            }
            /* second pass: the sums relative to that term */
            nsum_t s[8], a[8];
            for (int c = 0; c < nw; ++c) {
                s[c].s = s[c].c = 0.0;
                a[c].s = a[c].c = 0.0;
            }
            for (int64_t i = 0; i < N; ++i) {
                if (i == j)
                    continue;
                double e = 0.0;
                for (int k = 0; k < d; ++k)
                    e += fabs(x[(int64_t)k * N + i] - x[(int64_t)k * N + j]) /
                         h[b * d + k];
                double kv = exp(-(e - m));
                for (int c = 0; c < nw; ++c) {
                    double wc = w ? w[(int64_t)c * N + i] : 1.0;
                    nsum_add(&s[c], wc * kv);
                    nsum_add(&a[c], fabs(wc) * kv);
                }
            }
            out_min[(int64_t)b * N + j] = m;
            for (int c = 0; c < nw; ++c) {
                int64_t o = ((int64_t)c * nh + b) * N + j;
                out_sum[o] = nsum_get(&s[c]);
                out_abs[o] = nsum_get(&a[c]);
            }
        }
    return 0;
}

/*
 * Generalized ECDF of eq. (ECDFdelta), Section 1, at query points with a
 * sign pattern per query, without the 1/N factor:
 *
 *   S_q = sum_i y_i * prod_k [ x_{k,i} <=_{delta_{k,q}} z_{k,q} ]
 *
 * where <=_{+1} is <= and <=_{-1} is the strict <.  delta[q] is a bit mask:
 * bit k set means delta_{k,q} = -1.  Counts / sums as oracle_dominance.
 */
int oracle_ecdf_delta(int d, int64_t N, const double *x, const double *y,
                      int64_t Q, const double *z, const unsigned char *delta,
                      int64_t *out_cnt, double *out_sum, double *out_abs,
                      int nthreads)
{
    if (d < 1 || d > 8 || N < 0 || Q < 0 || !x || !z || !delta)
        return -1;
    if (!y && !out_cnt)
        return -1;
    if (y && (!out_sum || !out_abs))
        return -1;
    set_threads(nthreads);

#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t q = 0; q < Q; ++q) {
        int64_t cnt = 0;
        nsum_t s = {0.0, 0.0}, a = {0.0, 0.0};
        for (int64_t i = 0; i < N; ++i) {
            int inside = 1;
            for (int k = 0; k < d && inside; ++k) {
                double xi = x[(int64_t)k * N + i];
                double zq = z[(int64_t)k * Q + q];
                inside = ((delta[q] >> k) & 1) ? (xi < zq) : (xi <= zq);
            }
            if (!inside)
                continue;
            if (y) {
                nsum_add(&s, y[i]);
                nsum_add(&a, fabs(y[i]));
            } else {
                ++cnt;
            }
        }
        if (y) {
            out_sum[q] = nsum_get(&s);
            out_abs[q] = nsum_get(&a);
        } else {
            out_cnt[q] = cnt;
        }
    }
    return 0;
}

/*
 * Kernel sums of two more compatible kernels (Section 3.2 and Appendix C),
 * without their normalising constants, for nw weight channels and nh
 * bandwidth vectors, layout as oracle_laplace_sums:
 *
 *   kind 0, uniform (eq. (uniform_kde_nD)):
 *     S = sum_i w_i prod_k [ lo_k <= x_{k,i} <= hi_k ],
 *     lo_k = z_k - h_k and hi_k = z_k + h_k, each rounded to a double
 *   kind 1, additive Matern-3/2 (eq. (Matern32_average)): with
 *     e_i = sum_k |x_{k,i} - z_k| / h_k,  S = sum_i w_i (1 + e_i) exp(-e_i)
 *
 * A holds the same sums with |w_i|.
 */
int oracle_kernel_sums(int kind, int d, int64_t N, const double *x, int nw,
                       const double *w, int64_t Q, const double *z, int nh,
                       const double *h, double *out_sum, double *out_abs,
                       int nthreads)
{
    if (d < 1 || N < 0 || Q < 0 || nh < 1 || !x || !z || !h || !out_sum ||
        !out_abs || (kind != 0 && kind != 1))
        return -1;
    if (w == NULL)
        nw = 1;
    if (nw < 1 || nw > 8 || nh > 64)
        return -1;
    for (int b = 0; b < nh; ++b)
        for (int k = 0; k < d; ++k)
            if (!(h[b * d + k] > 0.0))
                return -1;
    set_threads(nthreads);

#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t q = 0; q < Q; ++q) {
        nsum_t acc_s[8 * 64], acc_a[8 * 64];
        for (int t = 0; t < nw * nh; ++t) {
            acc_s[t].s = acc_s[t].c = 0.0;
            acc_a[t].s = acc_a[t].c = 0.0;
        }
        for (int64_t i = 0; i < N; ++i) {
            for (int b = 0; b < nh; ++b) {
                double kv;
                if (kind == 0) {
                    int inside = 1;
                    for (int k = 0; k < d && inside; ++k) {
                        double xi = x[(int64_t)k * N + i];
                        double zq = z[(int64_t)k * Q + q];
                        double hk = h[b * d + k];
                        double lo = zq - hk, hi = zq + hk;
                        inside = lo <= xi && xi <= hi;
                    }
                    kv = inside ? 1.0 : 0.0;
                } else {
                    double e = 0.0;
                    for (int k = 0; k < d; ++k)
                        e += fabs(x[(int64_t)k * N + i] - z[(int64_t)k * Q + q]) /
                             h[b * d + k];
                    kv = (1.0 + e) * exp(-e);
                }
                for (int c = 0; c < nw; ++c) {
                    double wc = w ? w[(int64_t)c * N + i] : 1.0;
                    nsum_add(&acc_s[c * nh + b], wc * kv);
                    nsum_add(&acc_a[c * nh + b], fabs(wc) * kv);
                }
            }
        }
        for (int c = 0; c < nw; ++c)
            for (int b = 0; b < nh; ++b) {
                int64_t o = ((int64_t)c * nh + b) * Q + q;
                out_sum[o] = nsum_get(&acc_s[c * nh + b]);
                out_abs[o] = nsum_get(&acc_a[c * nh + b]);
            }
    }
    return 0;
}
