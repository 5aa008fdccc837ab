/*
 * mecdf.h -- C ABI of libmecdf, exact multivariate ECDF / ESF and Laplacian
 * kernel sums on an AMD MI355X (gfx950) GPU.
 *
 * Method: Langrene & Warin, "Fast multivariate empirical cumulative
 * distribution function with connection to kernel density estimation",
 * arXiv 2005.03246.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Data layout.  Sample points are passed structure-of-arrays as a device
 * array x of d*N doubles with x[k*N + i] = coordinate k of point i (the
 * paper's x_{k,i}, Section 1).  x is always float64: membership is decided by
 * exact comparisons in the input precision and x is never converted.
 *
 * Weights.  y (or w) is a device array of N values.  With prec == MECDF_F64
 * it holds doubles and results are doubles; with prec == MECDF_F32C it holds
 * floats and results are floats.  What F32C computes in float32 differs by
 * path: the grid path bins and scans in float32 with Kahan compensation; the
 * points path sums float32 weights with Kahan compensation; the kernel-sum
 * path forms its exponentials and runs its scans in float32 without
 * compensation (each scan level's result is added into float64 sums, and the
 * decay over a long run is formed from the float64 coordinates of its ends
 * rather than multiplied out), and its leave-one-out scores are float64.
 * Where an entry point accepts y == NULL, y is taken as 1 and the result is
 * the raw integer count (int64, no 1/N factor): the classical ECDF of
 * Section 1 times N.
 *
 * Ownership.  The caller owns every buffer.  Device pointers must point to
 * memory on the current HIP device; host pointers (grid sizes, nodes,
 * bandwidths) are read before the call returns.  The library owns only an
 * internal per-device workspace, grown on demand and kept until
 * mecdf_release(); the environment variable MECDF_WORKSPACE_LIMIT (bytes)
 * caps it.
 *
 * Streams.  stream is a hipStream_t (NULL = the default stream).  Work is
 * enqueued on it in order and the call returns without waiting for the GPU,
 * except where a comment says otherwise.  Two calls that overlap in time on
 * one device share the workspace and race; issue them on one stream.
 *
 * Errors.  Every int-returning function returns MECDF_OK (0) or a negative
 * code.  Argument errors are detected on the host before anything is
 * enqueued and leave the outputs untouched.  A HIP runtime failure returns
 * MECDF_EDEVICE.  mecdf_last_error() gives a message for the calling thread's
 * most recent failure.  NaN inputs are not errors: they follow IEEE
 * comparisons (a NaN coordinate makes both <= and > false), so a point with a
 * NaN coordinate counts for no query and a NaN query counts nothing.
 */
#ifndef MECDF_H
#define MECDF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    MECDF_OK = 0,
    MECDF_EINVAL = -1,       /* invalid argument                          */
    MECDF_ENOMEM = -2,       /* workspace allocation failed or over limit */
    MECDF_EDEVICE = -3,      /* HIP runtime error                         */
    MECDF_EUNSUPPORTED = -4, /* valid but outside the supported sizes     */
    MECDF_EIO = -5           /* a checkpoint file could not be read/written */
};

enum {
    MECDF_F64 = 0,  /* float64 weights and results                        */
    MECDF_F32C = 1  /* float32 weights and results, compensated summation */
};

/* Largest supported dimension d (the paper's experiments go up to 6). */
#define MECDF_MAX_DIM 6

const char *mecdf_strerror(int code);
const char *mecdf_last_error(void);

/*
 * ecdf_grid -- generalized ECDF at every node of a rectilinear grid.
 *
 * Computes F_N(z) = (1/N) sum_i y_i 1{x_{1,i} <= z_1, ..., x_{d,i} <= z_d}
 * (eq. (ECDF), Section 1) at the M_1 x ... x M_d nodes of the grid of
 * Section 2.1, through the local sums of eq. (partial_sums) and the d-fold
 * prefix sum of eq. (ECDF_decomposition).
 *
 *   d      1..MECDF_MAX_DIM
 *   N      number of sample points (>= 1; 0 is allowed only with y == NULL)
 *   x      device, d*N doubles, x[k*N + i]
 *   y      device, N weights (double or float per prec) or NULL for counts
 *   M      host, d grid sizes M_k >= 1
 *   z      host, sum(M_k) doubles: the nodes of axis 0, then axis 1, ...;
 *          each axis strictly increasing and finite
 *   F      device, prod(M_k) results in C order (last axis fastest):
 *          int64 counts (y == NULL), else double/float F_N
 *   prec   MECDF_F64 or MECDF_F32C (ignored when y == NULL)
 *
 * Limits: prod(M_k + 1) < 2^31 cells and M_d <= 4000.  Results are
 * deterministic: the same inputs give bitwise-equal outputs.
 */
int ecdf_grid(int d, int64_t N, const double *x, const void *y,
              const int64_t *M, const double *z, void *F, int prec,
              void *stream);

/*
 * esf_grid -- generalized ESF (eq. (ESF), Section 1) at every grid node:
 * Fbar_N(z) = (1/N) sum_i y_i 1{x_{1,i} > z_1, ..., x_{d,i} > z_d}, strict in
 * every coordinate.  It equals the ECDF of the reflected data with the strict
 * inequality (Section 1, eq. (ECDFdelta) with delta = -1) and is obtained
 * from the same local sums with suffix sums.  Arguments as ecdf_grid, with
 * the result written to Fbar.
 */
int esf_grid(int d, int64_t N, const double *x, const void *y,
             const int64_t *M, const double *z, void *Fbar, int prec,
             void *stream);

/*
 * ecdf_esf_grid -- both of the above from one binning pass.  Either output
 * pointer may be NULL (then that function is skipped); not both.
 */
int ecdf_esf_grid(int d, int64_t N, const double *x, const void *y,
                  const int64_t *M, const double *z, void *F, void *Fbar,
                  int prec, void *stream);

/*
 * ecdf_esf_grid_noalloc -- ecdf_esf_grid for callers that cannot allocate
 * device memory (work recorded under stream capture, tight serving loops,
 * harnesses that forbid allocation).  Same arguments, results and argument
 * errors as ecdf_esf_grid, but the call allocates nothing: its working memory
 * is a fixed array of MECDF_NOALLOC_SCRATCH_BYTES bytes that the library
 * holds on each device it runs on until the process ends, and the nodes z
 * are copied from the caller's host array on the stream (read before the
 * call returns).  A problem whose working memory exceeds the array returns
 * MECDF_EUNSUPPORTED before anything is enqueued; it takes about 12 bytes
 * per point for counts, 20 with float32 and 28 with float64 weights, plus
 * 12 bytes per grid line (the product of M_k + 1 over all axes but the last)
 * and the nodes, so about 2.3 million float64 points fit.  Every call on one
 * device uses the same array and leaves its contents behind: calls that
 * overlap in time on a device (other streams or threads) race; issue them on
 * one stream.
 */
#define MECDF_NOALLOC_SCRATCH_BYTES (64u << 20)
int ecdf_esf_grid_noalloc(int d, int64_t N, const double *x, const void *y,
                          const int64_t *M, const double *z, void *F, void *Fbar,
                          int prec, void *stream);

/*
 * mecdf_grid_interp -- values given at the nodes of a rectilinear grid (for
 * example the output of ecdf_grid) at arbitrary points, by multilinear
 * interpolation: the route from a grid evaluation to values at the sample
 * points whose error Section 4.1 (ECDF) and Section 4.2 (KDE) measure.
 *
 *   d, M, z  the grid as in ecdf_grid (host), any sizes M_k >= 1
 *   G        device, prod(M_k) values in C order (double, or float with
 *            MECDF_F32C; interpolation is computed in float64)
 *   Q, q     Q >= 0 points, device d*Q doubles, q[k*Q + p]
 *   out      device Q results (type of G)
 *
 * Along each axis a point outside [z_0, z_{M-1}] takes the value at the
 * nearest end node (no extrapolation); an axis with one node is constant; a
 * NaN coordinate gives NaN.
 */
int mecdf_grid_interp(int d, const int64_t *M, const double *z, const void *G,
                      int64_t Q, const double *q, void *out, int prec,
                      void *stream);

/*
 * ecdf_points -- generalized ECDF at the sample points themselves
 * (Section 2.2): F[j] = F_N(x_j) = (1/N) sum_i y_i 1{x_i <= x_j componentwise}.
 * Unlike the recursion's own output in Section 2.2, which leaves the point
 * itself out and uses strict inequalities, the result follows eq. (ECDF)
 * literally: <= in every coordinate, the point itself and exact duplicates
 * included.
 *
 *   x   device, d*N doubles;  y  device N weights or NULL (int64 counts)
 *   F   device, N results in input order
 *
 * Limits: N <= 2^26 (MECDF_EUNSUPPORTED above).  Results are deterministic.
 * Up to N = 20000, 24000, 32000, 46000, 80000, 150000 for d = 1 .. 6 (or
 * the value of the environment variable MECDF_POINTS_DIRECT_MAX) every pair
 * is evaluated directly; above, the divide-and-conquer recursion runs.
 * Neither waits for the device.
 */
int ecdf_points(int d, int64_t N, const double *x, const void *y, void *F,
                int prec, void *stream);

/*
 * esf_points -- generalized ESF at the sample points (eq. (ESF) with z = x_j):
 * F[j] = (1/N) sum_i y_i 1{x_i > x_j strictly in every coordinate}.
 * Arguments as ecdf_points.
 */
int esf_points(int d, int64_t N, const double *x, const void *y, void *F,
               int prec, void *stream);

/*
 * ecdf_delta_at -- the generalized ECDF of eq. (ECDFdelta) (Section 1) at Q
 * arbitrary points, each with its own inequality pattern:
 *
 *   F[q] = (1/N) sum_i y_i prod_k 1{x_{k,i} <=_{delta_{k,q}} z_{k,q}}
 *
 * where <=_{+1} is <= and <=_{-1} is the strict <.  The points recursion of
 * Section 2.2 runs over the N data items and Q query items; a query's rank on
 * each axis is found among the distinct data values, so ties with data
 * values and the strict / non-strict choice are exact.
 *
 *   x      device d*N doubles (N >= 1);  y  device N weights or NULL (counts)
 *   Q, z   Q >= 0 query points, device d*Q doubles, z[k*Q + q]
 *   delta  device Q bytes, bit k set for delta_k = -1 (strict), clear for
 *          <=; or NULL for <= everywhere (then F[q] = F_N(z_q) of eq. (ECDF))
 *   F      device Q results: int64 counts (y == NULL) or double / float F_N
 *
 * A query with a NaN coordinate counts nothing (F = 0), as does a data point
 * with one for every query.  Limits: N <= 2^26 and Q <= 2^26
 * (MECDF_EUNSUPPORTED above).  Deterministic; does not wait for the device.
 */
int ecdf_delta_at(int d, int64_t N, const double *x, const void *y, int64_t Q,
                  const double *z, const uint8_t *delta, void *F, int prec,
                  void *stream);

/*
 * kde_uniform -- the weighted uniform-kernel density estimate of eq.
 * (uniform_kde_nD) (Section 3.2) at Q arbitrary points (pass z = x for the
 * sample points), for nh bandwidth vectors:
 *
 *   f[b*Q + q] = 1/(2^d N prod_k h_{b,k}) sum_i w_i prod_k 1{lo_k <= x_{k,i} <= hi_k}
 *
 * with lo_k = z_{k,q} - h_{b,k} and hi_k = z_{k,q} + h_{b,k}, each rounded to
 * a double, computed as eq. (uniform_decomposition_nD): the signed sum of
 * ecdf_delta_at at the 2^d box corners, all corners of a bandwidth in one
 * recursion.  When z is x itself (the same pointer, Q == N) the corners'
 * ranks are read from tables over the distinct data values instead of being
 * searched per corner (same results, bit for bit, as a copy of x passed as
 * z).  With w == NULL the box counts are exact integers before the
 * final scaling; weighted sums are float64 differences of F_N values (their
 * error is relative to the total |w| mass, not to the box's).
 *
 *   x, N       as ecdf_delta_at;  w  device N weights or NULL (all 1)
 *   Q, z       device query points as ecdf_delta_at
 *   nh, h      host nh*d positive bandwidths, h[b*d + k]
 *   f          device nh*Q results (double, or float with MECDF_F32C)
 *
 * Limits: Q 2^d <= 2^26.  Deterministic; does not wait for the device.
 */
int kde_uniform(int d, int64_t N, const double *x, const void *w, int64_t Q,
                const double *z, int nh, const double *h, void *f, int prec,
                void *stream);

/*
 * kde_laplace -- weighted Laplacian-kernel density estimate at the sample
 * points for nh bandwidth vectors (eq. (Laplacian_kde_nD), Section 3.1),
 * evaluated through the 2^d sign-orthant ECDF decomposition of
 * eq. (Laplacian_decomposition_nD) with all orthants in one recursion
 * (Appendix D):
 *
 *   f[b*N + j] = 1/(2^d N prod_k h_{b,k}) sum_i w_i exp(-sum_k |x_{k,i} - x_{k,j}| / h_{b,k})
 *
 * (the point itself included, kernel value 1 at distance 0), and the
 * likelihood cross-validation score
 *
 *   lcv[b] = (1/N) sum_j log fhat_{-j}(x_j),
 *   fhat_{-j} = 1/(2^d (N-1) prod_k h_{b,k}) sum_{i != j} w_i exp(...).
 *
 *   d     1..MECDF_MAX_DIM
 *   N     >= 2
 *   x     device d*N doubles
 *   w     device N doubles (float with MECDF_F32C) or NULL for w = 1
 *   nh    number of bandwidth vectors, 1..256
 *   h     host, nh*d positive finite doubles, h[b*d + k]
 *   f     device nh*N results (double, or float with MECDF_F32C) or NULL
 *   lcv   device nh doubles or NULL
 *
 * The logarithm in lcv is taken of the leave-one-out sum relative to the
 * nearest other point, so the score stays finite where every kernel term is
 * below the float64 range.  d = 1..3 run the recursion (O(N log^(d-1) N) per
 * bandwidth); d = 4..6 evaluate every pair directly (O(N^2 d)).
 *
 * Limits: N <= 2^28, N <= 2^24 for d = 3 and N <= 2^20 for d >= 4
 * (MECDF_EUNSUPPORTED above).
 */
int kde_laplace(int d, int64_t N, const double *x, const void *w, int nh,
                const double *h, void *f, double *lcv, int prec, void *stream);

/*
 * kreg_laplace -- Nadaraya-Watson kernel regression with the Laplacian
 * kernel at the sample points (weights w = response, Section 3.1):
 *
 *   m[b*N + j] = sum_i y_i K_b(x_i - x_j) / sum_i K_b(x_i - x_j)   (self included)
 *   cv[b]      = (1/N) sum_j (y_j - m_{-j})^2,  m_{-j} the same ratio over i != j
 *
 * Arguments as kde_laplace with y the response (required).
 */
int kreg_laplace(int d, int64_t N, const double *x, const void *y, int nh,
                 const double *h, void *m, double *cv, int prec, void *stream);

/*
 * kde_laplace_H / kreg_laplace_H -- kde_laplace and kreg_laplace with general
 * symmetric positive definite bandwidth matrices (Appendix B,
 * eq. (kde_nD_H)), read as the paper does: with H = R diag(h)^2 R^T, the
 * estimator with diagonal bandwidth h in the coordinates R^T x,
 *
 *   f[b*N + j] = 1/(2^d N prod_k h_k) sum_i w_i exp(-|| diag(1/h) R^T (x_i - x_j) ||_1).
 *
 * (For the product form of the Laplacian kernel this depends on R, which is
 * unique up to the signs and order of its columns when the eigenvalues are
 * distinct; with a repeated eigenvalue the eigenvectors the library's Jacobi
 * sweeps find are used.)  H: host, nh row-major d x d matrices; the points
 * are rotated on the device and the kernel sums run as in kde_laplace (one
 * pass per matrix).  Other arguments as kde_laplace / kreg_laplace;
 * MECDF_EINVAL for a matrix that is not positive definite or whose two
 * triangles differ by more than 1e-12 of its largest entry (otherwise its
 * symmetric part is used).
 */
int kde_laplace_H(int d, int64_t N, const double *x, const void *w, int nh,
                  const double *H, void *f, double *lcv, int prec, void *stream);
int kreg_laplace_H(int d, int64_t N, const double *x, const void *y, int nh,
                   const double *H, void *m, double *cv, int prec, void *stream);

/*
 * kreg_loclin_laplace -- local-linear regression with the Laplacian kernel at
 * the sample points: m[b*N + j] is the intercept of the weighted
 * least-squares fit of y ~ a + c^T (x - x_j) with weights
 * exp(-sum_k |x_{k,i} - x_{k,j}| / h_{b,k}) (the point itself included).
 * Its moments are kernel sums with the weights 1, x_l, x_l x_m, y and y x_l
 * (1 + d + d(d+1)/2 + 1 + d calls of the kernel-sum path per bandwidth,
 * float64), expanded about x_j, and a (d+1) x (d+1) system per point is
 * solved with partial pivoting; where a pivot is below 1e-10 of the largest
 * diagonal entry the local constant (Nadaraya-Watson) estimate is returned.
 * The expansion about x_j loses about (|x_j| / local spread)^2 in relative
 * accuracy to cancellation.  Arguments as kreg_laplace (m required).
 */
int kreg_loclin_laplace(int d, int64_t N, const double *x, const void *y, int nh,
                        const double *h, void *m, int prec, void *stream);

/*
 * kde_laplace_grid -- the Laplacian kernel density estimate of kde_laplace at
 * every node of a rectilinear grid (the paper's "fast summation" KDE,
 * Section 3 with the grid of Section 2.1):
 *
 *   f[b*G + node] = 1/(2^d N prod_k h_{b,k}) sum_i w_i exp(-sum_k |x_{k,i} - z_k| / h_{b,k})
 *
 * for the G = prod(M_k) nodes z in C order.  Each point's weight is carried
 * to the nodes of its cell's corners (factors <= 1) and spread by decayed
 * scans along every axis, 2^d channels, the two channels of a corner pair
 * added after the scan of their axis: O(N log N) once and O(N + 2^d G) per
 * bandwidth.
 *
 *   x, w, nh, h, prec  as kde_laplace (N >= 1)
 *   M, z               the grid as ecdf_grid (host)
 *   f                  device nh*G results (double, or float with MECDF_F32C)
 *
 * Points with a NaN coordinate are left out.  Far from every point the sums
 * underflow to 0 as float64 sums do.  Float32 weights and results are
 * converted; the arithmetic is float64.  Limits: prod(M_k + 1) < 2^31 - 1
 * cells.  Deterministic.
 */
int kde_laplace_grid(int d, int64_t N, const double *x, const void *w,
                     const int64_t *M, const double *z, int nh, const double *h,
                     void *f, int prec, void *stream);

/*
 * kreg_laplace_grid -- the Nadaraya-Watson estimate of kreg_laplace at every
 * grid node: m[b*G + node] = sum_i y_i K / sum_i K (NaN where both sums
 * underflow).  Arguments as kde_laplace_grid with y the response.
 */
int kreg_laplace_grid(int d, int64_t N, const double *x, const void *y,
                      const int64_t *M, const double *z, int nh, const double *h,
                      void *m, int prec, void *stream);

/*
 * kde_matern32_grid -- kernel density estimate at every grid node with the
 * additive multivariate Matern-3/2 kernel of Appendix C, eq.
 * (Matern32_average), K_d(u) = (1 + sum_k |u_k|) exp(-sum_k |u_k|) /
 * (2^d (1 + d)), u = (x - z) / h:
 *
 *   f[b*G + node] = 1/(N prod_k h_{b,k}) sum_i w_i K_d((x_i - z) / h_b)
 *
 * through its CDF decomposition (eq. (Matern32_decomposition_nD)): 2^d (d+1)
 * channels, the plain exponential sums and one distance-weighted sum per
 * axis, spread by decayed scans (the distance sums move with the plain sums
 * along their own axis).  Arguments, layout, errors and precision as
 * kde_laplace_grid; d = 1..6.
 */
int kde_matern32_grid(int d, int64_t N, const double *x, const void *w,
                      const int64_t *M, const double *z, int nh, const double *h,
                      void *f, int prec, void *stream);

/*
 * kreg_matern32_grid -- the Nadaraya-Watson estimate with the same kernel at
 * every grid node: m[b*G + node] = sum_i y_i K / sum_i K (NaN where both sums
 * underflow).  Arguments as kreg_laplace_grid; d = 1..6.
 */
int kreg_matern32_grid(int d, int64_t N, const double *x, const void *y,
                       const int64_t *M, const double *z, int nh, const double *h,
                       void *m, int prec, void *stream);

/* ---------------------------------------------------------------------
 * Bandwidth selection (batched exact LOO likelihood cross-validation, and a
 * learned proposal that only decides where to evaluate it).
 * ------------------------------------------------------------------- */

/* One dataset: d coordinates (1..3) of N points, device x[k*N + i]. */
typedef struct {
    int d;
    int64_t N;
    const double *x;
} mecdf_dataset;

/*
 * mecdf_kde_lcv_batched -- the likelihood CV score of kde_laplace for many
 * datasets and isotropic bandwidths: for dataset s, the nh[s] bandwidths
 * h[off_s .. off_s + nh[s]) (off_s = nh[0] + ... + nh[s-1]), each used on
 * every axis, give lcv[off_s + b] (device doubles).  best (device, nsets
 * ints, or NULL) receives each dataset's index b of its largest score (the
 * lowest such b on ties; -1 when nh[s] = 0): the grid-search choice, and the
 * label mecdf_bw_train takes.  sets, nh and h are host arrays.  Every
 * dataset is checked before the first is run; same errors as kde_laplace.
 * The small datasets are scored by one work-queue launch on the stream; the
 * recursions of the larger ones run on a few streams the library keeps
 * beside it (default priority), which wait for the work enqueued on the
 * stream before the call and which the stream waits for before the best
 * indices are taken, so the call is ordered on the stream as a whole.
 */
int mecdf_kde_lcv_batched(const mecdf_dataset *sets, int nsets, const int *nh,
                          const double *h, double *lcv, int *best, int prec,
                          void *stream);

/*
 * Batched scores prepared once and run repeatedly: mecdf_lcv_plan_create
 * takes the arguments of mecdf_kde_lcv_batched (the same outputs, written on
 * every run), copies what the kernels read from the host into memory the
 * plan owns (with its own working memory, so other calls cannot disturb it)
 * and records the work queue of the small datasets into a HIP graph.
 * mecdf_lcv_plan_run launches that graph on the plan's own stream, enqueues
 * the recursions of the larger datasets on the given stream meanwhile, joins
 * the two on the given stream and writes the best indices (the datasets may
 * change in value between runs, not in place or size; runs of one plan must
 * not overlap).  mecdf_lcv_plan_destroy waits for the device and frees the
 * plan.  Creation waits for the device.  For callers that score the same
 * shapes repeatedly.
 */
typedef struct mecdf_lcv_plan_s *mecdf_lcv_plan;
int mecdf_lcv_plan_create(const mecdf_dataset *sets, int nsets, const int *nh,
                          const double *h, double *lcv, int *best, int prec,
                          mecdf_lcv_plan *plan);
int mecdf_lcv_plan_run(mecdf_lcv_plan plan, void *stream);
void mecdf_lcv_plan_destroy(mecdf_lcv_plan plan);

/*
 * mecdf_autotune -- chooses, per precision and d = 1, 2, 3, up to which N the
 * batched scores use the work queue (every pair, one launch for all small
 * datasets) rather than the recursion, by timing both on the current device
 * for N = 512 .. 32768 with 64 bandwidths; writes the choice and the times as
 * JSON to path (NULL: the file the library reads, $MECDF_TUNE_FILE or
 * tune_<arch>.json beside libmecdf.so) and uses it from then on.  The library
 * reads that file on first use when its architecture matches the device's;
 * otherwise built-in values apply.  Takes seconds; waits for the device.
 *
 * mecdf_tuning -- the values in use: queue_max_n[p * 3 + d - 1] for
 * precision p (0 float64, 1 float32) and d, and where they came from (a file
 * path, "built-in defaults" or "set by the caller") into source (cap bytes).
 * mecdf_tuning_set replaces them for this process (each in 0..2^24).
 */
int mecdf_autotune(const char *path, void *stream);
int mecdf_tuning(int64_t *queue_max_n, char *source, int cap);
int mecdf_tuning_set(const int64_t *queue_max_n);

/*
 * mecdf_bw_features -- 32 summary statistics per dataset (device floats,
 * feat[s*32 + q]), computed on the device in one block per dataset:
 * log N / 10, d / 3, per-axis log sd, skewness, excess kurtosis / 10,
 * mean |correlation|, log h0 with h0 = (geometric-mean sd) N^(-1/(d+4))
 * (index 12), log geometric-mean sd, per-axis mean |x - mean| / sd, the
 * fraction of points within half a sd of the mean (indices 17..19) and the
 * fractions within a quarter, one and two sd (20 + 3k .. 22 + 3k for axis k);
 * unused entries are 0.
 */
int mecdf_bw_features(const mecdf_dataset *sets, int nsets, float *feat,
                      void *stream);

/*
 * Network 32 -> 128 -> 128 -> 1 with ReLU activations; its parameters are
 * one device float vector of MECDF_MLP_PARAMS entries laid out as
 * W1[128][32], b1[128], W2[128][128], b2[128], w3[128], b3.  Matrix products
 * use bfloat16 operands (round to nearest even) with float32 accumulation.
 *
 * mecdf_mlp_forward: out[r] for the B rows feat[r*32 .. r*32+32).
 * mecdf_mlp_grad:    gradient of the mean squared error
 *                    (1/B) sum_r (out[r] - target[r])^2 into grad[MECDF_MLP_PARAMS]
 *                    and the loss into loss[0] (loss may be NULL).
 * mecdf_mlp_train:   `steps` full-batch Adam steps (beta1 0.9, beta2 0.999,
 *                    eps 1e-8, learning rate lr) with decoupled weight decay
 *                    (each step also subtracts lr * wd * params; wd >= 0)
 *                    updating params in place; adam is device
 *                    float[2*MECDF_MLP_PARAMS], zero before the first step;
 *                    losses[t] (device, optional) is the loss before step t.
 * All pointers are device pointers; B >= 1.
 */
#define MECDF_MLP_PARAMS 20865
int mecdf_mlp_forward(int B, const float *feat, const float *params, float *out,
                      void *stream);
int mecdf_mlp_grad(int B, const float *feat, const float *target,
                   const float *params, float *grad, float *loss, void *stream);
int mecdf_mlp_train(int B, const float *feat, const float *target, float *params,
                    float *adam, int steps, float lr, float wd, float *losses,
                    void *stream);

/*
 * mecdf_bw_train -- trains the network of mecdf_bw_select on grid labels.
 * The target of dataset r is log(hgrid[label[r]]) - feat[r*32 + 12] (the
 * grid optimum relative to the rule-of-thumb bandwidth); training runs
 * `steps` full-batch steps of mecdf_mlp_train's Adam with decoupled weight
 * decay.
 *
 *   B, feat     B >= 1 datasets, device float[B*32] from mecdf_bw_features
 *   label       device int[B], grid indices in [0, nhg) (the best output of
 *               mecdf_kde_lcv_batched); checked on the host (one wait)
 *   nhg, hgrid  host, the ascending bandwidth grid
 *   seed        seeds fresh parameters (He-style normals from a counter-based
 *               generator: the same seed gives the same parameters)
 *   params      device float[MECDF_MLP_PARAMS]; adam device
 *               float[2*MECDF_MLP_PARAMS] (Adam moments)
 *   losses      device float[steps] or NULL: the loss before each step
 *   checkpoint  host path or NULL
 *   step        in: Adam steps already taken on params/adam (0 = start
 *               fresh from the seed, which overwrites params and adam);
 *               out: the total after this call
 *
 * With a checkpoint path naming an existing file, the parameters, moments
 * and step count are read from it (it must have been written with the same
 * seed: MECDF_EINVAL otherwise; MECDF_EIO when it is not a whole
 * checkpoint) and training continues from there, so that training in parts
 * gives the same parameters as in one call.  When a path is given the file is
 * written (replaced atomically) after the steps, and the call waits for the
 * device.
 */
int mecdf_bw_train(int B, const float *feat, const int *label, int nhg,
                   const double *hgrid, int steps, float lr, float wd,
                   uint64_t seed, float *params, float *adam, float *losses,
                   const char *checkpoint, int64_t *step, void *stream);

/*
 * mecdf_bw_select -- likelihood-CV bandwidth on an ascending grid of nhg
 * isotropic bandwidths (hgrid, host).  The network proposes
 * log h = feat[12] + net(feat); the exact LOO likelihood score is evaluated
 * at the four grid bandwidths around the proposal (grid indices
 * round(j) - 2 .. round(j) + 1 for the proposal's fractional index j, a
 * window centred within half a step of j, clamped to the grid).  With mode MECDF_BW_EXTEND the evaluated window is
 * then extended by four grid points at a time towards the best score until
 * the best score is interior to it (or at the grid's end); with
 * MECDF_BW_WINDOW the four-point window is the answer.  The windows of all
 * datasets are scored together by the batched scores of
 * mecdf_kde_lcv_batched, one round per extension.  Returns, per dataset
 * (host arrays), the chosen grid index, its LCV score (lcv_out may be NULL)
 * and the number of bandwidths evaluated (evals_out may be NULL).  Every
 * returned score is an exact evaluation.  Synchronous: waits for the device
 * after the proposals and after each round.
 */
#define MECDF_BW_EXTEND 0
#define MECDF_BW_WINDOW 1
int mecdf_bw_select(const mecdf_dataset *sets, int nsets, const float *params,
                    int nhg, const double *hgrid, int mode, int *hidx_out,
                    double *lcv_out, int *evals_out, void *stream);

/* Frees the workspace of every device (synchronises those devices). */
void mecdf_release(void);

/*
 * Kernel timing support for benchmarks (not part of the method).  While
 * enabled (on = 1), every kernel launch of the entry points above is
 * bracketed by a pair of HIP events on the caller's stream; with on = 2
 * ("cold"), a 1 GiB device buffer that the library allocates once is also
 * read before each bracketed group, outside its events, so that the group's
 * inputs are not in the 256 MB infinity cache.  mecdf_profile_collect waits for
 * the recorded events and writes, for up to max distinct kernel names in
 * launch order, the name (64 bytes each, NUL-terminated, into names), the
 * summed duration in milliseconds and the launch count; it returns the number
 * of names written or a negative error.  mecdf_profile_reset forgets the
 * records.  Not thread-safe against concurrent entry-point calls.
 */
int mecdf_profile_enable(int on);
void mecdf_profile_reset(void);
int mecdf_profile_collect(int max, char *names, double *total_ms,
                          int64_t *launches);

#ifdef __cplusplus
}
#endif

#endif /* MECDF_H */
