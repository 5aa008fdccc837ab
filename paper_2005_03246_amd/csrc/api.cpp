// C ABI of libmecdf: argument validation and dispatch (see include/mecdf.h).
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>

#include "common.hpp"

namespace mecdf {
int grid_run(int d, int64_t N, const double *x, const void *y,
             const int64_t *M, const double *z, void *F, void *Fbar, int prec,
             hipStream_t s);
int points_run(int d, int64_t N, const double *x, const void *y, void *F,
               int survival, int prec, hipStream_t s);
int kde_run(int d, int64_t N, const double *x, const void *w, int nh,
            const double *h, void *f, double *score, int regression,
            int prec, hipStream_t s);
}  // namespace mecdf

using namespace mecdf;

namespace {

int fail(int code, const std::string &msg) {
    set_error(msg);
    return code;
}

int check_common(int d, int64_t N, const double *x, int prec, int maxd) {
    if (d < 1 || d > maxd)
        return fail(MECDF_EINVAL, "d must be in 1.." + std::to_string(maxd));
    if (N < 0)
        return fail(MECDF_EINVAL, "N must be >= 0");
    if (N >= (int64_t(1) << 31))
        return fail(MECDF_EUNSUPPORTED, "N must be < 2^31");
    if (N > 0 && x == nullptr)
        return fail(MECDF_EINVAL, "x is NULL");
    if (prec != MECDF_F64 && prec != MECDF_F32C)
        return fail(MECDF_EINVAL, "prec must be MECDF_F64 or MECDF_F32C");
    return MECDF_OK;
}

int grid_entry(int d, int64_t N, const double *x, const void *y,
               const int64_t *M, const double *z, void *F, void *Fbar,
               int prec, void *stream) {
    MECDF_TRY(check_common(d, N, x, prec, MECDF_MAX_DIM));
    if (y != nullptr && N == 0)
        return fail(MECDF_EINVAL, "weighted ECDF needs N >= 1 (1/N factor)");
    if (M == nullptr || z == nullptr)
        return fail(MECDF_EINVAL, "grid sizes M and nodes z are required");
    if (F == nullptr && Fbar == nullptr)
        return fail(MECDF_EINVAL, "no output requested");
    double cells = 1.0;
    int64_t off = 0;
    for (int k = 0; k < d; ++k) {
        if (M[k] < 1)
            return fail(MECDF_EINVAL, "grid size M_k must be >= 1");
        if (M[k] > (int64_t(1) << 24))
            return fail(MECDF_EUNSUPPORTED, "grid size M_k too large");
        for (int64_t j = 0; j < M[k]; ++j) {
            double v = z[off + j];
            if (!std::isfinite(v))
                return fail(MECDF_EINVAL, "grid nodes must be finite");
            if (j > 0 && !(z[off + j - 1] < v))
                return fail(MECDF_EINVAL,
                            "grid nodes must be strictly increasing per axis");
        }
        off += M[k];
        cells *= (double)(M[k] + 1);
    }
    if (cells >= 2147483648.0)
        return fail(MECDF_EUNSUPPORTED, "grid has 2^31 or more cells");
    if (M[d - 1] > 4000)
        return fail(MECDF_EUNSUPPORTED, "last grid axis must have <= 4000 nodes");
    return grid_run(d, N, x, y, M, z, F, Fbar, prec, (hipStream_t)stream);
}

}  // namespace

extern "C" {

const char *mecdf_strerror(int code) {
    switch (code) {
    case MECDF_OK:
        return "success";
    case MECDF_EINVAL:
        return "invalid argument";
    case MECDF_ENOMEM:
        return "out of device memory or over the workspace limit";
    case MECDF_EDEVICE:
        return "HIP runtime error";
    case MECDF_EUNSUPPORTED:
        return "unsupported size or option";
    default:
        return "unknown error code";
    }
}

const char *mecdf_last_error(void) { return mecdf::last_error(); }

int ecdf_grid(int d, int64_t N, const double *x, const void *y,
              const int64_t *M, const double *z, void *F, int prec,
              void *stream) {
    if (F == nullptr)
        return fail(MECDF_EINVAL, "F is NULL");
    return grid_entry(d, N, x, y, M, z, F, nullptr, prec, stream);
}

int esf_grid(int d, int64_t N, const double *x, const void *y,
             const int64_t *M, const double *z, void *Fbar, int prec,
             void *stream) {
    if (Fbar == nullptr)
        return fail(MECDF_EINVAL, "Fbar is NULL");
    return grid_entry(d, N, x, y, M, z, nullptr, Fbar, prec, stream);
}

int ecdf_esf_grid(int d, int64_t N, const double *x, const void *y,
                  const int64_t *M, const double *z, void *F, void *Fbar,
                  int prec, void *stream) {
    return grid_entry(d, N, x, y, M, z, F, Fbar, prec, stream);
}

int ecdf_points(int d, int64_t N, const double *x, const void *y, void *F,
                int prec, void *stream) {
    MECDF_TRY(check_common(d, N, x, prec, MECDF_MAX_DIM));
    if (F == nullptr && N > 0)
        return fail(MECDF_EINVAL, "F is NULL");
    if (y != nullptr && N == 0)
        return fail(MECDF_EINVAL, "weighted ECDF needs N >= 1");
    if (N == 0)
        return MECDF_OK;
    return points_run(d, N, x, y, F, 0, prec, (hipStream_t)stream);
}

int esf_points(int d, int64_t N, const double *x, const void *y, void *F,
               int prec, void *stream) {
    MECDF_TRY(check_common(d, N, x, prec, MECDF_MAX_DIM));
    if (F == nullptr && N > 0)
        return fail(MECDF_EINVAL, "F is NULL");
    if (y != nullptr && N == 0)
        return fail(MECDF_EINVAL, "weighted ESF needs N >= 1");
    if (N == 0)
        return MECDF_OK;
    return points_run(d, N, x, y, F, 1, prec, (hipStream_t)stream);
}

static int kde_check(int d, int64_t N, const double *x, int nh,
                     const double *h, void *out, double *score, int prec) {
    MECDF_TRY(check_common(d, N, x, prec, 3));
    if (N < 2)
        return fail(MECDF_EINVAL, "kernel sums at the points need N >= 2");
    if (nh < 1 || nh > 256)
        return fail(MECDF_EINVAL, "nh must be in 1..256");
    if (h == nullptr)
        return fail(MECDF_EINVAL, "h is NULL");
    for (int i = 0; i < nh * d; ++i)
        if (!(h[i] > 0.0) || !std::isfinite(h[i]))
            return fail(MECDF_EINVAL, "bandwidths must be positive and finite");
    if (out == nullptr && score == nullptr)
        return fail(MECDF_EINVAL, "no output requested");
    return MECDF_OK;
}

int kde_laplace(int d, int64_t N, const double *x, const void *w, int nh,
                const double *h, void *f, double *lcv, int prec, void *stream) {
    MECDF_TRY(kde_check(d, N, x, nh, h, f, lcv, prec));
    return kde_run(d, N, x, w, nh, h, f, lcv, 0, prec, (hipStream_t)stream);
}

int kreg_laplace(int d, int64_t N, const double *x, const void *y, int nh,
                 const double *h, void *m, double *cv, int prec, void *stream) {
    MECDF_TRY(kde_check(d, N, x, nh, h, m, cv, prec));
    if (y == nullptr)
        return fail(MECDF_EINVAL, "y is NULL");
    return kde_run(d, N, x, y, nh, h, m, cv, 1, prec, (hipStream_t)stream);
}

void mecdf_release(void) { mecdf::workspace_release_all(); }

}  // extern "C"
