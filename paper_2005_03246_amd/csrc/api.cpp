// C ABI of libmecdf: argument validation and dispatch (see include/mecdf.h).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <string>
#include <vector>

#include "common.hpp"

namespace mecdf {
int grid_run(int d, int64_t N, const double *x, const void *y,
             const int64_t *M, const double *z, void *F, void *Fbar, int prec,
             hipStream_t s);
int points_delta_run(int d, int64_t N, const double *x, const void *y, int64_t Q,
                     const double *z, const uint8_t *delta, void *F, int prec, hipStream_t s);
int kde_uniform_run(int d, int64_t N, const double *x, const void *w, int64_t Q,
                    const double *z, int nh, const double *h, void *f, int prec,
                    hipStream_t s);
int points_run(int d, int64_t N, const double *x, const void *y, void *F,
               int survival, int prec, hipStream_t s);
int kde_run(int d, int64_t N, const double *x, const void *w, int nh,
            const double *h, void *f, double *score, int regression,
            int prec, hipStream_t s);
int bw_features(const mecdf_dataset *sets, int nsets, float *feat, hipStream_t s);
int mlp_forward(int B, const float *X, const float *P, float *out, hipStream_t s);
int mlp_grad(int B, const float *X, const float *T, const float *P, float *G, float *loss,
             hipStream_t s);
int mlp_train(int B, const float *X, const float *T, float *P, float *adam, int steps,
              float lr, float wd, float *losses, hipStream_t s);
int mlp_init(uint64_t seed, float *P, float *adam, hipStream_t s);
int bw_train_steps(int B, const float *feat, const int *label, int nhg, const double *hgrid,
                   int steps, float lr, float wd, float *P, float *adam, float *losses,
                   int64_t t0, hipStream_t s);
int lcv_argmax(const double *score, const int *cnt, int nsets, int *best, hipStream_t s);
int batch_lcv(const mecdf_dataset *sets, int nsets, const int *nh, const double *h,
              double *lcv, int *best, int prec, int force, hipStream_t s);
int lcv_plan_create(const mecdf_dataset *sets, int nsets, const int *nh, const double *h,
                    double *lcv, int *best, int prec, void **out);
int lcv_plan_run(void *plan, hipStream_t s);
void lcv_plan_destroy(void *plan);
int autotune(const char *path, hipStream_t s);
int tuning_info(int64_t *queue_max, char *source, int cap);
int tuning_set(const int64_t *queue_max);
int grid_interp(int d, const int64_t *M, const double *z, const void *G, int64_t Q,
                const double *q, void *out, int prec, hipStream_t s);
int gridkde_run(int d, int64_t N, const double *x, const void *w, const int64_t *M,
                const double *z, int nh, const double *h, void *out, int regression,
                int matern, int prec, hipStream_t s);
int kde_matrix_run(int d, int64_t N, const double *x, const void *w, int nh, const double *H,
                   void *f, double *score, int regression, int prec, hipStream_t s);
int loclin_run(int d, int64_t N, const double *x, const void *y, int nh, const double *h,
               void *m, int prec, hipStream_t s);
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

// per-axis node counts >= 1 (at most max_m), finite strictly increasing nodes
int check_nodes(int d, const int64_t *M, const double *z, int64_t max_m) {
    if (M == nullptr || z == nullptr)
        return fail(MECDF_EINVAL, "grid sizes M and nodes z are required");
    int64_t off = 0;
    for (int k = 0; k < d; ++k) {
        if (M[k] < 1)
            return fail(MECDF_EINVAL, "grid size M_k must be >= 1");
        if (M[k] > max_m)
            return fail(MECDF_EUNSUPPORTED, "grid size M_k too large");
        for (int64_t j = 0; j < M[k]; ++j) {
            double v = z[off + j];
            if (!std::isfinite(v))
                return fail(MECDF_EINVAL, "grid nodes must be finite");
            if (j > 0 && !(z[off + j - 1] < v))
                return fail(MECDF_EINVAL, "grid nodes must be strictly increasing per axis");
        }
        off += M[k];
    }
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
    case MECDF_EIO:
        return "file input/output error";
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

int ecdf_esf_grid_noalloc(int d, int64_t N, const double *x, const void *y,
                          const int64_t *M, const double *z, void *F, void *Fbar,
                          int prec, void *stream) {
    void *ws = nullptr;
    size_t cap = 0;
    MECDF_TRY(noalloc_scratch(&ws, &cap));
    FixedWorkspace fixed(ws, cap);
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

int ecdf_delta_at(int d, int64_t N, const double *x, const void *y, int64_t Q,
                  const double *z, const uint8_t *delta, void *F, int prec, void *stream) {
    MECDF_TRY(check_common(d, N, x, prec, MECDF_MAX_DIM));
    if (N < 1)
        return fail(MECDF_EINVAL, "queries at arbitrary points need N >= 1");
    if (Q < 0)
        return fail(MECDF_EINVAL, "Q must be >= 0");
    if (Q == 0)
        return MECDF_OK;
    if (z == nullptr || F == nullptr)
        return fail(MECDF_EINVAL, "z and F are required");
    return points_delta_run(d, N, x, y, Q, z, delta, F, prec, (hipStream_t)stream);
}

int kde_uniform(int d, int64_t N, const double *x, const void *w, int64_t Q,
                const double *z, int nh, const double *h, void *f, int prec, void *stream) {
    MECDF_TRY(check_common(d, N, x, prec, MECDF_MAX_DIM));
    if (N < 1)
        return fail(MECDF_EINVAL, "the uniform kernel sums need N >= 1");
    if (Q < 0)
        return fail(MECDF_EINVAL, "Q must be >= 0");
    if (nh < 1 || nh > 256)
        return fail(MECDF_EINVAL, "nh must be in 1..256");
    if (h == nullptr)
        return fail(MECDF_EINVAL, "h is NULL");
    for (int i = 0; i < nh * d; ++i)
        if (!(h[i] > 0.0) || !std::isfinite(h[i]))
            return fail(MECDF_EINVAL, "bandwidths must be positive and finite");
    if (Q == 0)
        return MECDF_OK;
    if (z == nullptr || f == nullptr)
        return fail(MECDF_EINVAL, "z and f are required");
    if (Q > ((int64_t(1) << 26) >> d))
        return fail(MECDF_EUNSUPPORTED, "the uniform kernel sums take Q <= 2^26 / 2^d");
    return kde_uniform_run(d, N, x, w, Q, z, nh, h, f, prec, (hipStream_t)stream);
}

static int kde_check(int d, int64_t N, const double *x, int nh,
                     const double *h, void *out, double *score, int prec) {
    MECDF_TRY(check_common(d, N, x, prec, MECDF_MAX_DIM));
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

static int check_sets(const mecdf_dataset *sets, int nsets) {
    if (nsets < 1 || sets == nullptr)
        return fail(MECDF_EINVAL, "need at least one dataset");
    for (int i = 0; i < nsets; ++i) {
        if (sets[i].d < 1 || sets[i].d > 3)
            return fail(MECDF_EINVAL, "dataset dimension must be 1..3");
        if (sets[i].N < 2 || sets[i].x == nullptr)
            return fail(MECDF_EINVAL, "datasets need N >= 2 points");
        // the kernel-sum limits, checked for every dataset before any is run
        if (sets[i].N > (int64_t(1) << 28) || (sets[i].d == 3 && sets[i].N > (int64_t(1) << 24)))
            return fail(MECDF_EUNSUPPORTED,
                        "dataset too large: kernel sums support N <= 2^28 (2^24 for d = 3)");
    }
    return MECDF_OK;
}

static int check_batch(const mecdf_dataset *sets, int nsets, const int *nh, const double *h,
                       const double *lcv) {
    MECDF_TRY(check_sets(sets, nsets));
    if (nh == nullptr || h == nullptr || lcv == nullptr)
        return fail(MECDF_EINVAL, "nh, h and lcv are required");
    int64_t off = 0;
    for (int i = 0; i < nsets; ++i) {
        if (nh[i] < 0 || nh[i] > 256)
            return fail(MECDF_EINVAL, "nh must be in 0..256 per dataset");
        for (int b = 0; b < nh[i]; ++b)
            if (!(h[off + b] > 0.0) || !std::isfinite(h[off + b]))
                return fail(MECDF_EINVAL, "bandwidths must be positive and finite");
        off += nh[i];
    }
    return MECDF_OK;
}

int mecdf_kde_lcv_batched(const mecdf_dataset *sets, int nsets, const int *nh,
                          const double *h, double *lcv, int *best, int prec, void *stream) {
    MECDF_TRY(check_batch(sets, nsets, nh, h, lcv));
    if (prec != MECDF_F64 && prec != MECDF_F32C)
        return fail(MECDF_EINVAL, "prec must be MECDF_F64 or MECDF_F32C");
    return batch_lcv(sets, nsets, nh, h, lcv, best, prec, -1, (hipStream_t)stream);
}

int mecdf_lcv_plan_create(const mecdf_dataset *sets, int nsets, const int *nh,
                          const double *h, double *lcv, int *best, int prec,
                          mecdf_lcv_plan *plan) {
    if (plan == nullptr)
        return fail(MECDF_EINVAL, "plan is NULL");
    *plan = nullptr;
    MECDF_TRY(check_batch(sets, nsets, nh, h, lcv));
    if (prec != MECDF_F64 && prec != MECDF_F32C)
        return fail(MECDF_EINVAL, "prec must be MECDF_F64 or MECDF_F32C");
    void *p = nullptr;
    MECDF_TRY(lcv_plan_create(sets, nsets, nh, h, lcv, best, prec, &p));
    *plan = (mecdf_lcv_plan)p;
    return MECDF_OK;
}

int mecdf_lcv_plan_run(mecdf_lcv_plan plan, void *stream) {
    if (plan == nullptr)
        return fail(MECDF_EINVAL, "plan is NULL");
    return lcv_plan_run((void *)plan, (hipStream_t)stream);
}

void mecdf_lcv_plan_destroy(mecdf_lcv_plan plan) {
    if (plan)
        lcv_plan_destroy((void *)plan);
}

int mecdf_autotune(const char *path, void *stream) {
    return autotune(path, (hipStream_t)stream);
}

int mecdf_tuning(int64_t *queue_max_n, char *source, int cap) {
    return tuning_info(queue_max_n, source, cap);
}

int mecdf_tuning_set(const int64_t *queue_max_n) {
    if (queue_max_n == nullptr)
        return fail(MECDF_EINVAL, "queue_max_n is NULL");
    return tuning_set(queue_max_n);
}

int mecdf_bw_features(const mecdf_dataset *sets, int nsets, float *feat, void *stream) {
    MECDF_TRY(check_sets(sets, nsets));
    if (feat == nullptr)
        return fail(MECDF_EINVAL, "feat is NULL");
    return bw_features(sets, nsets, feat, (hipStream_t)stream);
}

int mecdf_mlp_forward(int B, const float *feat, const float *params, float *out,
                      void *stream) {
    if (B < 1 || !feat || !params || !out)
        return fail(MECDF_EINVAL, "mlp_forward: bad arguments");
    return mlp_forward(B, feat, params, out, (hipStream_t)stream);
}

int mecdf_mlp_grad(int B, const float *feat, const float *target, const float *params,
                   float *grad, float *loss, void *stream) {
    if (B < 1 || !feat || !target || !params || !grad)
        return fail(MECDF_EINVAL, "mlp_grad: bad arguments");
    return mlp_grad(B, feat, target, params, grad, loss, (hipStream_t)stream);
}

int mecdf_mlp_train(int B, const float *feat, const float *target, float *params,
                    float *adam, int steps, float lr, float wd, float *losses, void *stream) {
    if (B < 1 || !feat || !target || !params || !adam || steps < 0 || !(lr > 0.f) ||
        !(wd >= 0.f))
        return fail(MECDF_EINVAL, "mlp_train: bad arguments");
    return mlp_train(B, feat, target, params, adam, steps, lr, wd, losses,
                     (hipStream_t)stream);
}

// ------------------------------------------------------------ checkpoints
// File layout (host byte order): "MECDFBW1", uint32 version (1), uint32
// parameter count, uint64 seed, int64 step count, float parameters, float
// Adam moments (first, then second), uint64 FNV-1a hash of everything before
// it.  Written to "<path>.tmp" and renamed over the path.
namespace {
const char kCkptMagic[8] = {'M', 'E', 'C', 'D', 'F', 'B', 'W', '1'};

uint64_t fnv1a(const unsigned char *p, size_t n, uint64_t h = 0xcbf29ce484222325ull) {
    for (size_t i = 0; i < n; ++i) {
        h ^= p[i];
        h *= 0x100000001b3ull;
    }
    return h;
}

struct CkptHeader {
    char magic[8];
    uint32_t version, nparams;
    uint64_t seed;
    int64_t step;
};

int ckpt_write(const char *path, uint64_t seed, int64_t step, const std::vector<float> &p,
               const std::vector<float> &m) {
    CkptHeader h;
    std::memcpy(h.magic, kCkptMagic, 8);
    h.version = 1;
    h.nparams = (uint32_t)p.size();
    h.seed = seed;
    h.step = step;
    uint64_t hash = fnv1a((const unsigned char *)&h, sizeof(h));
    hash = fnv1a((const unsigned char *)p.data(), sizeof(float) * p.size(), hash);
    hash = fnv1a((const unsigned char *)m.data(), sizeof(float) * m.size(), hash);
    const std::string tmp = std::string(path) + ".tmp";
    FILE *f = std::fopen(tmp.c_str(), "wb");
    if (!f)
        return fail(MECDF_EIO, std::string("checkpoint: cannot write ") + tmp);
    bool ok = std::fwrite(&h, sizeof(h), 1, f) == 1 &&
              std::fwrite(p.data(), sizeof(float), p.size(), f) == p.size() &&
              std::fwrite(m.data(), sizeof(float), m.size(), f) == m.size() &&
              std::fwrite(&hash, sizeof(hash), 1, f) == 1;
    ok = (std::fclose(f) == 0) && ok;
    if (!ok || std::rename(tmp.c_str(), path) != 0) {
        std::remove(tmp.c_str());
        return fail(MECDF_EIO, std::string("checkpoint: writing ") + path + " failed");
    }
    return MECDF_OK;
}

// found = false when the file does not exist; a file that exists must be whole
int ckpt_read(const char *path, uint64_t seed, std::vector<float> &p, std::vector<float> &m,
              int64_t &step, bool &found) {
    found = false;
    FILE *f = std::fopen(path, "rb");
    if (!f)
        return MECDF_OK;
    CkptHeader h;
    uint64_t hash = 0;
    bool ok = std::fread(&h, sizeof(h), 1, f) == 1 && std::memcmp(h.magic, kCkptMagic, 8) == 0 &&
              h.version == 1 && h.nparams == (uint32_t)p.size();
    ok = ok && std::fread(p.data(), sizeof(float), p.size(), f) == p.size() &&
         std::fread(m.data(), sizeof(float), m.size(), f) == m.size() &&
         std::fread(&hash, sizeof(hash), 1, f) == 1;
    std::fclose(f);
    if (ok) {
        uint64_t want = fnv1a((const unsigned char *)&h, sizeof(h));
        want = fnv1a((const unsigned char *)p.data(), sizeof(float) * p.size(), want);
        want = fnv1a((const unsigned char *)m.data(), sizeof(float) * m.size(), want);
        ok = want == hash;
    }
    if (!ok)
        return fail(MECDF_EIO, std::string("checkpoint: ") + path +
                                   " is not a whole bandwidth-network checkpoint");
    if (h.seed != seed)
        return fail(MECDF_EINVAL, std::string("checkpoint: ") + path +
                                      " was written with another seed");
    if (h.step < 0)
        return fail(MECDF_EIO, std::string("checkpoint: ") + path + " has a negative step count");
    step = h.step;
    found = true;
    return MECDF_OK;
}

bool grid_ok(int nhg, const double *hgrid) {
    if (nhg < 1 || hgrid == nullptr)
        return false;
    for (int j = 0; j < nhg; ++j)
        if (!(hgrid[j] > 0.0) || !std::isfinite(hgrid[j]) || (j > 0 && !(hgrid[j] > hgrid[j - 1])))
            return false;
    return true;
}
}  // namespace

int mecdf_bw_train(int B, const float *feat, const int *label, int nhg, const double *hgrid,
                   int steps, float lr, float wd, uint64_t seed, float *params, float *adam,
                   float *losses, const char *checkpoint, int64_t *step, void *stream) {
    if (B < 1 || !feat || !label || !params || !adam || !step || steps < 0 || !(lr > 0.f) ||
        !(wd >= 0.f) || !std::isfinite(lr) || !std::isfinite(wd) || *step < 0)
        return fail(MECDF_EINVAL, "bw_train: bad arguments");
    if (!grid_ok(nhg, hgrid))
        return fail(MECDF_EINVAL, "bw_train: hgrid must be positive, finite and ascending");
    hipStream_t s = (hipStream_t)stream;
    std::vector<int> hl((size_t)B);
    MECDF_TRY_HIP(hipMemcpyAsync(hl.data(), label, sizeof(int) * (size_t)B,
                                 hipMemcpyDeviceToHost, s));
    MECDF_TRY_HIP(hipStreamSynchronize(s));
    for (int r = 0; r < B; ++r)
        if (hl[r] < 0 || hl[r] >= nhg)
            return fail(MECDF_EINVAL, "bw_train: a label is outside the bandwidth grid");
    int64_t t0 = *step;
    bool found = false;
    if (checkpoint) {
        std::vector<float> p(MECDF_MLP_PARAMS), m(2 * (size_t)MECDF_MLP_PARAMS);
        int64_t fs = 0;
        MECDF_TRY(ckpt_read(checkpoint, seed, p, m, fs, found));
        if (found) {
            MECDF_TRY_HIP(hipMemcpyAsync(params, p.data(), sizeof(float) * p.size(),
                                         hipMemcpyHostToDevice, s));
            MECDF_TRY_HIP(hipMemcpyAsync(adam, m.data(), sizeof(float) * m.size(),
                                         hipMemcpyHostToDevice, s));
            MECDF_TRY_HIP(hipStreamSynchronize(s));  // p and m go out of scope
            t0 = fs;
        }
    }
    if (!found && t0 == 0)
        MECDF_TRY(mlp_init(seed, params, adam, s));
    MECDF_TRY(bw_train_steps(B, feat, label, nhg, hgrid, steps, lr, wd, params, adam, losses, t0,
                             s));
    *step = t0 + steps;
    if (checkpoint) {
        std::vector<float> p(MECDF_MLP_PARAMS), m(2 * (size_t)MECDF_MLP_PARAMS);
        MECDF_TRY_HIP(hipMemcpyAsync(p.data(), params, sizeof(float) * p.size(),
                                     hipMemcpyDeviceToHost, s));
        MECDF_TRY_HIP(hipMemcpyAsync(m.data(), adam, sizeof(float) * m.size(),
                                     hipMemcpyDeviceToHost, s));
        MECDF_TRY_HIP(hipStreamSynchronize(s));
        MECDF_TRY(ckpt_write(checkpoint, seed, *step, p, m));
    }
    return MECDF_OK;
}

int mecdf_bw_select(const mecdf_dataset *sets, int nsets, const float *params, int nhg,
                    const double *hgrid, int mode, int *hidx_out, double *lcv_out,
                    int *evals_out, void *stream) {
    MECDF_TRY(check_sets(sets, nsets));
    if (!params || !hidx_out || (mode != MECDF_BW_EXTEND && mode != MECDF_BW_WINDOW) ||
        nhg > 4096 || !grid_ok(nhg, hgrid))
        return fail(MECDF_EINVAL, "bw_select: bad arguments");
    hipStream_t s = (hipStream_t)stream;
    // device buffers of this call (outside the shared workspace, which the
    // batched scores below reuse)
    float *feat = nullptr, *pred = nullptr;
    double *scd = nullptr;
    MECDF_TRY_HIP(hipMalloc(&feat, sizeof(float) * 32 * nsets));
    hipError_t e1 = hipMalloc(&pred, sizeof(float) * nsets);
    hipError_t e2 = hipMalloc(&scd, sizeof(double) * 4 * (size_t)nsets);
    auto cleanup = [&]() {
        (void)hipFree(feat);
        (void)hipFree(pred);
        (void)hipFree(scd);
    };
    if (e1 != hipSuccess || e2 != hipSuccess) {
        cleanup();
        return fail(MECDF_ENOMEM, "bw_select: allocation failed");
    }
    int rc = bw_features(sets, nsets, feat, s);
    if (rc == MECDF_OK)
        rc = mlp_forward(nsets, feat, params, pred, s);
    std::vector<float> hf((size_t)32 * nsets), hp(nsets);
    if (rc == MECDF_OK &&
        (hipMemcpyAsync(hf.data(), feat, sizeof(float) * 32 * nsets, hipMemcpyDeviceToHost, s) !=
             hipSuccess ||
         hipMemcpyAsync(hp.data(), pred, sizeof(float) * nsets, hipMemcpyDeviceToHost, s) !=
             hipSuccess ||
         hipStreamSynchronize(s) != hipSuccess))
        rc = fail(MECDF_EDEVICE, "bw_select: copy failed");
    if (rc != MECDF_OK) {
        cleanup();
        return rc;
    }
    const double l0 = std::log(hgrid[0]);
    const double dl = nhg > 1 ? (std::log(hgrid[nhg - 1]) - l0) / (nhg - 1) : 1.0;
    const int w = nhg < 4 ? nhg : 4;
    // per dataset: the evaluated range [lo, hi] of grid indices, the scores
    // there (host copy), the best index
    std::vector<int> lo(nsets), hi(nsets), best(nsets), evals(nsets, 0);
    std::vector<std::vector<double>> sc(nsets, std::vector<double>(nhg, 0.0));
    // the next batch: per dataset its first grid index and count (0: none)
    std::vector<int> b0(nsets), bn(nsets);
    for (int i = 0; i < nsets; ++i) {
        const double lh = (double)hf[(size_t)i * 32 + 12] + (double)hp[i];
        double jf = std::isfinite(lh) ? (lh - l0) / dl : 0.0;
        jf = jf < -1e6 ? -1e6 : (jf > 1e6 ? 1e6 : jf);
        // the four grid points nearest the proposal: round(jf) - 2 .. round(jf) + 1
        int j0 = (int)std::lround(jf) - 2;
        if (j0 > nhg - w)
            j0 = nhg - w;
        if (j0 < 0)
            j0 = 0;
        b0[i] = j0;
        bn[i] = w;
        lo[i] = j0;
        hi[i] = j0 + w - 1;
    }
    std::vector<double> hl, got;
    for (;;) {
        // one batched evaluation of every dataset's pending bandwidths
        hl.clear();
        for (int i = 0; i < nsets; ++i)
            for (int b = 0; b < bn[i]; ++b)
                hl.push_back(hgrid[b0[i] + b]);
        if (hl.empty())
            break;
        rc = batch_lcv(sets, nsets, bn.data(), hl.data(), scd, nullptr, MECDF_F64, -1, s);
        got.resize(hl.size());
        if (rc == MECDF_OK &&
            (hipMemcpyAsync(got.data(), scd, sizeof(double) * got.size(), hipMemcpyDeviceToHost,
                            s) != hipSuccess ||
             hipStreamSynchronize(s) != hipSuccess))
            rc = fail(MECDF_EDEVICE, "bw_select: copy failed");
        if (rc != MECDF_OK)
            break;
        size_t k = 0;
        for (int i = 0; i < nsets; ++i) {
            for (int b = 0; b < bn[i]; ++b)
                sc[i][b0[i] + b] = got[k++];
            evals[i] += bn[i];
            lo[i] = std::min(lo[i], b0[i]);
            hi[i] = std::max(hi[i], b0[i] + bn[i] - 1);
            int bi = lo[i];
            for (int j = lo[i]; j <= hi[i]; ++j)
                if (sc[i][j] > sc[i][bi])
                    bi = j;
            best[i] = bi;
            bn[i] = 0;
            if (mode == MECDF_BW_EXTEND) {
                // widen towards the best score until it is interior
                if (bi == lo[i] && lo[i] > 0) {
                    b0[i] = lo[i] - 4 > 0 ? lo[i] - 4 : 0;
                    bn[i] = lo[i] - b0[i];
                } else if (bi == hi[i] && hi[i] < nhg - 1) {
                    b0[i] = hi[i] + 1;
                    bn[i] = hi[i] + 4 < nhg - 1 ? 4 : nhg - 1 - hi[i];
                }
            }
        }
    }
    cleanup();
    MECDF_TRY(rc);
    for (int i = 0; i < nsets; ++i) {
        hidx_out[i] = best[i];
        if (lcv_out)
            lcv_out[i] = sc[i][best[i]];
        if (evals_out)
            evals_out[i] = evals[i];
    }
    return MECDF_OK;
}

static int check_matrices(int d, int nh, const double *H) {
    if (nh < 1 || nh > 256)
        return fail(MECDF_EINVAL, "nh must be in 1..256");
    if (H == nullptr)
        return fail(MECDF_EINVAL, "H is NULL");
    for (int i = 0; i < nh * d * d; ++i)
        if (!std::isfinite(H[i]))
            return fail(MECDF_EINVAL, "bandwidth matrices must be finite");
    return MECDF_OK;
}

int kde_laplace_H(int d, int64_t N, const double *x, const void *w, int nh, const double *H,
                  void *f, double *lcv, int prec, void *stream) {
    MECDF_TRY(check_common(d, N, x, prec, MECDF_MAX_DIM));
    if (N < 2)
        return fail(MECDF_EINVAL, "kernel sums at the points need N >= 2");
    MECDF_TRY(check_matrices(d, nh, H));
    if (f == nullptr && lcv == nullptr)
        return fail(MECDF_EINVAL, "no output requested");
    return kde_matrix_run(d, N, x, w, nh, H, f, lcv, 0, prec, (hipStream_t)stream);
}

int kreg_laplace_H(int d, int64_t N, const double *x, const void *y, int nh, const double *H,
                   void *m, double *cv, int prec, void *stream) {
    MECDF_TRY(check_common(d, N, x, prec, MECDF_MAX_DIM));
    if (N < 2)
        return fail(MECDF_EINVAL, "kernel sums at the points need N >= 2");
    MECDF_TRY(check_matrices(d, nh, H));
    if (y == nullptr)
        return fail(MECDF_EINVAL, "y is NULL");
    if (m == nullptr && cv == nullptr)
        return fail(MECDF_EINVAL, "no output requested");
    return kde_matrix_run(d, N, x, y, nh, H, m, cv, 1, prec, (hipStream_t)stream);
}

int kreg_loclin_laplace(int d, int64_t N, const double *x, const void *y, int nh,
                        const double *h, void *m, int prec, void *stream) {
    MECDF_TRY(kde_check(d, N, x, nh, h, m, nullptr, prec));
    if (y == nullptr)
        return fail(MECDF_EINVAL, "y is NULL");
    if (m == nullptr)
        return fail(MECDF_EINVAL, "m is NULL");
    return loclin_run(d, N, x, y, nh, h, m, prec, (hipStream_t)stream);
}

static int gridkde_check(int d, int64_t N, const double *x, const int64_t *M, const double *z,
                         int nh, const double *h, void *out, int prec, int matern) {
    MECDF_TRY(check_common(d, N, x, prec, MECDF_MAX_DIM));
    if (N < 1)
        return fail(MECDF_EINVAL, "grid kernel sums need N >= 1");
    if (nh < 1 || nh > 256)
        return fail(MECDF_EINVAL, "nh must be in 1..256");
    if (h == nullptr || out == nullptr)
        return fail(MECDF_EINVAL, "h and the output are required");
    for (int i = 0; i < nh * d; ++i)
        if (!(h[i] > 0.0) || !std::isfinite(h[i]))
            return fail(MECDF_EINVAL, "bandwidths must be positive and finite");
    MECDF_TRY(check_nodes(d, M, z, int64_t(1) << 24));
    double cells = 1.0, nodes = 1.0;
    for (int k = 0; k < d; ++k) {
        cells *= (double)(M[k] + 1);
        nodes *= (double)M[k];
    }
    if (cells >= 2147483647.0)
        return fail(MECDF_EUNSUPPORTED, "grid has 2^31 - 1 or more cells");
    // the corner arrays and their half-size scan outputs, two values each
    const double slots = matern ? (double)(1 + d) : 1.0;
    if (nodes * 1.5 * (double)(1 << d) * slots * 2.0 * 8.0 > 64e9)
        return fail(MECDF_EUNSUPPORTED, "grid too large for the 2^d channel arrays");
    return MECDF_OK;
}

int kde_laplace_grid(int d, int64_t N, const double *x, const void *w, const int64_t *M,
                     const double *z, int nh, const double *h, void *f, int prec,
                     void *stream) {
    MECDF_TRY(gridkde_check(d, N, x, M, z, nh, h, f, prec, 0));
    return gridkde_run(d, N, x, w, M, z, nh, h, f, 0, 0, prec, (hipStream_t)stream);
}

int kreg_laplace_grid(int d, int64_t N, const double *x, const void *y, const int64_t *M,
                      const double *z, int nh, const double *h, void *m, int prec,
                      void *stream) {
    MECDF_TRY(gridkde_check(d, N, x, M, z, nh, h, m, prec, 0));
    if (y == nullptr)
        return fail(MECDF_EINVAL, "y is NULL");
    return gridkde_run(d, N, x, y, M, z, nh, h, m, 1, 0, prec, (hipStream_t)stream);
}

int kde_matern32_grid(int d, int64_t N, const double *x, const void *w, const int64_t *M,
                      const double *z, int nh, const double *h, void *f, int prec,
                      void *stream) {
    MECDF_TRY(gridkde_check(d, N, x, M, z, nh, h, f, prec, 1));
    return gridkde_run(d, N, x, w, M, z, nh, h, f, 0, 1, prec, (hipStream_t)stream);
}

int kreg_matern32_grid(int d, int64_t N, const double *x, const void *y, const int64_t *M,
                       const double *z, int nh, const double *h, void *m, int prec,
                       void *stream) {
    MECDF_TRY(gridkde_check(d, N, x, M, z, nh, h, m, prec, 1));
    if (y == nullptr)
        return fail(MECDF_EINVAL, "y is NULL");
    return gridkde_run(d, N, x, y, M, z, nh, h, m, 1, 1, prec, (hipStream_t)stream);
}

int mecdf_grid_interp(int d, const int64_t *M, const double *z, const void *G, int64_t Q,
                      const double *q, void *out, int prec, void *stream) {
    if (d < 1 || d > MECDF_MAX_DIM)
        return fail(MECDF_EINVAL, "d must be in 1.." + std::to_string(MECDF_MAX_DIM));
    if (prec != MECDF_F64 && prec != MECDF_F32C)
        return fail(MECDF_EINVAL, "prec must be MECDF_F64 or MECDF_F32C");
    if (Q < 0)
        return fail(MECDF_EINVAL, "Q must be >= 0");
    if (Q >= (int64_t(1) << 40))
        return fail(MECDF_EUNSUPPORTED, "Q too large");
    MECDF_TRY(check_nodes(d, M, z, int64_t(1) << 24));
    if (Q > 0 && (G == nullptr || q == nullptr || out == nullptr))
        return fail(MECDF_EINVAL, "G, q and out are required");
    return grid_interp(d, M, z, G, Q, q, out, prec, (hipStream_t)stream);
}

void mecdf_release(void) { mecdf::workspace_release_all(); }

}  // extern "C"
