// Batched likelihood cross-validation: the leave-one-out log-likelihood score
// of the Laplacian density (eq. (Laplacian_kde_nD), Section 3.1; Section 3.2
// names likelihood cross-validation for this kernel) for many datasets of
// uneven size and dimension, each with its own list of isotropic bandwidths.
//
// Small datasets are all scored by one persistent work-queue launch: a work
// unit is one dataset, 256 of its points as queries and four of its
// bandwidths; each workgroup takes units in turn and sums every other point of
// the dataset into each query's leave-one-out sum relative to its nearest
// point (so the logarithm exists where every kernel term is below the float64
// range), staging the points through LDS; the 256 log terms of a unit are
// added in a fixed tree and the units of a (dataset, bandwidth) in order.
// Larger datasets run the orthant recursion of kde_laplace, spread over a
// few streams beside the caller's so that several run at once.  Which size is "small" is chosen per dimension and precision by an
// autotuner that times both on the device (mecdf_autotune) and keeps its
// choice in a JSON file keyed by the GPU architecture.
//
// A plan (mecdf_lcv_plan_*) records the work queue once into a hipGraph and
// replays it beside the recursions of the larger datasets.
#include <dlfcn.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "common.hpp"
#include "lse.hpp"

namespace mecdf {

int kde_run(int d, int64_t N, const double *x, const void *w, int nh, const double *h,
            void *f, double *score, int regression, int prec, hipStream_t s);
int launch_seg_argmax(const double *score, const int64_t *off, int nsets, int *best,
                      hipStream_t s);
int lcv_argmax(const double *score, const int *cnt, int nsets, int *best, hipStream_t s);

// ------------------------------------------------------------- work queue
constexpr int kQBand = 4;     // bandwidths per work unit
constexpr int kQDim = 3;      // largest dimension of the batched datasets
constexpr int kQueueGroups = 2048;

struct QSet {
    const double *x;  // d * n, x[k * n + i]
    int64_t n;
    int d, nh;
    int64_t hoff;  // first bandwidth (and score) of the dataset in the flat lists
    int64_t u0;    // first work unit
    int64_t p0;    // first partial sum
    int64_t r0;    // first score row among the queued datasets
    int nqb;       // query blocks of 256 points
};

// the last set whose field (u0 or r0) is <= v (sets in increasing order)
__device__ __forceinline__ int qset_find(const QSet *sets, int nsets, int64_t v, bool rows) {
    int lo = 0, hi = nsets - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        const int64_t f = rows ? sets[mid].r0 : sets[mid].u0;
        if (f <= v)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

template <typename T> __device__ __forceinline__ T qexp(T v);
template <> __device__ __forceinline__ double qexp<double>(double v) { return exp(v); }
template <> __device__ __forceinline__ float qexp<float>(float v) { return expf(v); }

// part[p0 + b * nqb + qb] = sum over the 256 queries of block qb of
// log fhat_{-j}(x_j) at bandwidth b (T: the type the exponentials are formed
// in; sums are float64).
template <typename T>
__global__ __launch_bounds__(256) void k_lcv_queue(const QSet *__restrict__ sets, int nsets,
                                                   int64_t nunits, const double *__restrict__ h,
                                                   double *__restrict__ part) {
    __shared__ double sx[kQDim][256];
    __shared__ double red[256];
    __shared__ int s_set;
    const int t = threadIdx.x;
    for (int64_t u = blockIdx.x; u < nunits; u += gridDim.x) {
        if (t == 0)
            s_set = qset_find(sets, nsets, u, false);
        __syncthreads();
        const QSet S = sets[s_set];
        const int64_t w = u - S.u0;
        const int bb = (int)(w / S.nqb), qb = (int)(w - (int64_t)bb * S.nqb);
        const int b0 = bb * kQBand;
        const int nb = S.nh - b0 < kQBand ? S.nh - b0 : kQBand;
        double ih[kQBand], lnorm[kQBand];
#pragma unroll
        for (int b = 0; b < kQBand; ++b) {
            const double hb = h[S.hoff + b0 + (b < nb ? b : nb - 1)];
            ih[b] = 1.0 / hb;
            // log of 1 / (2^d (n - 1) h^d)
            lnorm[b] = -((double)S.d * log(2.0 * hb) + log((double)(S.n - 1)));
        }
        const int64_t j = (int64_t)qb * 256 + t;
        const bool valid = j < S.n;
        double q[kQDim];
#pragma unroll
        for (int k = 0; k < kQDim; ++k)
            q[k] = (valid && k < S.d) ? S.x[(int64_t)k * S.n + j] : 0.0;
        LooAcc<1> acc[kQBand];
#pragma unroll
        for (int b = 0; b < kQBand; ++b)
            loo_init(acc[b]);
        const double one[1] = {1.0};
        for (int64_t t0 = 0; t0 < S.n; t0 += 256) {
            const int64_t i = t0 + t;
            __syncthreads();  // the previous tile has been read
#pragma unroll
            for (int k = 0; k < kQDim; ++k)
                sx[k][t] = (k < S.d && i < S.n) ? S.x[(int64_t)k * S.n + i] : 0.0;
            __syncthreads();
            const int cnt = (S.n - t0) < 256 ? (int)(S.n - t0) : 256;
            for (int v = 0; v < cnt; ++v) {
                if (t0 + v == j)
                    continue;
                // unused coordinates are 0 on both sides
                const double l1 =
                    fabs(sx[0][v] - q[0]) + fabs(sx[1][v] - q[1]) + fabs(sx[2][v] - q[2]);
#pragma unroll
                for (int b = 0; b < kQBand; ++b) {
                    const double e = l1 * ih[b];
                    const T f = qexp<T>((T)(-fabs(e - acc[b].m)));
                    loo_add(acc[b], e, (double)f, one);
                }
            }
        }
#pragma unroll
        for (int b = 0; b < kQBand; ++b) {
            red[t] = (valid && b < nb)
                         ? -acc[b].m + log(acc[b].s[0] + acc[b].c[0]) + lnorm[b]
                         : 0.0;
            __syncthreads();
            for (int off = 128; off > 0; off >>= 1) {
                if (t < off)
                    red[t] += red[t + off];
                __syncthreads();
            }
            if (t == 0 && b < nb)
                part[S.p0 + (int64_t)(b0 + b) * S.nqb + qb] = red[0];
            __syncthreads();
        }
    }
}

// lcv[hoff + b] = (sum over the query blocks, in order) / n, one thread per row
__global__ __launch_bounds__(256) void k_lcv_rows(const QSet *__restrict__ sets, int nsets,
                                                  int64_t nrows, const double *__restrict__ part,
                                                  double *__restrict__ lcv) {
    const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (r >= nrows)
        return;
    const QSet S = sets[qset_find(sets, nsets, r, true)];
    const int64_t b = r - S.r0;
    double sum = 0.0;
    for (int q = 0; q < S.nqb; ++q)
        sum += part[S.p0 + b * S.nqb + q];
    lcv[S.hoff + b] = sum / (double)S.n;
}

// ------------------------------------------------------------- tuning
namespace {
std::mutex g_tune_mu;
bool g_tune_loaded = false;
// largest N scored by the work queue, per precision and dimension 1..3
int64_t g_direct_max[2][kQDim] = {{4096, 2048, 2048}, {8192, 4096, 4096}};
std::string g_tune_source = "built-in defaults";

std::string arch_name() {
    int dev = 0;
    hipDeviceProp_t p;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&p, dev) != hipSuccess)
        return "unknown";
    std::string a = p.gcnArchName;
    const size_t c = a.find(':');
    return c == std::string::npos ? a : a.substr(0, c);
}

std::string default_tune_path() {
    if (const char *e = std::getenv("MECDF_TUNE_FILE"))
        if (*e)
            return e;
    Dl_info info;
    std::string dir = ".";
    if (dladdr((void *)&default_tune_path, &info) && info.dli_fname) {
        dir = info.dli_fname;
        const size_t sl = dir.rfind('/');
        dir = sl == std::string::npos ? "." : dir.substr(0, sl);
    }
    return dir + "/tune_" + arch_name() + ".json";
}

// reads the list of three integers after "key": [ in text, past `after`
bool parse_triple(const std::string &text, const std::string &key, int64_t out[kQDim]) {
    const size_t a = text.find("\"kde_queue_max_n\"");
    if (a == std::string::npos)
        return false;
    const size_t k = text.find("\"" + key + "\"", a);
    if (k == std::string::npos)
        return false;
    const size_t b = text.find('[', k);
    if (b == std::string::npos)
        return false;
    long long v[kQDim];
    if (std::sscanf(text.c_str() + b, "[ %lld , %lld , %lld ]", &v[0], &v[1], &v[2]) != kQDim)
        return false;
    for (int i = 0; i < kQDim; ++i) {
        if (v[i] < 0)
            return false;
        out[i] = v[i];
    }
    return true;
}

void load_tuning_locked() {
    if (g_tune_loaded)
        return;
    g_tune_loaded = true;
    const std::string path = default_tune_path();
    FILE *f = std::fopen(path.c_str(), "rb");
    if (!f)
        return;
    std::string text;
    char buf[4096];
    size_t got;
    while ((got = std::fread(buf, 1, sizeof(buf), f)) > 0)
        text.append(buf, got);
    std::fclose(f);
    if (text.find("\"arch\": \"" + arch_name() + "\"") == std::string::npos)
        return;  // tuned on another GPU
    int64_t a[kQDim], b[kQDim];
    if (parse_triple(text, "f64", a) && parse_triple(text, "f32c", b)) {
        std::memcpy(g_direct_max[0], a, sizeof(a));
        std::memcpy(g_direct_max[1], b, sizeof(b));
        g_tune_source = path;
    }
}
}  // namespace

int64_t queue_max_n(int d, int prec) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_tuning_locked();
    return g_direct_max[prec == MECDF_F32C ? 1 : 0][d - 1];
}

// ------------------------------------------------------------- layout
struct BatchLayout {
    std::vector<QSet> q;     // queued datasets
    std::vector<int> dc;     // datasets for the recursion
    std::vector<int64_t> hoff;
    std::vector<int64_t> off;  // nsets + 1 score offsets
    int64_t nunits = 0, nparts = 0, nrows = 0, nh_total = 0;
};

// force: -1 tuned choice, 0 every dataset to the recursion, 1 every one to the queue
static BatchLayout batch_layout(const mecdf_dataset *sets, int nsets, const int *nh, int prec,
                                int force) {
    BatchLayout L;
    L.off.assign((size_t)nsets + 1, 0);
    for (int i = 0; i < nsets; ++i)
        L.off[i + 1] = L.off[i] + nh[i];
    L.nh_total = L.off[nsets];
    for (int i = 0; i < nsets; ++i) {
        if (nh[i] == 0)
            continue;
        const bool queued = force >= 0 ? force == 1 : sets[i].N <= queue_max_n(sets[i].d, prec);
        if (!queued) {
            L.dc.push_back(i);
            continue;
        }
        QSet qs;
        qs.x = sets[i].x;
        qs.n = sets[i].N;
        qs.d = sets[i].d;
        qs.nh = nh[i];
        qs.hoff = L.off[i];
        qs.nqb = (int)ceil_div(sets[i].N, 256);
        qs.u0 = L.nunits;
        qs.p0 = L.nparts;
        qs.r0 = L.nrows;
        L.nunits += (int64_t)qs.nqb * ceil_div(nh[i], kQBand);
        L.nparts += (int64_t)qs.nqb * nh[i];
        L.nrows += nh[i];
        L.q.push_back(qs);
    }
    return L;
}

// device data of the queue: descriptors, flat bandwidths, partial sums, offsets
struct QueueMem {
    QSet *sets = nullptr;
    double *h = nullptr;
    double *part = nullptr;
    int64_t *off = nullptr;
};

static void queue_plan(ArenaPlan &pl, const BatchLayout &L) {
    pl.add<QSet>(L.q.size() + 1);
    pl.add<double>((size_t)L.nh_total + 1);
    pl.add<double>((size_t)L.nparts + 1);
    pl.add<int64_t>(L.off.size());
}

static QueueMem queue_take(Arena &a, const BatchLayout &L) {
    QueueMem m;
    m.sets = a.take<QSet>(L.q.size() + 1);
    m.h = a.take<double>((size_t)L.nh_total + 1);
    m.part = a.take<double>((size_t)L.nparts + 1);
    m.off = a.take<int64_t>(L.off.size());
    return m;
}

static int queue_launch(const BatchLayout &L, const QueueMem &m, int prec, double *lcv,
                        hipStream_t s) {
    if (L.q.empty())
        return MECDF_OK;
    ProfScope prof("lcv_queue", s);
    const unsigned g = (unsigned)std::min<int64_t>(L.nunits, kQueueGroups);
    if (prec == MECDF_F32C)
        hipLaunchKernelGGL(k_lcv_queue<float>, dim3(g), dim3(256), 0, s, m.sets,
                           (int)L.q.size(), L.nunits, m.h, m.part);
    else
        hipLaunchKernelGGL(k_lcv_queue<double>, dim3(g), dim3(256), 0, s, m.sets,
                           (int)L.q.size(), L.nunits, m.h, m.part);
    hipLaunchKernelGGL(k_lcv_rows, dim3((unsigned)ceil_div(L.nrows, 256)), dim3(256), 0, s,
                       m.sets, (int)L.q.size(), L.nrows, m.part, lcv);
    MECDF_LAUNCH_CHECK();
    return MECDF_OK;
}

// the recursion for one dataset, isotropic bandwidths expanded per axis
static int dc_run(const mecdf_dataset &ds, int nh, const double *h, double *lcv, int prec,
                  hipStream_t s) {
    std::vector<double> hh((size_t)nh * ds.d);
    for (int b = 0; b < nh; ++b)
        for (int k = 0; k < ds.d; ++k)
            hh[(size_t)b * ds.d + k] = h[b];
    return kde_run(ds.d, ds.N, ds.x, nullptr, nh, hh.data(), nullptr, lcv, 0, prec, s);
}

// The recursions of the larger datasets run beside each other, dataset j on
// side stream j mod kSideStreams (each a chain of small launches that leaves
// most of the GPU idle on its own), each stream in its own region of working
// memory, sized for the largest of its datasets.
static int dc_regions(const BatchLayout &L, const mecdf_dataset *sets, const int *nh,
                      const double *h, double *lcv, int prec,
                      size_t (&region)[kSideStreams]) {
    for (int k = 0; k < kSideStreams; ++k)
        region[k] = 0;
    for (size_t j = 0; j < L.dc.size(); ++j) {
        const int i = L.dc[j];
        size_t b = 0;
        set_workspace_sizing(&b);
        const int rc = dc_run(sets[i], nh[i], h + L.off[i], lcv + L.off[i], prec, nullptr);
        set_workspace_sizing(nullptr);
        if (rc != kSizingOnly && rc != MECDF_OK)
            return rc;
        const size_t k = j % kSideStreams;
        region[k] = std::max(region[k], (b + 255) & ~size_t(255));
    }
    return MECDF_OK;
}

static int dc_launch(const std::vector<mecdf_dataset> &sets, const std::vector<int> &nh,
                     const std::vector<const double *> &h, const std::vector<double *> &lcv,
                     int prec, char *const (&base)[kSideStreams],
                     const size_t (&region)[kSideStreams], hipStream_t s) {
    if (sets.empty())
        return MECDF_OK;
    hipStream_t side[kSideStreams];
    MECDF_TRY(side_streams(s, side));
    for (size_t j = 0; j < sets.size(); ++j) {
        const size_t k = j % kSideStreams;
        FixedWorkspace fixed(base[k], region[k]);
        MECDF_TRY(dc_run(sets[j], nh[j], h[j], lcv[j], prec, side[k]));
    }
    return side_streams_join(s);
}

// Eager batch on the caller's stream: the work queue there, the recursions
// on the side streams, joined back before the best indices are taken; the
// library workspace holds the queue's data and the recursions' regions.
int batch_lcv(const mecdf_dataset *sets, int nsets, const int *nh, const double *h,
              double *lcv, int *best, int prec, int force, hipStream_t s) {
    const BatchLayout L = batch_layout(sets, nsets, nh, prec, force);
    size_t region[kSideStreams];
    MECDF_TRY(dc_regions(L, sets, nh, h, lcv, prec, region));
    ArenaPlan pl;
    if (!L.q.empty())
        queue_plan(pl, L);
    for (int k = 0; k < kSideStreams; ++k)
        pl.add<char>(region[k]);
    void *wsb = nullptr;
    MECDF_TRY(workspace_reserve(pl.used, &wsb));
    Arena a;
    a.base = (char *)wsb;
    QueueMem m;
    if (!L.q.empty())
        m = queue_take(a, L);
    char *base[kSideStreams];
    for (int k = 0; k < kSideStreams; ++k)
        base[k] = a.take<char>(region[k]);
    if (!L.q.empty()) {
        MECDF_TRY(upload_small(L.q.data(), sizeof(QSet) * L.q.size(), m.sets, s));
        MECDF_TRY(upload_small(h, sizeof(double) * (size_t)L.nh_total, m.h, s));
        MECDF_TRY(queue_launch(L, m, prec, lcv, s));
    }
    std::vector<mecdf_dataset> ds;
    std::vector<int> dn;
    std::vector<const double *> dh;
    std::vector<double *> dl;
    for (int i : L.dc) {
        ds.push_back(sets[i]);
        dn.push_back(nh[i]);
        dh.push_back(h + L.off[i]);
        dl.push_back(lcv + L.off[i]);
    }
    MECDF_TRY(dc_launch(ds, dn, dh, dl, prec, base, region, s));
    if (best)
        MECDF_TRY(lcv_argmax(lcv, nh, nsets, best, s));
    return MECDF_OK;
}

// ------------------------------------------------------------- graph plan
// A plan keeps everything a batch reads from the host in memory it owns,
// with its own working memory.  The work queue of the small datasets (its
// two kernels) is recorded once into a HIP graph.  A run forks that graph
// onto the plan's side stream, enqueues the recursions of the larger datasets
// on the library's side streams meanwhile (one chain of launches per dataset,
// in the plan's working memory), joins them all and writes the best indices.  The
// recursions are not recorded: one dataset's chain is up to ~6000 launches
// and hundreds of them would make a graph of hundreds of thousands of nodes
// in one dependency chain.
struct LcvPlan {
    int dev = 0;
    void *mem = nullptr;
    hipStream_t side = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    // what a run enqueues besides the graph
    std::vector<mecdf_dataset> dc_sets;
    std::vector<int> dc_nh;
    std::vector<std::vector<double>> dc_h;
    std::vector<double *> dc_lcv;
    char *dc_base[kSideStreams] = {};
    size_t dc_region[kSideStreams] = {};
    int prec = MECDF_F64;
    int nsets = 0;
    double *lcv = nullptr;
    int *best = nullptr;
    int64_t *off = nullptr;
};

static void plan_free(LcvPlan *p) {
    if (!p)
        return;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(p->dev);
    if (p->exec)
        (void)hipGraphExecDestroy(p->exec);
    if (p->graph)
        (void)hipGraphDestroy(p->graph);
    if (p->fork)
        (void)hipEventDestroy(p->fork);
    if (p->join)
        (void)hipEventDestroy(p->join);
    if (p->side)
        (void)hipStreamDestroy(p->side);
    if (p->mem) {
        (void)hipDeviceSynchronize();
        (void)hipFree(p->mem);
    }
    (void)hipSetDevice(cur);
    delete p;
}

static int plan_build(LcvPlan *p, const mecdf_dataset *sets, int nsets, const int *nh,
                      const double *h, double *lcv, int *best, int prec, int force) {
    const BatchLayout L = batch_layout(sets, nsets, nh, prec, force);
    MECDF_TRY(dc_regions(L, sets, nh, h, lcv, prec, p->dc_region));
    ArenaPlan pl;
    queue_plan(pl, L);
    for (int k = 0; k < kSideStreams; ++k)
        pl.add<char>(p->dc_region[k]);
    MECDF_TRY_HIP(hipMalloc(&p->mem, pl.used));
    Arena a;
    a.base = (char *)p->mem;
    const QueueMem m = queue_take(a, L);
    for (int k = 0; k < kSideStreams; ++k)
        p->dc_base[k] = a.take<char>(p->dc_region[k]);
    int rc = MECDF_OK;
    MECDF_TRY_HIP(hipMemcpy(m.sets, L.q.data(), sizeof(QSet) * L.q.size(),
                            hipMemcpyHostToDevice));
    MECDF_TRY_HIP(hipMemcpy(m.h, h, sizeof(double) * (size_t)L.nh_total,
                            hipMemcpyHostToDevice));
    MECDF_TRY_HIP(hipMemcpy(m.off, L.off.data(), sizeof(int64_t) * L.off.size(),
                            hipMemcpyHostToDevice));
    for (int i : L.dc) {
        p->dc_sets.push_back(sets[i]);
        p->dc_nh.push_back(nh[i]);
        p->dc_h.emplace_back(h + L.off[i], h + L.off[i] + nh[i]);
        p->dc_lcv.push_back(lcv + L.off[i]);
    }
    p->prec = prec;
    p->nsets = nsets;
    p->lcv = lcv;
    p->best = best;
    p->off = m.off;
    MECDF_TRY_HIP(hipStreamCreateWithFlags(&p->side, hipStreamNonBlocking));
    MECDF_TRY_HIP(hipEventCreateWithFlags(&p->fork, hipEventDisableTiming));
    MECDF_TRY_HIP(hipEventCreateWithFlags(&p->join, hipEventDisableTiming));
    if (L.q.empty())
        return MECDF_OK;
    // the queue's two kernels, recorded on a private stream
    hipStream_t rec = nullptr;
    MECDF_TRY_HIP(hipStreamCreateWithFlags(&rec, hipStreamNonBlocking));
    const int prof = profiling_enabled() ? 1 : 0;
    (void)mecdf_profile_enable(0);  // no timing events inside the graph
    rc = MECDF_OK;
    hipError_t e = hipStreamBeginCapture(rec, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        rc = queue_launch(L, m, prec, lcv, rec);
        hipError_t e2 = hipStreamEndCapture(rec, &p->graph);
        if (rc == MECDF_OK && e2 != hipSuccess) {
            set_error(std::string("hipStreamEndCapture: ") + hipGetErrorString(e2));
            rc = MECDF_EDEVICE;
        }
    } else {
        set_error(std::string("hipStreamBeginCapture: ") + hipGetErrorString(e));
        rc = MECDF_EDEVICE;
    }
    (void)mecdf_profile_enable(prof);
    (void)hipStreamDestroy(rec);
    MECDF_TRY(rc);
    MECDF_TRY_HIP(hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0));
    return MECDF_OK;
}

int lcv_plan_create(const mecdf_dataset *sets, int nsets, const int *nh, const double *h,
                    double *lcv, int *best, int prec, void **out) {
    LcvPlan *p = new LcvPlan();
    if (hipGetDevice(&p->dev) != hipSuccess) {
        delete p;
        return MECDF_EDEVICE;
    }
    const int rc = plan_build(p, sets, nsets, nh, h, lcv, best, prec, -1);
    if (rc != MECDF_OK) {
        plan_free(p);
        return rc;
    }
    *out = p;
    return MECDF_OK;
}

int lcv_plan_run(void *plan, hipStream_t s) {
    LcvPlan *p = (LcvPlan *)plan;
    if (p->exec) {
        MECDF_TRY_HIP(hipEventRecord(p->fork, s));
        MECDF_TRY_HIP(hipStreamWaitEvent(p->side, p->fork, 0));
        MECDF_TRY_HIP(hipGraphLaunch(p->exec, p->side));
        MECDF_TRY_HIP(hipEventRecord(p->join, p->side));
    }
    {
        std::vector<const double *> dh;
        for (const auto &v : p->dc_h)
            dh.push_back(v.data());
        MECDF_TRY(dc_launch(p->dc_sets, p->dc_nh, dh, p->dc_lcv, p->prec, p->dc_base,
                            p->dc_region, s));
    }
    if (p->exec)
        MECDF_TRY_HIP(hipStreamWaitEvent(s, p->join, 0));
    if (p->best)
        MECDF_TRY(launch_seg_argmax(p->lcv, p->off, p->nsets, p->best, s));
    return MECDF_OK;
}

void lcv_plan_destroy(void *plan) { plan_free((LcvPlan *)plan); }

// ------------------------------------------------------------- autotuner
// Times the queue against the recursion for one synthetic dataset per
// (precision, d, N) on the current device and keeps, per precision and d, the
// largest N up to which the queue was faster at every size.  The sample is a
// seeded normal sample (SplitMix64 + Box-Muller on the device); 64 bandwidths
// from 0.01 to 1.
__global__ void k_tune_sample(double *x, int64_t total, uint64_t seed) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= total)
        return;
    uint64_t z = seed + 0x9e3779b97f4a7c15ull * (uint64_t)(i + 1);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    z ^= z >> 31;
    uint64_t y = z + 0x9e3779b97f4a7c15ull;
    y = (y ^ (y >> 30)) * 0xbf58476d1ce4e5b9ull;
    y = (y ^ (y >> 27)) * 0x94d049bb133111ebull;
    y ^= y >> 31;
    const double u1 = ((double)(z >> 11) + 1.0) * 0x1.0p-53;
    const double u2 = (double)(y >> 11) * 0x1.0p-53;
    x[i] = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

int autotune(const char *path, hipStream_t s) {
    static const int64_t sizes[] = {512, 1024, 2048, 4096, 8192, 16384, 32768};
    constexpr int ns = sizeof(sizes) / sizeof(sizes[0]);
    const int64_t nmax = sizes[ns - 1];
    double *x = nullptr, *lcv = nullptr;
    MECDF_TRY_HIP(hipMalloc(&x, sizeof(double) * kQDim * nmax));
    if (hipMalloc(&lcv, sizeof(double) * 64) != hipSuccess) {
        (void)hipFree(x);
        set_error("autotune: allocation failed");
        return MECDF_ENOMEM;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    std::vector<double> h(64);
    for (int j = 0; j < 64; ++j)
        h[j] = 0.01 * std::pow(100.0, j / 63.0);
    const int nh = 64;
    double times[2][kQDim][ns][2];
    int64_t best[2][kQDim];
    int rc = MECDF_OK;
    for (int prec = 0; prec < 2 && rc == MECDF_OK; ++prec)
        for (int d = 1; d <= kQDim && rc == MECDF_OK; ++d) {
            best[prec][d - 1] = 0;
            bool queue_wins = true;
            for (int k = 0; k < ns && rc == MECDF_OK; ++k) {
                const int64_t n = sizes[k];
                hipLaunchKernelGGL(k_tune_sample, dim3((unsigned)ceil_div(d * n, 256)), dim3(256),
                                   0, s, x, (int64_t)d * n, (uint64_t)(1000 * d + k));
                mecdf_dataset ds{d, n, x};
                times[prec][d - 1][k][1] = -1.0;  // the queue is not timed past its loss
                for (int way = 0; way < (queue_wins ? 2 : 1) && rc == MECDF_OK; ++way) {
                    float ms[3];
                    for (int r = 0; r < 4 && rc == MECDF_OK; ++r) {  // one warm-up
                        (void)hipEventRecord(e0, s);
                        rc = batch_lcv(&ds, 1, &nh, h.data(), lcv, nullptr,
                                       prec ? MECDF_F32C : MECDF_F64, way, s);
                        (void)hipEventRecord(e1, s);
                        if (hipEventSynchronize(e1) != hipSuccess)
                            rc = MECDF_EDEVICE;
                        if (r > 0)
                            (void)hipEventElapsedTime(&ms[r - 1], e0, e1);
                    }
                    std::sort(ms, ms + 3);
                    times[prec][d - 1][k][way] = ms[1];
                }
                if (queue_wins && times[prec][d - 1][k][1] <= times[prec][d - 1][k][0])
                    best[prec][d - 1] = n;
                else
                    queue_wins = false;  // larger sizes go to the recursion
            }
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(x);
    (void)hipFree(lcv);
    MECDF_TRY(rc);
    const std::string arch = arch_name();
    const std::string out = (path && *path) ? std::string(path) : default_tune_path();
    const std::string tmp = out + ".tmp";
    FILE *f = std::fopen(tmp.c_str(), "wb");
    if (!f) {
        set_error("autotune: cannot write " + tmp);
        return MECDF_EIO;
    }
    std::fprintf(f, "{\n  \"arch\": \"%s\",\n", arch.c_str());
    std::fprintf(f, "  \"what\": \"largest N per d = 1, 2, 3 scored by the work queue\",\n");
    std::fprintf(f, "  \"kde_queue_max_n\": {\"f64\": [%lld, %lld, %lld], \"f32c\": [%lld, %lld, "
                    "%lld]},\n",
                 (long long)best[0][0], (long long)best[0][1], (long long)best[0][2],
                 (long long)best[1][0], (long long)best[1][1], (long long)best[1][2]);
    std::fprintf(f, "  \"ms_64_bandwidths\": [\n");
    for (int prec = 0; prec < 2; ++prec)
        for (int d = 1; d <= kQDim; ++d)
            for (int k = 0; k < ns; ++k)
                std::fprintf(f, "    {\"prec\": \"%s\", \"d\": %d, \"N\": %lld, \"recursion\": %.4f, "
                                "\"queue\": %.4f}%s\n",
                             prec ? "f32c" : "f64", d, (long long)sizes[k],
                             times[prec][d - 1][k][0], times[prec][d - 1][k][1],
                             (prec == 1 && d == kQDim && k == ns - 1) ? "" : ",");
    std::fprintf(f, "  ]\n}\n");
    const bool ok = std::fclose(f) == 0 && std::rename(tmp.c_str(), out.c_str()) == 0;
    if (!ok) {
        set_error("autotune: writing " + out + " failed");
        return MECDF_EIO;
    }
    std::lock_guard<std::mutex> lk(g_tune_mu);
    std::memcpy(g_direct_max, best, sizeof(best));
    g_tune_loaded = true;
    g_tune_source = out;
    return MECDF_OK;
}

int tuning_set(const int64_t *queue_max /* [2][3] */) {
    for (int i = 0; i < 2 * kQDim; ++i)
        if (queue_max[i] < 0 || queue_max[i] > (int64_t(1) << 24)) {
            set_error("tuning: queue sizes must be in 0..2^24");
            return MECDF_EINVAL;
        }
    std::lock_guard<std::mutex> lk(g_tune_mu);
    std::memcpy(g_direct_max, queue_max, sizeof(g_direct_max));
    g_tune_loaded = true;
    g_tune_source = "set by the caller";
    return MECDF_OK;
}

int tuning_info(int64_t *queue_max /* [2][3] */, char *source, int cap) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_tuning_locked();
    if (queue_max)
        std::memcpy(queue_max, g_direct_max, sizeof(g_direct_max));
    if (source && cap > 0)
        std::snprintf(source, (size_t)cap, "%s", g_tune_source.c_str());
    return MECDF_OK;
}

}  // namespace mecdf
