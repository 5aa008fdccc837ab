// Grid path: generalized ECDF / ESF at every node of a rectilinear grid
// (Section 2.1 of Langrene & Warin, arXiv 2005.03246).
//
// The paper bins the points into the local sums s of eq. (partial_sums)
// (Appendix A, by per-axis sorting or mesh division) and then runs the
// nested running sums of its lexicographic sweep, which amount to a d-fold
// prefix sum (eq. (ECDF_decomposition)).  On the GPU the same sums are formed
// as follows, deterministically (no floating-point atomics):
//
//   k_cellkey   per point, the cell index c_k = #{nodes of axis k < x_k} of
//               every axis (exact comparisons; a mesh-division guess checked
//               against the two neighbouring nodes, binary search otherwise),
//               packed as (line << bd) | c_last, where "line" enumerates the
//               cells of axes 0..d-2 and bd bits hold the last-axis cell.
//   radix sort  stable LSD passes on the line bits: each line's points become
//               contiguous, in input order.
//   k_line      one wavefront per line: the line's points are binned into the
//               M_last+1 cells of the last axis (64 at a time: a bitonic sort
//               in registers, then a segmented scan, then one add per cell in
//               LDS, all in a fixed order), followed by the inclusive prefix
//               along the last axis (ECDF) and the exclusive suffix (ESF),
//               written as rows of the output arrays.
//   k_axis_scan the remaining d-1 axes: inclusive prefix (ECDF) or inclusive
//               suffix over node rows (ESF) along axis k, in place, coalesced
//               across the contiguous trailing axes; the last pass divides by N.
//
// The ECDF at node j only needs cells c <= j on every axis, the ESF only cells
// c >= j+1 (eq. (ESF)); so the ECDF array holds the cells 0..M_k-1 of each
// axis and the ESF array the cells 1..M_k shifted down by one, and both
// arrays have exactly the output shape prod(M_k).
#include "common.hpp"
#include "radix.hpp"

namespace mecdf {

struct GridInfo {
    int d;
    int M[MECDF_MAX_DIM];
    int off[MECDF_MAX_DIM];
    uint32_t C[MECDF_MAX_DIM];
    int bd;      // bits holding the last-axis cell index (values 0..M_last)
    uint32_t L;  // number of lines; points with a NaN coordinate go to line L
    // Key layout of the line part.  packed != 0: each axis k < d-1 has its own
    // bit field [sh[k], sh[k] + nb[k]) (axis 0 has room for one extra value,
    // M_0 + 1, that marks a dropped point), so each radix pass sorts on one
    // axis's cells.  packed == 0: the mixed-radix line index sits above bd.
    int packed;
    int sh[MECDF_MAX_DIM];
    int nb[MECDF_MAX_DIM];
};

// mixed-radix line index of a key (L for a dropped point)
__device__ __forceinline__ uint32_t key_line(uint32_t key, const GridInfo &g) {
    if (!g.packed)
        return key >> g.bd;
    uint32_t c0 = (key >> g.sh[0]) & ((1u << g.nb[0]) - 1u);
    if (c0 >= g.C[0])
        return g.L;
    uint32_t line = c0;
    for (int k = 1; k < g.d - 1; ++k)
        line = line * g.C[k] + ((key >> g.sh[k]) & ((1u << g.nb[k]) - 1u));
    return line;
}

// Number of nodes strictly below v: the cell of eq. (partial_sums) holding v,
// cell c meaning z_{c-1} < v <= z_c (z_{-1} = -inf, z_M = +inf).  NaN maps
// to 0 and is filtered by the caller.
template <typename NodePtr>
__device__ __forceinline__ uint32_t cell_index(NodePtr z, int M, double v) {
    double z0 = z[0];
    double zl = z[M - 1];
    if (!(v > z0))
        return 0u;
    if (v > zl)
        return (uint32_t)M;
    // z0 < v <= zl: the answer is in [1, M-1].  Guess by mesh division (the
    // uniform-grid index of Appendix A.2) and check it exactly.
    int c = (int)ceil((v - z0) / (zl - z0) * (double)(M - 1));
    c = c < 1 ? 1 : (c > M - 1 ? M - 1 : c);
    if (z[c - 1] < v && v <= z[c])
        return (uint32_t)c;
    int lo = 1, hi = M - 1;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (z[mid] < v)
            lo = mid + 1;
        else
            hi = mid;
    }
    return (uint32_t)lo;
}

constexpr int kKeyPts = 4;  // points per thread per iteration

template <int D, bool kLds>
__global__ __launch_bounds__(256) void k_cellkey(const double *__restrict__ x,
                                                 int64_t n, GridInfo g,
                                                 const double *__restrict__ nodes_g,
                                                 int total_nodes,
                                                 uint32_t *__restrict__ keys) {
    extern __shared__ double s_nodes[];
    if constexpr (kLds) {
        for (int i = threadIdx.x; i < total_nodes; i += 256)
            s_nodes[i] = nodes_g[i];
        __syncthreads();
    }
    const int64_t step = (int64_t)gridDim.x * 256 * kKeyPts;
    for (int64_t b = (int64_t)blockIdx.x * 256 * kKeyPts + threadIdx.x; b < n; b += step) {
        double v[kKeyPts][D];
#pragma unroll
        for (int q = 0; q < kKeyPts; ++q) {
            int64_t i = b + (int64_t)q * 256;
#pragma unroll
            for (int k = 0; k < D; ++k)
                v[q][k] = i < n ? __builtin_nontemporal_load(x + (int64_t)k * n + i) : 0.0;
        }
#pragma unroll
        for (int q = 0; q < kKeyPts; ++q) {
            int64_t i = b + (int64_t)q * 256;
            if (i >= n)
                break;
            uint32_t line = 0, packed = 0, clast = 0;
            bool bad = false;
#pragma unroll
            for (int k = 0; k < D; ++k) {
                double vv = v[q][k];
                bad |= (vv != vv);
                uint32_t c;
                if constexpr (kLds)
                    c = cell_index(s_nodes + g.off[k], g.M[k], vv);
                else
                    c = cell_index(nodes_g + g.off[k], g.M[k], vv);
                if (k < D - 1) {
                    line = line * g.C[k] + c;
                    packed |= c << g.sh[k];
                } else {
                    clast = c;
                }
            }
            uint32_t key;
            if (g.packed)
                key = bad ? (g.C[0] << g.sh[0]) : (packed | clast);
            else
                key = bad ? (g.L << g.bd) : ((line << g.bd) | clast);
            keys[i] = key;
        }
    }
}

template <int D>
static void launch_cellkey(bool lds, int64_t nb, hipStream_t s, const double *x,
                           int64_t N, const GridInfo &g, const double *nodes,
                           int total_nodes, uint32_t *k0) {
    if (lds)
        hipLaunchKernelGGL((k_cellkey<D, true>), dim3((unsigned)nb), dim3(256),
                           sizeof(double) * total_nodes, s, x, N, g, nodes,
                           total_nodes, k0);
    else
        hipLaunchKernelGGL((k_cellkey<D, false>), dim3((unsigned)nb), dim3(256), 0,
                           s, x, N, g, nodes, total_nodes, k0);
}

__global__ __launch_bounds__(256) void k_line_bounds(const uint32_t *__restrict__ keys,
                                                     int64_t n, GridInfo g,
                                                     uint32_t *__restrict__ lstart) {
    const uint32_t L = g.L;
    // lstart[l] = first sorted position whose line is >= l, for l = 0..L+1
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < n; p += stride) {
        int64_t ln = key_line(keys[p], g);
        int64_t prev = p > 0 ? (int64_t)key_line(keys[p - 1], g) : -1;
        for (int64_t l = prev + 1; l <= ln; ++l)
            lstart[l] = (uint32_t)p;
        if (p == n - 1)
            for (int64_t l = ln + 1; l <= (int64_t)L + 1; ++l)
                lstart[l] = (uint32_t)n;
    }
}

__global__ void k_fill_u32(uint32_t *a, int64_t n, uint32_t v) {
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n)
        a[i] = v;
}

// accumulator of a bin: exact int64 counts, float64, or Kahan float32
template <typename T> struct BinAcc {
    T v;
    __device__ __forceinline__ void zero() { v = T(0); }
    __device__ __forceinline__ void add(T a) { v += a; }
    __device__ __forceinline__ T get() const { return v; }
};
template <> struct BinAcc<float> {
    KahanF k;
    __device__ __forceinline__ void zero() { k.s = 0.f; k.c = 0.f; }
    __device__ __forceinline__ void add(float a) { k.add(a); }
    __device__ __forceinline__ float get() const { return k.get(); }
};

template <typename T> __device__ __forceinline__ T finish(T v, int scale, double N) {
    if constexpr (std::is_same<T, int64_t>::value) {
        return v;
    } else {
        return scale ? (T)((double)v / N) : v;
    }
}

__device__ __forceinline__ void wave_lds_fence() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

constexpr int kLineWaves = 4;

// LDS of one line block: the bins of the four waves.  After they are
// combined into the first set, the prefix and suffix rows reuse the second
// and third.
inline size_t line_lds_bytes(int Cl) { return (size_t)kLineWaves * Cl * 8; }

// One workgroup (4 wavefronts) per line.  Wave w bins the chunks w, w+4, ...
// of 64 points into its own bins: lanes holding the same cell are found with
// ballots on the cell bits, and the lowest such lane adds their values in
// lane order.  The four bin sets are then combined in wave order, so every
// sum is taken in an order fixed by the input order alone.
template <typename T, typename P>
__global__ __launch_bounds__(256) void k_line(const uint32_t *__restrict__ keys,
                                              const P *__restrict__ pay,
                                              const uint32_t *__restrict__ lstart,
                                              GridInfo g, T *__restrict__ F,
                                              T *__restrict__ Fbar, int scale,
                                              double N) {
    extern __shared__ __attribute__((aligned(16))) char s_raw[];
    constexpr bool kPay = !std::is_same<P, NoPayload>::value;
    const int tid = threadIdx.x;
    const int w = tid >> 6;
    const int lane = tid & 63;
    const int64_t line = blockIdx.x;
    const int d = g.d;
    const int Cl = (int)g.C[d - 1];
    const int Ml = Cl - 1;

    // row of the ECDF array (cells <= M_k-1 on axes 0..d-2) and of the ESF
    // array (cells >= 1, shifted down by one)
    int64_t rowE = 0, rowS = 0;
    bool doE = F != nullptr, doS = Fbar != nullptr;
    {
        int64_t t = line;
        int64_t mul = 1;
        for (int k = d - 2; k >= 0; --k) {
            int64_t c = t % g.C[k];
            t /= g.C[k];
            doE = doE && (c <= g.M[k] - 1);
            doS = doS && (c >= 1);
            rowE += c * mul;
            rowS += (c - 1) * mul;
            mul *= g.M[k];
        }
    }
    if (!doE && !doS)
        return;  // uniform over the block

    BinAcc<T> *bins = reinterpret_cast<BinAcc<T> *>(s_raw);
    BinAcc<T> *mybins = bins + (size_t)w * Cl;
    T *Pout = reinterpret_cast<T *>(bins + Cl);
    T *Qout = reinterpret_cast<T *>(bins + 2 * (size_t)Cl);
    for (int c = lane; c < Cl; c += 64)
        mybins[c].zero();
    wave_lds_fence();

    const uint32_t s0 = lstart[line], e0 = lstart[line + 1];
    const uint32_t cmask = (1u << g.bd) - 1u;
    const uint64_t lt = lanemask_lt();
    for (uint32_t p0 = s0 + (uint32_t)w * 64u; p0 < e0; p0 += 64u * kLineWaves) {
        uint32_t p = p0 + lane;
        bool v = p < e0;
        uint32_t c = v ? (keys[p] & cmask) : 0u;
        uint64_t peers = __ballot(v);
        for (int b = 0; b < g.bd; ++b) {
            bool bit = (c >> b) & 1u;
            uint64_t bal = __ballot(v && bit);
            peers &= bit ? bal : ~bal;
        }
        bool leader = v && (peers & lt) == 0;
        if constexpr (kPay) {
            T val = v ? (T)pay[p] : T(0);
            // leaders sum their group in lane order (other lanes follow along)
            T acc = T(0);
            uint64_t m = leader ? peers : 0ull;
            while (__ballot(m != 0ull) != 0ull) {
                int j = m ? (__ffsll((unsigned long long)m) - 1) : lane;
                T o = shfl(val, j);
                if (m) {
                    acc = acc + o;
                    m &= m - 1ull;
                }
            }
            if (leader)
                mybins[c].add(acc);
        } else {
            if (leader)
                mybins[c].add((T)__popcll(peers));
        }
        wave_lds_fence();
    }
    __syncthreads();
    // combine the wave bins in wave order into bins[0]
    for (int c = tid; c < Cl; c += 256) {
        BinAcc<T> t;
        t.zero();
        for (int q = 0; q < kLineWaves; ++q)
            t.add(bins[(size_t)q * Cl + c].get());
        bins[c] = t;
    }
    __syncthreads();

    // last-axis scans: wave 0 the inclusive prefix (ECDF), wave 1 the
    // exclusive suffix (ESF); each lane owns a contiguous run of cells
    if (w < 2) {
        const int ch = (Cl + 63) / 64;
        const int b0 = lane * ch < Cl ? lane * ch : Cl;
        const int b1 = b0 + ch < Cl ? b0 + ch : Cl;
        BinAcc<T> tot;
        tot.zero();
        for (int c = b0; c < b1; ++c)
            tot.add(bins[c].get());
        T tv = tot.get();
        if (w == 0 && doE) {
            T inc = wave_inclusive_scan(tv);
            T ex = shfl_up(inc, 1);
            if (lane == 0)
                ex = T(0);
            BinAcc<T> run;
            run.zero();
            run.add(ex);
            for (int c = b0; c < b1; ++c) {
                run.add(bins[c].get());
                if (c < Ml)
                    Pout[c] = run.get();
            }
        }
        if (w == 1 && doS) {
            T sinc = wave_inclusive_suffix(tv);
            T sex = shfl_down(sinc, 1);
            if (lane == 63)
                sex = T(0);
            BinAcc<T> run;
            run.zero();
            run.add(sex);
            for (int c = b1 - 1; c >= b0; --c) {
                if (c < Ml)
                    Qout[c] = run.get();
                run.add(bins[c].get());
            }
        }
    }
    __syncthreads();
    if (doE) {
        T *dst = F + rowE * Ml;
        for (int j = tid; j < Ml; j += 256)
            dst[j] = finish(Pout[j], scale, N);
    }
    if (doS) {
        T *dst = Fbar + rowS * Ml;
        for (int j = tid; j < Ml; j += 256)
            dst[j] = finish(Qout[j], scale, N);
    }
}

// In-place inclusive prefix (suffix != 0: suffix) along one axis of an array
// viewed as [outer][Mk][inner]; one thread per (outer, inner) column.
template <typename T>
__global__ __launch_bounds__(256) void k_axis_scan(T *__restrict__ A, int64_t outer,
                                                   int64_t Mk, int64_t inner,
                                                   int suffix, int scale, double N) {
    int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= outer * inner)
        return;
    int64_t o = t / inner;
    int64_t i = t - o * inner;
    T *col = A + o * Mk * inner + i;
    BinAcc<T> run;
    run.zero();
    constexpr int U = 8;
    int64_t j = 0;
    for (; j + U <= Mk; j += U) {
        T v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            int64_t jj = suffix ? (Mk - 1 - (j + u)) : (j + u);
            v[u] = col[jj * inner];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            int64_t jj = suffix ? (Mk - 1 - (j + u)) : (j + u);
            run.add(v[u]);
            col[jj * inner] = finish(run.get(), scale, N);
        }
    }
    for (; j < Mk; ++j) {
        int64_t jj = suffix ? (Mk - 1 - j) : j;
        run.add(col[jj * inner]);
        col[jj * inner] = finish(run.get(), scale, N);
    }
}

template <typename T, typename P>
static int grid_run_t(int d, int64_t N, const double *x, const P *y,
                      const int64_t *M, const double *z, T *F, T *Fbar,
                      hipStream_t s) {
    GridInfo g{};
    g.d = d;
    int total_nodes = 0;
    for (int k = 0; k < d; ++k) {
        g.M[k] = (int)M[k];
        g.off[k] = total_nodes;
        g.C[k] = (uint32_t)(M[k] + 1);
        total_nodes += (int)M[k];
    }
    uint64_t L = 1;
    for (int k = 0; k < d - 1; ++k)
        L *= g.C[k];
    g.L = (uint32_t)L;
    g.bd = bits_for((uint64_t)M[d - 1]);
    const int lb = bits_for(L);  // line values 0..L (L = dropped)
    {
        int tot = g.bd;
        for (int k = d - 2; k >= 0; --k) {
            g.nb[k] = bits_for((uint64_t)M[k] + (k == 0 ? 1 : 0));
            g.sh[k] = tot;
            tot += g.nb[k];
        }
        g.packed = (d >= 2 && tot <= 32) ? 1 : 0;
    }
    const int Cl = (int)g.C[d - 1];
    const int Ml = Cl - 1;

    int64_t total_out = 1;
    for (int k = 0; k < d; ++k)
        total_out *= M[k];

    ArenaPlan pl;
    pl.add<double>((size_t)total_nodes);
    pl.add<uint32_t>((size_t)N);  // keys in input order
    pl.add<uint32_t>((size_t)N);
    pl.add<uint32_t>((size_t)N);
    if constexpr (!std::is_same<P, NoPayload>::value) {
        pl.add<P>((size_t)N);
        pl.add<P>((size_t)N);
    }
    pl.add<uint32_t>((size_t)L + 2);
    radix_plan(pl, N);
    void *wsb = nullptr;
    MECDF_TRY(workspace_reserve(pl.used, &wsb));
    Arena a;
    a.base = (char *)wsb;
    double *nodes = a.take<double>((size_t)total_nodes);
    uint32_t *k0 = a.take<uint32_t>((size_t)N);
    uint32_t *k1 = a.take<uint32_t>((size_t)N);
    uint32_t *k2 = a.take<uint32_t>((size_t)N);
    P *p1 = nullptr, *p2 = nullptr;
    if constexpr (!std::is_same<P, NoPayload>::value) {
        p1 = a.take<P>((size_t)N);
        p2 = a.take<P>((size_t)N);
    }
    uint32_t *lstart = a.take<uint32_t>((size_t)L + 2);
    RadixScratch rs = radix_take(a, N);

    MECDF_TRY(upload_small(z, sizeof(double) * total_nodes, nodes, s));

    const uint32_t *ks = k0;
    const P *ps = y;
    if (N > 0) {
        int64_t nb = ceil_div(N, 256);
        if (nb > 8192)
            nb = 8192;
        int64_t nbk = ceil_div(N, 256 * kKeyPts);
        if (nbk > 4096)
            nbk = 4096;
        bool lds = total_nodes <= 12288;
        {
            ProfScope prof1("grid_cellkey", s);
            switch (d) {
            case 1: launch_cellkey<1>(lds, nbk, s, x, N, g, nodes, total_nodes, k0); break;
            case 2: launch_cellkey<2>(lds, nbk, s, x, N, g, nodes, total_nodes, k0); break;
            case 3: launch_cellkey<3>(lds, nbk, s, x, N, g, nodes, total_nodes, k0); break;
            case 4: launch_cellkey<4>(lds, nbk, s, x, N, g, nodes, total_nodes, k0); break;
            case 5: launch_cellkey<5>(lds, nbk, s, x, N, g, nodes, total_nodes, k0); break;
            default: launch_cellkey<6>(lds, nbk, s, x, N, g, nodes, total_nodes, k0); break;
            }
        }
        MECDF_LAUNCH_CHECK();
        int which = 0;
        if (g.packed) {
            // one pass (or more, for axes over 9 bits) per axis, last line axis first
            const uint32_t *ck = k0;
            const P *cp = y;
            int cur = 0;
            for (int k = d - 2; k >= 0; --k) {
                for (int b = g.sh[k]; b < g.sh[k] + g.nb[k]; b += kRadixMaxBits) {
                    int bits = g.sh[k] + g.nb[k] - b;
                    bits = bits < kRadixMaxBits ? bits : kRadixMaxBits;
                    uint32_t *nk = (cur == 1) ? k2 : k1;
                    P *np = (cur == 1) ? p2 : p1;
                    MECDF_TRY((radix_pass<uint32_t, P>(ck, cp, nk, np, N, b, bits, rs, s)));
                    cur = (cur == 1) ? 2 : 1;
                    ck = nk;
                    cp = np;
                }
            }
            which = cur;
        } else {
            MECDF_TRY((radix_sort_bits<uint32_t, P>(k0, y, k1, p1, k2, p2, N, g.bd,
                                                    g.bd + lb, rs, s, &which)));
        }
        ks = which == 0 ? k0 : (which == 1 ? k1 : k2);
        ps = which == 0 ? y : (which == 1 ? p1 : p2);
        ProfScope prof2("grid_line_bounds", s);
        hipLaunchKernelGGL(k_line_bounds, dim3((unsigned)nb), dim3(256), 0, s, ks,
                           N, g, lstart);
        MECDF_LAUNCH_CHECK();
    } else {
        hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)ceil_div(L + 2, 256)), dim3(256),
                           0, s, lstart, (int64_t)L + 2, 0u);
        MECDF_LAUNCH_CHECK();
    }

    size_t lb_bytes = line_lds_bytes(Cl);
    if (lb_bytes > 160 * 1024) {
        set_error("last grid axis too large for the line kernel");
        return MECDF_EUNSUPPORTED;
    }
    if (lb_bytes > 64 * 1024)
        MECDF_TRY_HIP(hipFuncSetAttribute((const void *)k_line<T, P>,
                                          hipFuncAttributeMaxDynamicSharedMemorySize,
                                          (int)lb_bytes));
    {
        ProfScope prof3("grid_line", s);
        hipLaunchKernelGGL((k_line<T, P>), dim3((unsigned)L), dim3(256), lb_bytes, s,
                           ks, ps, lstart, g, F, Fbar, d == 1 ? 1 : 0, (double)N);
    }
    MECDF_LAUNCH_CHECK();

    // remaining axes, innermost first; the last pass divides by N
    for (int k = d - 2; k >= 0; --k) {
        int64_t outer = 1, inner = 1;
        for (int q = 0; q < k; ++q)
            outer *= M[q];
        for (int q = k + 1; q < d; ++q)
            inner *= M[q];
        int64_t nthreads = outer * inner;
        int64_t nbk = ceil_div(nthreads, 256);
        int scale = (k == 0) ? 1 : 0;
        ProfScope prof4("grid_axis_scan", s);
        if (F) {
            hipLaunchKernelGGL(k_axis_scan<T>, dim3((unsigned)nbk), dim3(256), 0, s,
                               F, outer, (int64_t)M[k], inner, 0, scale, (double)N);
        }
        if (Fbar) {
            hipLaunchKernelGGL(k_axis_scan<T>, dim3((unsigned)nbk), dim3(256), 0, s,
                               Fbar, outer, (int64_t)M[k], inner, 1, scale, (double)N);
        }
        MECDF_LAUNCH_CHECK();
    }
    (void)total_out;
    (void)Ml;
    return MECDF_OK;
}

int grid_run(int d, int64_t N, const double *x, const void *y,
             const int64_t *M, const double *z, void *F, void *Fbar, int prec,
             hipStream_t s) {
    if (y == nullptr)
        return grid_run_t<int64_t, NoPayload>(d, N, x, nullptr, M, z,
                                              (int64_t *)F, (int64_t *)Fbar, s);
    if (prec == MECDF_F64)
        return grid_run_t<double, double>(d, N, x, (const double *)y, M, z,
                                          (double *)F, (double *)Fbar, s);
    return grid_run_t<float, float>(d, N, x, (const float *)y, M, z, (float *)F,
                                    (float *)Fbar, s);
}

}  // namespace mecdf
