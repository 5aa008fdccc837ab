// Learned bandwidth proposal: on-device summary features of a dataset and a
// 32 -> 128 -> 128 -> 1 ReLU network that maps them to a log-bandwidth
// correction, trained on the device.  The bandwidth it proposes is only a
// starting point: the selected bandwidth is always the best of exact
// leave-one-out likelihood scores (see mecdf_bw_select), so kernel values
// stay exact.
//
// Numerics: matrix products take bfloat16 operands (round to nearest even)
// and accumulate in float32 on the matrix cores (v_mfma_f32_16x16x16_bf16);
// biases, the last layer, gradients and Adam run in float32 on the master
// weights.  Reductions over the batch are done in a fixed order.
//
// Parameter vector (float32, MECDF_MLP_PARAMS entries):
//   W1 [128][32] | b1 [128] | W2 [128][128] | b2 [128] | w3 [128] | b3 [1]
#include <vector>

#include "common.hpp"

namespace mecdf {

constexpr int kIn = 32, kH = 128;
constexpr int oW1 = 0, ob1 = oW1 + kH * kIn, oW2 = ob1 + kH, ob2 = oW2 + kH * kH,
              ow3 = ob2 + kH, ob3 = ow3 + kH, kParams = ob3 + 1;
static_assert(kParams == MECDF_MLP_PARAMS, "parameter layout");

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// float -> bfloat16 bits, round to nearest even (finite inputs)
__device__ __forceinline__ short bf16_bits(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (short)(u >> 16);
}
__device__ __forceinline__ float bf16_float(short b) {
    return __uint_as_float(((uint32_t)(uint16_t)b) << 16);
}

// D(16x16) += A(16x16) B(16x16); lane l holds A[l%16][4(l/16)+i],
// B[4(l/16)+i][l%16] and D[4(l/16)+i][l%16], i = 0..3
__device__ __forceinline__ f32x4 mfma16(bf16x4 a, bf16x4 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// ------------------------------------------------------------ features
struct DevSet {
    int d;
    int64_t n;
    const double *x;
};

// One block of 256 threads per dataset; deterministic tree reductions.
// Features (32 floats, zero padded):
//  0 log(n)/10   1 d/3   2-4 log sd_k   5-7 skewness_k   8-10 excess kurtosis_k/10
//  11 mean |corr|   12 log h0 (h0 = geometric-mean sd * n^(-1/(d+4)))
//  13 log geometric-mean sd   14-16 mean |x - mean| / sd   17-19 fraction of
//  points within half a sd of the mean
__device__ double block_sum256(double v, double *buf) {
    buf[threadIdx.x] = v;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            buf[threadIdx.x] += buf[threadIdx.x + w];
        __syncthreads();
    }
    double r = buf[0];
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(256) void k_features(const DevSet *__restrict__ sets,
                                                  float *__restrict__ feat) {
    __shared__ double buf[256];
    const DevSet S = sets[blockIdx.x];
    const int d = S.d;
    const int64_t n = S.n;
    double mean[3] = {0, 0, 0}, sd[3] = {1, 1, 1};
    for (int k = 0; k < d; ++k) {
        double s = 0.0;
        for (int64_t i = threadIdx.x; i < n; i += 256)
            s += S.x[(int64_t)k * n + i];
        mean[k] = block_sum256(s, buf) / (double)n;
    }
    double m2[3], m3[3], m4[3], mad[3], half[3], cov[3] = {0, 0, 0};
    for (int k = 0; k < d; ++k) {
        double a2 = 0, a3 = 0, a4 = 0, a1 = 0;
        for (int64_t i = threadIdx.x; i < n; i += 256) {
            double c = S.x[(int64_t)k * n + i] - mean[k];
            double c2 = c * c;
            a1 += fabs(c);
            a2 += c2;
            a3 += c2 * c;
            a4 += c2 * c2;
        }
        m2[k] = block_sum256(a2, buf) / (double)n;
        m3[k] = block_sum256(a3, buf) / (double)n;
        m4[k] = block_sum256(a4, buf) / (double)n;
        mad[k] = block_sum256(a1, buf) / (double)n;
        sd[k] = sqrt(m2[k]) > 1e-300 ? sqrt(m2[k]) : 1e-300;
    }
    double frac[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};  // within 1/4, 1, 2 sd
    for (int k = 0; k < d; ++k) {
        double c = 0, q1 = 0, q4 = 0, q8 = 0;
        for (int64_t i = threadIdx.x; i < n; i += 256) {
            const double a = fabs(S.x[(int64_t)k * n + i] - mean[k]);
            c += a <= 0.5 * sd[k] ? 1.0 : 0.0;
            q1 += a <= 0.25 * sd[k] ? 1.0 : 0.0;
            q4 += a <= sd[k] ? 1.0 : 0.0;
            q8 += a <= 2.0 * sd[k] ? 1.0 : 0.0;
        }
        half[k] = block_sum256(c, buf) / (double)n;
        frac[k][0] = block_sum256(q1, buf) / (double)n;
        frac[k][1] = block_sum256(q4, buf) / (double)n;
        frac[k][2] = block_sum256(q8, buf) / (double)n;
    }
    int np = 0;
    double corr_sum = 0.0;
    for (int a = 0; a < d; ++a)
        for (int b = a + 1; b < d; ++b) {
            double c = 0;
            for (int64_t i = threadIdx.x; i < n; i += 256)
                c += (S.x[(int64_t)a * n + i] - mean[a]) * (S.x[(int64_t)b * n + i] - mean[b]);
            double cv = block_sum256(c, buf) / (double)n;
            corr_sum += fabs(cv / (sd[a] * sd[b]));
            ++np;
        }
    (void)cov;
    if (threadIdx.x != 0)
        return;
    float *f = feat + (int64_t)blockIdx.x * kIn;
    for (int q = 0; q < kIn; ++q)
        f[q] = 0.f;
    double lg = 0.0;
    for (int k = 0; k < d; ++k)
        lg += log(sd[k]);
    lg /= d;
    f[0] = (float)(log((double)n) / 10.0);
    f[1] = (float)(d / 3.0);
    for (int k = 0; k < d; ++k) {
        f[2 + k] = (float)log(sd[k]);
        f[5 + k] = (float)(m3[k] / (sd[k] * sd[k] * sd[k]));
        f[8 + k] = (float)((m4[k] / (m2[k] * m2[k]) - 3.0) / 10.0);
        f[14 + k] = (float)(mad[k] / sd[k]);
        f[17 + k] = (float)half[k];
        for (int q = 0; q < 3; ++q)
            f[20 + 3 * k + q] = (float)frac[k][q];
    }
    f[11] = np ? (float)(corr_sum / np) : 0.f;
    f[12] = (float)(lg - log((double)n) / (d + 4.0));
    f[13] = (float)lg;
}

// ------------------------------------------------------------ network
// Activations kept for the backward pass (B rounded up to 16 = Bp):
//   XT  bf16 [32][Bp], A1T bf16 [128][Bp], A2 float [B][128], OUT float [B]
struct MlpBufs {
    short *W1b, *W2b;  // bf16 copies of the weight matrices
    short *XT, *A1T;
    float *A2, *OUT;
    short *DZ2T, *DZ1T;
    float *part;       // partial gradients
};

// Refreshes the bf16 copies of W1 and W2.
__global__ void k_mlp_cast(const float *__restrict__ P, short *__restrict__ W1b,
                           short *__restrict__ W2b) {
    int i = blockIdx.x * 256 + threadIdx.x;
    if (i < kH * kIn)
        W1b[i] = bf16_bits(P[oW1 + i]);
    if (i < kH * kH)
        W2b[i] = bf16_bits(P[oW2 + i]);
}

// Forward, one wavefront per 16 rows.
__global__ __launch_bounds__(64) void k_mlp_fwd(const float *__restrict__ X, int B, int Bp,
                                                const float *__restrict__ P,
                                                const short *__restrict__ W1b,
                                                const short *__restrict__ W2b,
                                                short *__restrict__ XT, short *__restrict__ A1T,
                                                float *__restrict__ A2, float *__restrict__ OUT) {
    __shared__ short sA[16][kH + 4];
    const int l = threadIdx.x;
    const int r0 = blockIdx.x * 16;
    const int lr = l % 16, lg = l / 16;
    // layer 1: A = X rows (K = 32 in two steps of 16)
    bf16x4 xa[2];
    for (int ks = 0; ks < 2; ++ks)
        for (int i = 0; i < 4; ++i) {
            int r = r0 + lr, k = ks * 16 + 4 * lg + i;
            float v = r < B ? X[(int64_t)r * kIn + k] : 0.f;
            xa[ks][i] = bf16_bits(v);
            XT[(int64_t)k * Bp + r] = xa[ks][i];
        }
    for (int ct = 0; ct < kH / 16; ++ct) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        for (int ks = 0; ks < 2; ++ks) {
            bf16x4 b;
            for (int i = 0; i < 4; ++i)
                b[i] = W1b[(ct * 16 + lr) * kIn + ks * 16 + 4 * lg + i];
            acc = mfma16(xa[ks], b, acc);
        }
        const int col = ct * 16 + lr;
        for (int i = 0; i < 4; ++i) {
            int row = 4 * lg + i;
            float z = acc[i] + P[ob1 + col];
            float a = z > 0.f ? z : 0.f;
            short ab = bf16_bits(a);
            sA[row][col] = ab;
            A1T[(int64_t)col * Bp + r0 + row] = ab;
        }
    }
    __syncthreads();
    // layer 2: A = a1 (bf16, K = 128)
    float dot[4] = {0.f, 0.f, 0.f, 0.f};
    for (int ct = 0; ct < kH / 16; ++ct) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        for (int ks = 0; ks < kH / 16; ++ks) {
            bf16x4 a, b;
            for (int i = 0; i < 4; ++i) {
                a[i] = sA[lr][ks * 16 + 4 * lg + i];
                b[i] = W2b[(ct * 16 + lr) * kH + ks * 16 + 4 * lg + i];
            }
            acc = mfma16(a, b, acc);
        }
        const int col = ct * 16 + lr;
        for (int i = 0; i < 4; ++i) {
            int row = r0 + 4 * lg + i;
            float z = acc[i] + P[ob2 + col];
            float a = z > 0.f ? z : 0.f;
            if (row < B)
                A2[(int64_t)row * kH + col] = a;
            dot[i] += a * P[ow3 + col];
        }
    }
    // reduce the 16 lanes of each lane group (fixed butterfly order)
    for (int i = 0; i < 4; ++i) {
        float v = dot[i];
        for (int m = 1; m < 16; m <<= 1)
            v += __shfl_xor(v, m, 64);
        dot[i] = v;
    }
    if (lr == 0)
        for (int i = 0; i < 4; ++i) {
            int row = r0 + 4 * lg + i;
            if (row < B)
                OUT[row] = dot[i] + P[ob3];
        }
}

// Backward, part 1 (one wavefront per 16 rows): output error g, dZ2 and
// dZ1 (bf16, transposed for the weight products) and per-tile partial sums
// of the bias and last-layer gradients.
// part layout per 16-row tile: [w3 grad 128][b3 1][b2 grad 128][b1 grad 128]
constexpr int kPart1 = kH + 1 + kH + kH;

__global__ __launch_bounds__(64) void k_mlp_bwd1(const float *__restrict__ target, int B, int Bp,
                                                 const float *__restrict__ P,
                                                 const short *__restrict__ W2b,
                                                 const short *__restrict__ A1T,
                                                 const float *__restrict__ A2,
                                                 const float *__restrict__ OUT,
                                                 short *__restrict__ DZ2T,
                                                 short *__restrict__ DZ1T,
                                                 float *__restrict__ part, float *__restrict__ sqerr) {
    __shared__ float sg[16];
    const int l = threadIdx.x;
    const int r0 = blockIdx.x * 16;
    const int lr = l % 16, lg = l / 16;
    if (l < 16) {
        int r = r0 + l;
        float e = r < B ? OUT[r] - target[r] : 0.f;
        sg[l] = 2.f * e / (float)B;
        sqerr[r0 + l] = e * e;  // Bp entries
    }
    __syncthreads();
    float *pt = part + (int64_t)blockIdx.x * kPart1;
    // last layer and b2: column c = l and l + 64 (fixed row order)
    for (int c = l; c < kH; c += 64) {
        float gw3 = 0.f, gb2 = 0.f;
        for (int i = 0; i < 16; ++i) {
            int r = r0 + i;
            if (r >= B)
                break;
            float a = A2[(int64_t)r * kH + c];
            gw3 += sg[i] * a;
            gb2 += a > 0.f ? sg[i] * P[ow3 + c] : 0.f;
        }
        pt[c] = gw3;
        pt[kH + 1 + c] = gb2;
    }
    if (l == 0) {
        float gb3 = 0.f;
        for (int i = 0; i < 16; ++i)
            gb3 += sg[i];
        pt[kH] = gb3;
    }
    // dZ2 in the A layout: rows r0 + lr, columns o = ks*16 + 4 lg + i
    // dA1 = dZ2 W2  (K = 128 over o), then dZ1 = dA1 * [a1 > 0]
    bf16x4 dz[kH / 16];
    for (int ks = 0; ks < kH / 16; ++ks)
        for (int i = 0; i < 4; ++i) {
            int r = r0 + lr, o = ks * 16 + 4 * lg + i;
            float v = 0.f;
            if (r < B && A2[(int64_t)r * kH + o] > 0.f)
                v = sg[lr] * P[ow3 + o];
            dz[ks][i] = bf16_bits(v);
            DZ2T[(int64_t)o * Bp + r] = dz[ks][i];
        }
    float gb1[4 * (kH / 16)];
    for (int ct = 0; ct < kH / 16; ++ct) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        for (int ks = 0; ks < kH / 16; ++ks) {
            bf16x4 b;  // B[k = o][n = i] = W2[o][i]
            for (int i = 0; i < 4; ++i)
                b[i] = W2b[(ks * 16 + 4 * lg + i) * kH + ct * 16 + lr];
            acc = mfma16(dz[ks], b, acc);
        }
        const int col = ct * 16 + lr;
        for (int i = 0; i < 4; ++i) {
            int row = r0 + 4 * lg + i;
            float a1 = bf16_float(A1T[(int64_t)col * Bp + row]);
            float v = (row < B && a1 > 0.f) ? acc[i] : 0.f;
            DZ1T[(int64_t)col * Bp + row] = bf16_bits(v);
            gb1[ct * 4 + i] = v;
        }
    }
    // b1 partials: column col = ct*16 + lr gets the 16 rows held by the 4 lane
    // groups; sum them in a fixed order through LDS
    __shared__ float sb[4][kH];
    for (int ct = 0; ct < kH / 16; ++ct) {
        float v = 0.f;
        for (int i = 0; i < 4; ++i)
            v += gb1[ct * 4 + i];
        sb[lg][ct * 16 + lr] = v;
    }
    __syncthreads();
    for (int c = l; c < kH; c += 64)
        pt[kH + 1 + kH + c] = sb[0][c] + sb[1][c] + sb[2][c] + sb[3][c];
}

// Weight gradients G = D^T A over the batch: D^T given as DT [M][Bp] (bf16),
// A as AT [N][Bp] (bf16), K = rows in chunks of kKc.  One wavefront per
// (16x16 output tile, row chunk); partials [chunk][M][N].
constexpr int kKc = 256;

__global__ __launch_bounds__(64) void k_mlp_wgrad(const short *__restrict__ DT,
                                                  const short *__restrict__ AT, int M, int N,
                                                  int Bp, float *__restrict__ part) {
    const int l = threadIdx.x;
    const int lr = l % 16, lg = l / 16;
    const int tiles_n = N / 16;
    const int tm = blockIdx.x / tiles_n, tn = blockIdx.x % tiles_n;
    const int chunk = blockIdx.y;
    const int k0 = chunk * kKc;
    const int k1 = (k0 + kKc) < Bp ? (k0 + kKc) : Bp;
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    for (int ks = k0; ks < k1; ks += 16) {
        bf16x4 a, b;
        for (int i = 0; i < 4; ++i) {
            a[i] = DT[(int64_t)(tm * 16 + lr) * Bp + ks + 4 * lg + i];
            b[i] = AT[(int64_t)(tn * 16 + lr) * Bp + ks + 4 * lg + i];
        }
        acc = mfma16(a, b, acc);
    }
    float *pt = part + (int64_t)chunk * M * N;
    for (int i = 0; i < 4; ++i)
        pt[(tm * 16 + 4 * lg + i) * N + tn * 16 + lr] = acc[i];
}

// Sums the partials in chunk order into the gradient vector.
__global__ void k_mlp_gsum(const float *__restrict__ p1, int ntile, const float *__restrict__ pW2,
                           const float *__restrict__ pW1, int nchunk,
                           const float *__restrict__ sqerr, int Bp, int B,
                           float *__restrict__ G, float *__restrict__ loss) {
    int i = blockIdx.x * 256 + threadIdx.x;
    if (i < kH * kIn) {
        float s = 0.f;
        for (int c = 0; c < nchunk; ++c)
            s += pW1[(int64_t)c * kH * kIn + i];
        G[oW1 + i] = s;
    }
    if (i < kH * kH) {
        float s = 0.f;
        for (int c = 0; c < nchunk; ++c)
            s += pW2[(int64_t)c * kH * kH + i];
        G[oW2 + i] = s;
    }
    if (i < kH) {
        float a = 0.f, b = 0.f, c1 = 0.f;
        for (int t = 0; t < ntile; ++t) {
            const float *pt = p1 + (int64_t)t * kPart1;
            a += pt[i];
            b += pt[kH + 1 + i];
            c1 += pt[kH + 1 + kH + i];
        }
        G[ow3 + i] = a;
        G[ob2 + i] = b;
        G[ob1 + i] = c1;
    }
    if (i == 0) {
        float s = 0.f;
        for (int t = 0; t < ntile; ++t)
            s += p1[(int64_t)t * kPart1 + kH];
        G[ob3] = s;
        if (loss) {
            double e = 0.0;
            for (int r = 0; r < Bp; ++r)
                e += sqerr[r];
            *loss = (float)(e / B);
        }
    }
}

// Adam step with decoupled weight decay: p -= lr (m^ / (sqrt(v^) + eps) + wd p)
__global__ void k_mlp_adam(float *__restrict__ P, const float *__restrict__ G,
                           float *__restrict__ m, float *__restrict__ v, float lr, float wd,
                           float b1, float b2, float eps, float c1, float c2) {
    int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= kParams)
        return;
    float g = G[i];
    float mi = b1 * m[i] + (1.f - b1) * g;
    float vi = b2 * v[i] + (1.f - b2) * g * g;
    m[i] = mi;
    v[i] = vi;
    float p = P[i];
    P[i] = p - lr * ((mi / c1) / (sqrtf(vi / c2) + eps) + wd * p);
}

// Initial parameters from a seed: He-style normals for W1 (sd sqrt(2/32)) and
// W2 (sd sqrt(2/128)), w3 with sd 0.1 sqrt(1/128), zero biases.  Each entry
// draws its own pair of uniforms from a counter-based generator (SplitMix64
// of seed and the entry's index), turned into a normal by Box-Muller.
__device__ __forceinline__ uint64_t splitmix64(uint64_t z) {
    z += 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

__global__ void k_mlp_init(float *__restrict__ P, uint64_t seed) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= kParams)
        return;
    const uint64_t a = splitmix64(seed ^ splitmix64(2 * (uint64_t)i + 1));
    const uint64_t b = splitmix64(a);
    const double u1 = ((double)(a >> 11) + 1.0) * 0x1.0p-53;  // (0, 1]
    const double u2 = (double)(b >> 11) * 0x1.0p-53;          // [0, 1)
    const double z = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
    double sd = 0.0;
    if (i < ob1)
        sd = sqrt(2.0 / kIn);
    else if (i >= oW2 && i < ob2)
        sd = sqrt(2.0 / kH);
    else if (i >= ow3 && i < ob3)
        sd = 0.1 * sqrt(1.0 / kH);
    P[i] = (float)(sd * z);
}

// Regression targets of the proposal: T[r] = log(h of the label's grid index)
// minus the rule-of-thumb log h0 (feature 12).
__global__ void k_bw_targets(const float *__restrict__ feat, const int *__restrict__ label,
                             const double *__restrict__ hgrid, int B, float *__restrict__ T) {
    const int r = blockIdx.x * 256 + threadIdx.x;
    if (r < B)
        T[r] = (float)(log(hgrid[label[r]]) - (double)feat[(int64_t)r * kIn + 12]);
}

__global__ void k_fill_f32(float *__restrict__ a, int64_t n, float v) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n)
        a[i] = v;
}

// ------------------------------------------------------------ host side
struct MlpWork {
    MlpBufs b;
    float *G, *p1, *pW1, *pW2, *sq;
    int Bp, ntile, nchunk;
};

// extra: bytes of caller scratch carved after the network's buffers (*extra_out)
static int mlp_work(int B, MlpWork &w, size_t extra = 0, void **extra_out = nullptr) {
    w.Bp = (int)ceil_div(B, 16) * 16;
    w.ntile = w.Bp / 16;
    w.nchunk = (int)ceil_div(w.Bp, kKc);
    ArenaPlan pl;
    pl.add<short>(kH * kIn);
    pl.add<short>(kH * kH);
    pl.add<short>((size_t)kIn * w.Bp);
    pl.add<short>((size_t)kH * w.Bp);
    pl.add<float>((size_t)w.Bp * kH);
    pl.add<float>((size_t)w.Bp);
    pl.add<short>((size_t)kH * w.Bp);
    pl.add<short>((size_t)kH * w.Bp);
    pl.add<float>(kParams);
    pl.add<float>((size_t)w.ntile * kPart1);
    pl.add<float>((size_t)w.nchunk * kH * kIn);
    pl.add<float>((size_t)w.nchunk * kH * kH);
    pl.add<float>((size_t)w.Bp);
    pl.add<char>(extra);
    void *base = nullptr;
    MECDF_TRY(workspace_reserve(pl.used, &base));
    Arena a;
    a.base = (char *)base;
    w.b.W1b = a.take<short>(kH * kIn);
    w.b.W2b = a.take<short>(kH * kH);
    w.b.XT = a.take<short>((size_t)kIn * w.Bp);
    w.b.A1T = a.take<short>((size_t)kH * w.Bp);
    w.b.A2 = a.take<float>((size_t)w.Bp * kH);
    w.b.OUT = a.take<float>((size_t)w.Bp);
    w.b.DZ2T = a.take<short>((size_t)kH * w.Bp);
    w.b.DZ1T = a.take<short>((size_t)kH * w.Bp);
    w.G = a.take<float>(kParams);
    w.p1 = a.take<float>((size_t)w.ntile * kPart1);
    w.pW1 = a.take<float>((size_t)w.nchunk * kH * kIn);
    w.pW2 = a.take<float>((size_t)w.nchunk * kH * kH);
    w.sq = a.take<float>((size_t)w.Bp);
    char *ex = a.take<char>(extra);
    if (extra_out)
        *extra_out = ex;
    return MECDF_OK;
}

static int mlp_forward_w(MlpWork &w, int B, const float *X, const float *P, hipStream_t s) {
    ProfScope prof("mlp_forward", s);
    hipLaunchKernelGGL(k_mlp_cast, dim3((unsigned)ceil_div(kH * kH, 256)), dim3(256), 0, s, P,
                       w.b.W1b, w.b.W2b);
    hipLaunchKernelGGL(k_mlp_fwd, dim3((unsigned)w.ntile), dim3(64), 0, s, X, B, w.Bp, P,
                       w.b.W1b, w.b.W2b, w.b.XT, w.b.A1T, w.b.A2, w.b.OUT);
    MECDF_LAUNCH_CHECK();
    return MECDF_OK;
}

static int mlp_grad_w(MlpWork &w, int B, const float *T, const float *P, float *loss,
                      hipStream_t s) {
    ProfScope prof("mlp_backward", s);
    hipLaunchKernelGGL(k_mlp_bwd1, dim3((unsigned)w.ntile), dim3(64), 0, s, T, B, w.Bp, P,
                       w.b.W2b, w.b.A1T, w.b.A2, w.b.OUT, w.b.DZ2T, w.b.DZ1T, w.p1, w.sq);
    hipLaunchKernelGGL(k_mlp_wgrad, dim3((unsigned)(kH / 16 * kH / 16), (unsigned)w.nchunk),
                       dim3(64), 0, s, w.b.DZ2T, w.b.A1T, kH, kH, w.Bp, w.pW2);
    hipLaunchKernelGGL(k_mlp_wgrad, dim3((unsigned)(kH / 16 * kIn / 16), (unsigned)w.nchunk),
                       dim3(64), 0, s, w.b.DZ1T, w.b.XT, kH, kIn, w.Bp, w.pW1);
    hipLaunchKernelGGL(k_mlp_gsum, dim3((unsigned)ceil_div(kH * kH, 256)), dim3(256), 0, s, w.p1,
                       w.ntile, w.pW2, w.pW1, w.nchunk, w.sq, w.Bp, B, w.G, loss);
    MECDF_LAUNCH_CHECK();
    return MECDF_OK;
}

int mlp_forward(int B, const float *X, const float *P, float *out, hipStream_t s) {
    MlpWork w;
    MECDF_TRY(mlp_work(B, w));
    MECDF_TRY(mlp_forward_w(w, B, X, P, s));
    MECDF_TRY_HIP(hipMemcpyAsync(out, w.b.OUT, sizeof(float) * B, hipMemcpyDeviceToDevice, s));
    return MECDF_OK;
}

int mlp_grad(int B, const float *X, const float *T, const float *P, float *G, float *loss,
             hipStream_t s) {
    MlpWork w;
    MECDF_TRY(mlp_work(B, w));
    MECDF_TRY(mlp_forward_w(w, B, X, P, s));
    MECDF_TRY(mlp_grad_w(w, B, T, P, loss, s));
    MECDF_TRY_HIP(hipMemcpyAsync(G, w.G, sizeof(float) * kParams, hipMemcpyDeviceToDevice, s));
    return MECDF_OK;
}

// Adam steps t0 + 1 .. t0 + steps (the bias corrections continue from t0).
static int mlp_train_w(MlpWork &w, int B, const float *X, const float *T, float *P, float *adam,
                       int steps, float lr, float wd, float *losses, int64_t t0, hipStream_t s) {
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    double p1 = 1.0, p2 = 1.0;
    for (int64_t t = 0; t < t0; ++t) {
        p1 *= b1;
        p2 *= b2;
    }
    for (int t = 0; t < steps; ++t) {
        MECDF_TRY(mlp_forward_w(w, B, X, P, s));
        MECDF_TRY(mlp_grad_w(w, B, T, P, losses ? losses + t : nullptr, s));
        p1 *= b1;
        p2 *= b2;
        hipLaunchKernelGGL(k_mlp_adam, dim3((unsigned)ceil_div(kParams, 256)), dim3(256), 0, s, P,
                           w.G, adam, adam + kParams, lr, wd, b1, b2, eps, (float)(1.0 - p1),
                           (float)(1.0 - p2));
        MECDF_LAUNCH_CHECK();
    }
    return MECDF_OK;
}

int mlp_train(int B, const float *X, const float *T, float *P, float *adam, int steps, float lr,
              float wd, float *losses, hipStream_t s) {
    MlpWork w;
    MECDF_TRY(mlp_work(B, w));
    return mlp_train_w(w, B, X, T, P, adam, steps, lr, wd, losses, 0, s);
}

// Fresh parameters from the seed and zero Adam moments.
int mlp_init(uint64_t seed, float *P, float *adam, hipStream_t s) {
    hipLaunchKernelGGL(k_mlp_init, dim3((unsigned)ceil_div(kParams, 256)), dim3(256), 0, s, P,
                       seed);
    hipLaunchKernelGGL(k_fill_f32, dim3((unsigned)ceil_div(2 * kParams, 256)), dim3(256), 0, s,
                       adam, (int64_t)2 * kParams, 0.f);
    MECDF_LAUNCH_CHECK();
    return MECDF_OK;
}

// Training on grid labels: targets formed on the device from the labels and
// the grid (host), then Adam steps t0 + 1 .. t0 + steps.
int bw_train_steps(int B, const float *feat, const int *label, int nhg, const double *hgrid,
                   int steps, float lr, float wd, float *P, float *adam, float *losses,
                   int64_t t0, hipStream_t s) {
    MlpWork w;
    void *extra = nullptr;
    const size_t tbytes = ((sizeof(float) * (size_t)B + 255) / 256) * 256;
    MECDF_TRY(mlp_work(B, w, tbytes + sizeof(double) * (size_t)nhg, &extra));
    float *T = (float *)extra;
    double *hg = (double *)((char *)extra + tbytes);
    MECDF_TRY(upload_small(hgrid, sizeof(double) * (size_t)nhg, hg, s));
    hipLaunchKernelGGL(k_bw_targets, dim3((unsigned)ceil_div(B, 256)), dim3(256), 0, s, feat,
                       label, hg, B, T);
    MECDF_LAUNCH_CHECK();
    return mlp_train_w(w, B, feat, T, P, adam, steps, lr, wd, losses, t0, s);
}

int bw_features(const mecdf_dataset *sets, int nsets, float *feat, hipStream_t s) {
    std::vector<DevSet> hs(nsets);
    for (int i = 0; i < nsets; ++i) {
        hs[i].d = sets[i].d;
        hs[i].n = sets[i].N;
        hs[i].x = sets[i].x;
    }
    void *base = nullptr;
    MECDF_TRY(workspace_reserve(sizeof(DevSet) * nsets + 256, &base));
    MECDF_TRY(upload_small(hs.data(), sizeof(DevSet) * nsets, base, s));
    ProfScope prof("bw_features", s);
    hipLaunchKernelGGL(k_features, dim3((unsigned)nsets), dim3(256), 0, s, (const DevSet *)base,
                       feat);
    MECDF_LAUNCH_CHECK();
    return MECDF_OK;
}

}  // namespace mecdf
