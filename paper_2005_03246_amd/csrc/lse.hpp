// Sums of exponentials relative to their largest term, for leave-one-out
// kernel sums whose logarithm must exist where every term is below the
// float64 range (the log-sum-exp of the likelihood cross-validation score).
#pragma once

#include "common.hpp"

namespace mecdf {

// Leave-one-out kernel sums at a query j written relative to its nearest
// other point, so that their logarithm exists even where every term
// exp(-e_i) is below the float64 range:
//   e_i = sum_k |x_k,i - x_k,j| / h_k,   m = min_{i != j} e_i,
//   S_c = sum_{i != j} w_c,i exp(-(e_i - m)),   sum_{i != j} w_c,i exp(-e_i) = exp(-m) S_c.
// Accumulated in one pass: a smaller e_i rescales the sums seen so far by
// exp(-(m - e_i)) and becomes the new m.  Sums carry a Neumaier compensation
// term (rescaled with them).
template <int CH> struct LooAcc {
    double m;
    double s[CH], c[CH];
};

template <int CH> __device__ __forceinline__ void loo_init(LooAcc<CH> &a) {
    a.m = INFINITY;
#pragma unroll
    for (int c = 0; c < CH; ++c)
        a.s[c] = a.c[c] = 0.0;
}

__device__ __forceinline__ void neum_add(double &s, double &c, double v) {
    const double t = s + v;
    c += fabs(s) >= fabs(v) ? (s - t) + v : (v - t) + s;
    s = t;
}

// one term: scaled distance e with factor t = exp(-|e - m|) already formed
template <int CH>
__device__ __forceinline__ void loo_add(LooAcc<CH> &a, double e, double t, const double (&w)[CH]) {
    const bool lower = e < a.m;
#pragma unroll
    for (int c = 0; c < CH; ++c) {
        if (lower) {
            a.s[c] *= t;
            a.c[c] *= t;
        }
        neum_add(a.s[c], a.c[c], lower ? w[c] : w[c] * t);
    }
    a.m = lower ? e : a.m;
}

// b merged into a (a's terms first)
template <int CH> __device__ __forceinline__ void loo_merge(LooAcc<CH> &a, const LooAcc<CH> &b) {
    if (!(b.m < INFINITY))
        return;
    if (!(a.m < INFINITY)) {
        a = b;
        return;
    }
    const double m = a.m < b.m ? a.m : b.m;
    const double fa = exp(-(a.m - m)), fb = exp(-(b.m - m));
#pragma unroll
    for (int c = 0; c < CH; ++c) {
        double s = a.s[c] * fa, cc = a.c[c] * fa;
        neum_add(s, cc, b.s[c] * fb);
        neum_add(s, cc, b.c[c] * fb);
        a.s[c] = s;
        a.c[c] = cc;
    }
    a.m = m;
}

}  // namespace mecdf
