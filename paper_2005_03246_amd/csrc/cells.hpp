// The cell of a coordinate among the nodes of one grid axis, shared by the
// grid ECDF and the grid kernel sums.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mecdf {

// Number of nodes strictly below v: the cell of eq. (partial_sums) holding v,
// cell c meaning z_{c-1} < v <= z_c (z_{-1} = -inf, z_M = +inf).  NaN maps
// to 0 and is filtered by the caller.
template <typename NodePtr>
__device__ __forceinline__ uint32_t cell_index(NodePtr z, int M, double z0, double zl,
                                               double gs, double v) {
    if (!(v > z0))
        return 0u;
    if (v > zl)
        return (uint32_t)M;
    // z0 < v <= zl: the answer is in [1, M-1].  Guess by mesh division (the
    // uniform-grid index of Appendix A.2) and check it exactly.
    const int c = (int)fmin(fmax(ceil((v - z0) * gs), 1.0), (double)(M - 1));
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

}  // namespace mecdf
