// Fixed-order sum of j-split partials in the element-wise kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>

namespace cb {

// sum_{s < S} p[s * stride], added in split order.  The partials were just
// written by other CUs, so every load is a full memory round trip: the loads
// of 8 splits are issued before their sums.
__device__ __forceinline__ double split_sum(const double* __restrict__ p, size_t stride, int S) {
    constexpr int U = 8;
    double acc = 0.0;
    int s = 0;
    for (; s + U <= S; s += U) {
        double a[U];
#pragma unroll
        for (int u = 0; u < U; ++u) a[u] = p[(size_t)(s + u) * stride];
#pragma unroll
        for (int u = 0; u < U; ++u) acc += a[u];
    }
    for (; s < S; ++s) acc += p[(size_t)s * stride];
    return acc;
}

}  // namespace cb
