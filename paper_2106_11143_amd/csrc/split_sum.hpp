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

// The same sum for NA arrays at once, out[a] = sum_{s < S} p[a][s * stride[a]]:
// the loads of U splits of every array are issued before their sums, so NA
// arrays cost the round trips of one.  Each sum is in split order, as above.
template <int NA, int U = 8>
__device__ __forceinline__ void split_sums(const double* const (&p)[NA], const size_t (&stride)[NA], int S,
                                           double (&out)[NA]) {
#pragma unroll
    for (int c = 0; c < NA; ++c) out[c] = 0.0;
    int s = 0;
    for (; s + U <= S; s += U) {
        double a[NA][U];
#pragma unroll
        for (int c = 0; c < NA; ++c)
#pragma unroll
            for (int u = 0; u < U; ++u) a[c][u] = p[c][(size_t)(s + u) * stride[c]];
#pragma unroll
        for (int c = 0; c < NA; ++c)
#pragma unroll
            for (int u = 0; u < U; ++u) out[c] += a[c][u];
    }
    for (; s < S; ++s)
#pragma unroll
        for (int c = 0; c < NA; ++c) out[c] += p[c][(size_t)s * stride[c]];
}

}  // namespace cb
