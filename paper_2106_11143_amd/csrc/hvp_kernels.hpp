// Hessian-vector products of the Coulomb energy (all pairs), NV vectors per
// pass sharing the pair geometry.
//
// For the pair term k_C q_i q_j (|d|^2 + eps2)^{-1/2}, d = r_i - r_j, the
// 3x3 Hessian block is k_C q_i q_j (3 d d^T s^5 - I s^3) on the diagonal and
// its negative off it, so
//   (H v)_i = k_C q_i sum_{j != i} q_j [3 d (d . u) s^5 - u s^3],  u = v_i - v_j.
// Decomposition as in the force kernel: lane = i-particle (P per lane), the
// j loop uniform across the wave with j-data (x, y, z, q and the NV vectors'
// components at j) in SGPRs, j-splits writing partials [S][NV][3][n], the self
// pair masked only in the diagonal block, blocked summation per chunk.
#pragma once
#include <hip/hip_runtime.h>

#include "rsqrt.hpp"

namespace cb {

constexpr int kHvpChunk = 128;

// s3 = q r^{-3} and s5 = 3 q r^{-5} from r^2 (same refinement as the force).
template <int PREC>
__device__ __forceinline__ void hvp_scales(double r2, double q, const SeriesK& K, double& s3, double& s5) {
    if (PREC == PREC_IEEE) {
        const double r = 1.0 / __builtin_sqrt(r2);
        s3 = r * r * r * q;
        s5 = 3.0 * s3 * (r * r);
    } else if (PREC == PREC_FP32) {
        const double y0 = rsq_seed(r2);
        const double t = y0 * y0;
        s3 = (y0 * q) * t;
        s5 = 3.0 * s3 * t;
    } else {
        const double y0 = rsq_seed(r2);
        const double t = y0 * y0;
        const double e = __builtin_fma(-r2, t, 1.0);
        const double w = (y0 * q) * t;
        // r^{-2} = t / (1 - e) = t (1 + e + e^2 + ...)
        double y2;
        if (PREC == PREC_FP64) {
            const double p = __builtin_fma(e, K.c1875, K.c15);
            s3 = __builtin_fma(w, e * p, w);
            y2 = __builtin_fma(t, __builtin_fma(e, e, e), t);
        } else {
            s3 = __builtin_fma(w, K.c15 * e, w);
            y2 = __builtin_fma(t, e, t);
        }
        s5 = 3.0 * s3 * y2;
    }
}

template <int P, int NV>
struct HvpI {
    double x[P], y[P], z[P];
    double v[NV][3][P];
    int i[P];
};

template <int P, int NV>
struct HvpAcc {
    double h[NV][3][P];
    __device__ __forceinline__ void zero() {
#pragma unroll
        for (int b = 0; b < NV; ++b)
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int p = 0; p < P; ++p) h[b][c][p] = 0.0;
    }
    __device__ __forceinline__ void add(const HvpAcc& o) {
#pragma unroll
        for (int b = 0; b < NV; ++b)
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int p = 0; p < P; ++p) h[b][c][p] += o.h[b][c][p];
    }
};

template <int PREC, int P, int NV, bool MASK>
__device__ __forceinline__ void hvp_pair(const HvpI<P, NV>& ib, HvpAcc<P, NV>& a, int j, int n,
                                         const double* __restrict__ x, const double* __restrict__ y,
                                         const double* __restrict__ z, const double* __restrict__ q,
                                         const double* __restrict__ v, double eps2, const SeriesK& K) {
    const double xj = x[j], yj = y[j], zj = z[j], qj = q[j];
    double vj[NV][3];
#pragma unroll
    for (int b = 0; b < NV; ++b)
#pragma unroll
        for (int c = 0; c < 3; ++c) vj[b][c] = v[((size_t)b * 3 + c) * n + j];
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const double dx = ib.x[p] - xj, dy = ib.y[p] - yj, dz = ib.z[p] - zj;
        const double r2 = __builtin_fma(dx, dx, __builtin_fma(dy, dy, __builtin_fma(dz, dz, eps2)));
        double s3, s5;
        hvp_scales<PREC>(r2, qj, K, s3, s5);
        if (MASK && ib.i[p] == j) {
            s3 = 0.0;
            s5 = 0.0;
        }
#pragma unroll
        for (int b = 0; b < NV; ++b) {
            const double ux = ib.v[b][0][p] - vj[b][0];
            const double uy = ib.v[b][1][p] - vj[b][1];
            const double uz = ib.v[b][2][p] - vj[b][2];
            const double dot = __builtin_fma(dx, ux, __builtin_fma(dy, uy, dz * uz));
            const double c = dot * s5;
            a.h[b][0][p] = __builtin_fma(dx, c, __builtin_fma(-ux, s3, a.h[b][0][p]));
            a.h[b][1][p] = __builtin_fma(dy, c, __builtin_fma(-uy, s3, a.h[b][1][p]));
            a.h[b][2][p] = __builtin_fma(dz, c, __builtin_fma(-uz, s3, a.h[b][2][p]));
        }
    }
}

template <int PREC, int P, int NV, bool MASK>
__device__ __forceinline__ void hvp_range(const HvpI<P, NV>& ib, HvpAcc<P, NV>& tot, int ja, int jb, int n,
                                          const double* __restrict__ x, const double* __restrict__ y,
                                          const double* __restrict__ z, const double* __restrict__ q,
                                          const double* __restrict__ v, double eps2, const SeriesK& K) {
    constexpr int U = NV <= 2 ? 4 : (NV <= 4 ? 2 : 1);
    for (int jc = ja; jc < jb; jc += kHvpChunk) {
        const int je = min(jb, jc + kHvpChunk);
        HvpAcc<P, NV> a;
        a.zero();
        int j = jc;
        for (; j + U <= je; j += U) {
#pragma unroll
            for (int u = 0; u < U; ++u) hvp_pair<PREC, P, NV, MASK>(ib, a, j + u, n, x, y, z, q, v, eps2, K);
        }
        for (; j < je; ++j) hvp_pair<PREC, P, NV, MASK>(ib, a, j, n, x, y, z, q, v, eps2, K);
        tot.add(a);
    }
}

// part: [S][NV][3][n]; v: [NV][3][n].
template <int PREC, int P, int NV>
__global__ void __launch_bounds__(256) k_hvp(int n, const double* __restrict__ x, const double* __restrict__ y,
                                             const double* __restrict__ z, const double* __restrict__ q,
                                             const double* __restrict__ v, double eps2, int jlen,
                                             double* __restrict__ part) {
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int ibase = (blockIdx.x * (blockDim.x >> 6) + wave) * (64 * P);
    if (ibase >= n) return;
    const int s = blockIdx.y;
    const int j0 = s * jlen;
    const int j1 = min(n, j0 + jlen);
    HvpI<P, NV> ib;
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const int i = ibase + p * 64 + lane;
        const int ic = min(i, n - 1);
        ib.i[p] = i;
        ib.x[p] = x[ic];
        ib.y[p] = y[ic];
        ib.z[p] = z[ic];
#pragma unroll
        for (int b = 0; b < NV; ++b)
#pragma unroll
            for (int c = 0; c < 3; ++c) ib.v[b][c][p] = v[((size_t)b * 3 + c) * n + ic];
    }
    HvpAcc<P, NV> tot;
    tot.zero();
    const SeriesK K;
    const int dlo = max(j0, ibase), dhi = min(j1, ibase + 64 * P);
    hvp_range<PREC, P, NV, false>(ib, tot, j0, min(j1, ibase), n, x, y, z, q, v, eps2, K);
    if (dlo < dhi) hvp_range<PREC, P, NV, true>(ib, tot, dlo, dhi, n, x, y, z, q, v, eps2, K);
    hvp_range<PREC, P, NV, false>(ib, tot, max(j0, ibase + 64 * P), j1, n, x, y, z, q, v, eps2, K);
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const int i = ib.i[p];
        if (i < n) {
#pragma unroll
            for (int b = 0; b < NV; ++b)
#pragma unroll
                for (int c = 0; c < 3; ++c) part[(((size_t)s * NV + b) * 3 + c) * n + i] = tot.h[b][c][p];
        }
    }
}

}  // namespace cb
