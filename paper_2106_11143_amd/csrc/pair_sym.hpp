// All-pairs Coulomb force using Newton's third law: each unordered pair is
// evaluated once and its force is applied to both ions, halving the pair
// arithmetic of the paper's double loop (section 3).
//
// Tiling.  Ions are cut into i-blocks of IB = 64 P (one wave, P ions per
// lane).  Row I of the upper triangle holds the ions j >= (I+1) IB; it is cut
// into segments of JL ions.  One tile = (row I, segment s) = one workgroup of
// one wave.  Per j (uniform across the wave, fetched by scalar loads into
// SGPRs) each lane evaluates its P pairs once and
//   - adds q_i q_j d y^3 to its own i accumulators (force on i, up to k_C);
//   - adds q_i d y^3 over its P ions into a per-j value; after 8 j's the 24
//     per-j values (8 j x 3 components) are summed over the wave by a
//     reduce-scatter (wave_reduce.hpp), giving the reaction on those 8 j
//     (up to -k_C q_j), which one lane per value stores.
// The tile writes its i sums to Pi[tile][3][IB] and its reactions to
// R[tile][3][JL]; nothing is accumulated across workgroups, so results are
// deterministic.  The diagonal i-block (pairs inside one block) is evaluated
// directly by the finish kernel, which then adds, per ion, its i sums over
// the segments of its row and its reactions from every row above, in a
// fixed order.
#pragma once
#include <hip/hip_runtime.h>

#include "rsqrt.hpp"
#include "step_common.hpp"
#include "wave_reduce.hpp"

namespace cb {

// Segments of row I: ceil((n - (I+1) IB) / JL), or 0.
__host__ __device__ __forceinline__ int sym_nseg(int n, int IB, int JL, int I) {
    const long long a = (long long)n - (long long)(I + 1) * IB;
    return a > 0 ? (int)((a + JL - 1) / JL) : 0;
}

// rowstart[I] = first tile of row I (exclusive prefix sum), rowstart[nI] = tiles.
__global__ void k_sym_rows(int n, int IB, int JL, int nI, int* __restrict__ rowstart) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        int acc = 0;
        for (int I = 0; I < nI; ++I) {
            rowstart[I] = acc;
            acc += sym_nseg(n, IB, JL, I);
        }
        rowstart[nI] = acc;
    }
}

__global__ void k_sym_fill(int n, int IB, int JL, int nI, const int* __restrict__ rowstart, int2* __restrict__ tiles) {
    const int I = blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= nI) return;
    const int s0 = rowstart[I], ns = sym_nseg(n, IB, JL, I);
    for (int s = 0; s < ns; ++s) tiles[s0 + s] = make_int2(I, s);
}

// s = q r^{-3} refined as in the direct kernel (the series on r^-3).
template <int PREC>
__device__ __forceinline__ double sym_s(double r2, double q, const SeriesK& K) {
    double s, y;
    inv_r<PREC, true, false>(r2, q, K, s, y);
    return s;
}

// One group of 8 j's (jg .. jg+7; only the first cnt are live when TAIL):
// i sums into ia, the 8 reactions reduced over the wave and stored.
template <int PREC, int P, bool TAIL>
__device__ __forceinline__ void sym_group(int jg, int cnt, int j0, int JL, const double* __restrict__ x,
                                          const double* __restrict__ y, const double* __restrict__ z,
                                          const double* __restrict__ q, double eps2, const double (&xi)[P],
                                          const double (&yi)[P], const double (&zi)[P], const double (&qi)[P],
                                          double (&ia)[P][3], const SeriesK& K, double* __restrict__ Rt) {
    double jv[24];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const int j = TAIL ? jg + min(u, cnt - 1) : jg + u;
        const double xj = x[j], yj = y[j], zj = z[j], qj = q[j];
        double a0 = 0.0, a1 = 0.0, a2 = 0.0;
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const double dx = xi[p] - xj, dy = yi[p] - yj, dz = zi[p] - zj;
            const double r2 = __builtin_fma(dx, dx, __builtin_fma(dy, dy, __builtin_fma(dz, dz, eps2)));
            double s = sym_s<PREC>(r2, qi[p], K);  // q_i r^-3
            if (TAIL && u >= cnt) s = 0.0;
            const double sq = s * qj;  // q_i q_j r^-3
            ia[p][0] = __builtin_fma(dx, sq, ia[p][0]);
            ia[p][1] = __builtin_fma(dy, sq, ia[p][1]);
            ia[p][2] = __builtin_fma(dz, sq, ia[p][2]);
            a0 = __builtin_fma(dx, s, a0);
            a1 = __builtin_fma(dy, s, a1);
            a2 = __builtin_fma(dz, s, a2);
        }
        jv[u * 3 + 0] = a0;
        jv[u * 3 + 1] = a1;
        jv[u * 3 + 2] = a2;
    }
    double o[3];
    reduce_scatter24(jv, o);
    const int lane = threadIdx.x;
    const int g = lane >> 3, c = lane & 7;
    if ((!TAIL || g < cnt) && c < 3) Rt[(size_t)c * JL + (jg - j0) + g] = (c == 0) ? o[0] : ((c == 1) ? o[1] : o[2]);
}

template <int PREC, int P>
__global__ void __launch_bounds__(64, (P <= 2 ? 3 : 2)) k_pair_sym(int n, const double* __restrict__ x, const double* __restrict__ y,
                                                 const double* __restrict__ z, const double* __restrict__ q,
                                                 double eps2, int JL, const int2* __restrict__ tiles,
                                                 double* __restrict__ Pi, double* __restrict__ R) {
    constexpr int IB = 64 * P;
    const int t = blockIdx.x;
    const int2 tl = tiles[t];
    const int I = tl.x, sg = tl.y;
    const int lane = threadIdx.x;
    double xi[P], yi[P], zi[P], qi[P], ia[P][3];
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const int i = I * IB + p * 64 + lane;  // rows with tiles are full blocks
        xi[p] = x[i];
        yi[p] = y[i];
        zi[p] = z[i];
        qi[p] = q[i];
        ia[p][0] = ia[p][1] = ia[p][2] = 0.0;
    }
    const SeriesK K;
    const int j0 = (I + 1) * IB + sg * JL;
    const int j1 = min(n, j0 + JL);
    double* Rt = R + (size_t)t * 3 * JL;
    int jg = j0;
    for (; jg + 8 <= j1; jg += 8)
        sym_group<PREC, P, false>(jg, 8, j0, JL, x, y, z, q, eps2, xi, yi, zi, qi, ia, K, Rt);
    if (jg < j1) sym_group<PREC, P, true>(jg, j1 - jg, j0, JL, x, y, z, q, eps2, xi, yi, zi, qi, ia, K, Rt);
    double* Pt = Pi + (size_t)t * 3 * IB;
#pragma unroll
    for (int p = 0; p < P; ++p)
#pragma unroll
        for (int c = 0; c < 3; ++c) Pt[(size_t)c * IB + p * 64 + lane] = ia[p][c];
}

// Per ion k: direct pairs inside its own i-block, plus its i sums over the
// segments of its row, minus q_k times its reactions from the rows above;
// writes the finished force F = k_C (...) to F[3][n].  A wave's 64 ions lie
// in one i-block (IB is a multiple of 64), so the block's j loop is uniform.
template <int PREC>
__global__ void __launch_bounds__(256) k_sym_finish(int n, int IB, int JL, const double* __restrict__ x,
                                                    const double* __restrict__ y, const double* __restrict__ z,
                                                    const double* __restrict__ q, double eps2,
                                                    const int* __restrict__ rowstart,
                                                    const double* __restrict__ Pi, const double* __restrict__ R,
                                                    double* __restrict__ F) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int wbase = __builtin_amdgcn_readfirstlane(blockIdx.x * blockDim.x + (threadIdx.x & ~63));
    if (wbase >= n) return;
    const int kc = min(k, n - 1);
    const int Ik = wbase / IB;
    const int b0 = Ik * IB, b1 = min(n, b0 + IB);
    const double xk = x[kc], yk = y[kc], zk = z[kc];
    const SeriesK K;
    double d0 = 0.0, d1 = 0.0, d2 = 0.0;
    for (int j = b0; j < b1; ++j) {
        const double dx = xk - x[j], dy = yk - y[j], dz = zk - z[j];
        const double r2 = __builtin_fma(dx, dx, __builtin_fma(dy, dy, __builtin_fma(dz, dz, eps2)));
        double s = sym_s<PREC>(r2, q[j], K);
        if (j == kc) s = 0.0;
        d0 = __builtin_fma(dx, s, d0);
        d1 = __builtin_fma(dy, s, d1);
        d2 = __builtin_fma(dz, s, d2);
    }
    if (k >= n) return;
    const int off = k - b0;
    double p0 = 0.0, p1 = 0.0, p2 = 0.0;
    const int r0 = rowstart[Ik], r1 = rowstart[Ik + 1];
    for (int t = r0; t < r1; ++t) {
        const double* Pt = Pi + (size_t)t * 3 * IB + off;
        p0 += Pt[0];
        p1 += Pt[IB];
        p2 += Pt[2 * IB];
    }
    double e0 = 0.0, e1 = 0.0, e2 = 0.0;
    for (int I = 0; I < Ik; ++I) {
        const int rel = k - (I + 1) * IB;
        const int sI = rel / JL;
        const double* Rt = R + (size_t)(rowstart[I] + sI) * 3 * JL + (rel - sI * JL);
        e0 += Rt[0];
        e1 += Rt[JL];
        e2 += Rt[2 * JL];
    }
    const double qk = q[k];
    F[k] = kCoulomb * (p0 + qk * (d0 - e0));
    F[(size_t)n + k] = kCoulomb * (p1 + qk * (d1 - e1));
    F[2 * (size_t)n + k] = kCoulomb * (p2 + qk * (d2 - e2));
}

}  // namespace cb
