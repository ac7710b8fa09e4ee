// All-pairs kernels: Coulomb force and potential partial sums over j-splits.
//
// Work decomposition (MI355X, wave64):
//  - lane = i-particle; each lane owns P i-particles (i = wave_base + p*64 +
//    lane), kept in VGPRs with their accumulators;
//  - the j loop is uniform across the wave, so j-data (x_j, y_j, z_j, q_j) is
//    fetched with scalar loads and enters the FP64 VALU instructions as SGPR
//    operands: one fetch feeds 64*P pair interactions, with no LDS traffic
//    and no barriers (the GPU form of the paper's section 6.1 register reuse
//    of a packed j block);
//  - blockIdx.y = j-split s: the j range [s*jlen, min(n, (s+1)*jlen)) is
//    handled by its own workgroups, which write partial sums to
//    part[s][3][n]; a fixed-order sum over s follows (deterministic), so a
//    launch can fill 256 CUs even when n / (64 P) waves would not;
//  - the self pair is masked only in the j range that overlaps the wave's own
//    i range (the diagonal block); elsewhere the loop body has no select;
//  - blocked summation: each chunk of CHUNK j's is summed into a fresh
//    accumulator and then added to the running total, so rounding error
//    grows with sqrt(CHUNK) + sqrt(n / CHUNK) instead of sqrt(n).
#pragma once
#include <hip/hip_runtime.h>

#include "rsqrt.hpp"

namespace cb {

constexpr int kChunk = 128;  // j per blocked-summation chunk
constexpr int kUnroll = 8;   // j per unrolled group (one scalar fetch each)

template <int P>
struct IBlock {
    double x[P], y[P], z[P];
    int i[P];
};

template <int P, bool FORCE, bool POT>
struct Acc {
    double fx[P], fy[P], fz[P], ph[P];
    __device__ __forceinline__ void zero() {
#pragma unroll
        for (int p = 0; p < P; ++p) {
            if (FORCE) fx[p] = fy[p] = fz[p] = 0.0;
            if (POT) ph[p] = 0.0;
        }
    }
    __device__ __forceinline__ void add(const Acc& o) {
#pragma unroll
        for (int p = 0; p < P; ++p) {
            if (FORCE) {
                fx[p] += o.fx[p];
                fy[p] += o.fy[p];
                fz[p] += o.fz[p];
            }
            if (POT) ph[p] += o.ph[p];
        }
    }
    // this += c o (a chunk of one j charge c, summed without it)
    __device__ __forceinline__ void add_scaled(const Acc& o, double c) {
#pragma unroll
        for (int p = 0; p < P; ++p) {
            if (FORCE) {
                fx[p] = __builtin_fma(c, o.fx[p], fx[p]);
                fy[p] = __builtin_fma(c, o.fy[p], fy[p]);
                fz[p] = __builtin_fma(c, o.fz[p], fz[p]);
            }
            if (POT) ph[p] = __builtin_fma(c, o.ph[p], ph[p]);
        }
    }
};

// Whether every ion of [j0, j1) carries one charge, and that charge (qJ):
// the range's pairs then need no per-pair charge load or multiply (ions
// grouped by species, the paper's split of species into separate N-body
// sub-problems in section 2).  Wave-uniform; a non-finite charge makes it
// false.  Every lane of the wave must call it.
__device__ __forceinline__ bool range_charge(const double* __restrict__ q, int j0, int j1, double& qJ) {
    double lo = 0.0, hi = 0.0;
    bool fin = true;
    if (j1 > j0) lo = hi = q[j0];
    for (int j = j0 + (int)__lane_id(); j < j1; j += 64) {
        const double v = q[j];
        lo = fmin(lo, v);
        hi = fmax(hi, v);
        fin = fin && __builtin_isfinite(v);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        lo = fmin(lo, __shfl_xor(lo, o));
        hi = fmax(hi, __shfl_xor(hi, o));
    }
    qJ = lo;
    return __builtin_amdgcn_ballot_w64(!fin) == 0 && lo == hi;
}

// One pair (i, j): acc += q_j d / (r^2+eps2)^{3/2} and/or q_j / (r^2+eps2)^{1/2}
// (qj = 1 in ranges of one charge, which the caller applies per chunk).
template <int PREC, int P, bool FORCE, bool POT, bool MASK>
__device__ __forceinline__ void pair_j(const IBlock<P>& ib, Acc<P, FORCE, POT>& a, double xj, double yj,
                                       double zj, double qj, double eps2, int j, const SeriesK& K) {
#pragma unroll
    for (int p = 0; p < P; ++p) {
        double dx = ib.x[p] - xj;
        double dy = ib.y[p] - yj;
        double dz = ib.z[p] - zj;
        if (PREC == PREC_F32D) {
            dx = (double)(float)dx;
            dy = (double)(float)dy;
            dz = (double)(float)dz;
        }
        const double r2 = __builtin_fma(dx, dx, __builtin_fma(dy, dy, __builtin_fma(dz, dz, eps2)));
        double s, r;
        inv_r<PREC, FORCE, POT>(r2, qj, K, s, r);
        if (FORCE) {
            if (MASK) s = (ib.i[p] == j) ? 0.0 : s;
            a.fx[p] = __builtin_fma(dx, s, a.fx[p]);
            a.fy[p] = __builtin_fma(dy, s, a.fy[p]);
            a.fz[p] = __builtin_fma(dz, s, a.fz[p]);
        }
        if (POT) {
            if (MASK) r = (ib.i[p] == j) ? 0.0 : r;
            a.ph[p] = __builtin_fma(qj, r, a.ph[p]);
        }
    }
}

// UNI: every j of the range has charge qJ; the pairs are summed without it
// and each chunk's sums are scaled by qJ.
template <int PREC, int P, bool FORCE, bool POT, bool MASK, bool UNI>
__device__ __forceinline__ void pair_range(const IBlock<P>& ib, Acc<P, FORCE, POT>& tot, int ja, int jb,
                                           const double* __restrict__ x, const double* __restrict__ y,
                                           const double* __restrict__ z, const double* __restrict__ q,
                                           double eps2, double qJ, const SeriesK& K) {
    for (int jc = ja; jc < jb; jc += kChunk) {
        const int je = min(jb, jc + kChunk);
        Acc<P, FORCE, POT> a;
        a.zero();
        int j = jc;
        for (; j + kUnroll <= je; j += kUnroll) {
#pragma unroll
            for (int u = 0; u < kUnroll; ++u)
                pair_j<PREC, P, FORCE, POT, MASK>(ib, a, x[j + u], y[j + u], z[j + u], UNI ? 1.0 : q[j + u], eps2,
                                                  j + u, K);
        }
        for (; j < je; ++j) pair_j<PREC, P, FORCE, POT, MASK>(ib, a, x[j], y[j], z[j], UNI ? 1.0 : q[j], eps2, j, K);
        if (UNI)
            tot.add_scaled(a, qJ);
        else
            tot.add(a);
    }
}

// The j-split [j0, j1) of the wave at ibase: pairs before its own i-block,
// the diagonal (self pair masked), and after.
template <int PREC, int P, bool FORCE, bool POT, bool UNI>
__device__ __forceinline__ void pair_split(const IBlock<P>& ib, Acc<P, FORCE, POT>& tot, int ibase, int j0, int j1,
                                           const double* __restrict__ x, const double* __restrict__ y,
                                           const double* __restrict__ z, const double* __restrict__ q,
                                           double eps2, double qJ, const SeriesK& K) {
    const int dlo = max(j0, ibase), dhi = min(j1, ibase + 64 * P);
    pair_range<PREC, P, FORCE, POT, false, UNI>(ib, tot, j0, min(j1, ibase), x, y, z, q, eps2, qJ, K);
    if (dlo < dhi) pair_range<PREC, P, FORCE, POT, true, UNI>(ib, tot, dlo, dhi, x, y, z, q, eps2, qJ, K);
    pair_range<PREC, P, FORCE, POT, false, UNI>(ib, tot, max(j0, ibase + 64 * P), j1, x, y, z, q, eps2, qJ, K);
}

// part: [S][3][n] force partials (FORCE), ppot: [S][n] potential partials
// (POT); S = gridDim.y.  Workgroup = blockDim.x threads = blockDim.x/64 waves.
// The i's are i0 .. i0 + ni - 1 (all n for a whole force evaluation); the
// partial sums are indexed by i - i0: part[s][c][ni], ppot[s][ni].
template <int PREC, int P, bool FORCE, bool POT>
__global__ void __launch_bounds__(256) k_pair(int n, int i0, int ni, const double* __restrict__ x,
                                              const double* __restrict__ y, const double* __restrict__ z,
                                              const double* __restrict__ q, double eps2, int jlen,
                                              double* __restrict__ part, double* __restrict__ ppot) {
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int rbase = (blockIdx.x * (blockDim.x >> 6) + wave) * (64 * P);  // relative to i0
    if (rbase >= ni) return;
    const int ibase = i0 + rbase;
    const int iend = i0 + ni;
    const int s = blockIdx.y;
    const int j0 = s * jlen;
    const int j1 = min(n, j0 + jlen);

    IBlock<P> ib;
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const int i = ibase + p * 64 + lane;
        const int ic = min(i, iend - 1);
        ib.i[p] = i;
        ib.x[p] = x[ic];
        ib.y[p] = y[ic];
        ib.z[p] = z[ic];
    }
    Acc<P, FORCE, POT> tot;
    tot.zero();
    const SeriesK K;
    double qJ;
    if (range_charge(q, j0, j1, qJ))
        pair_split<PREC, P, FORCE, POT, true>(ib, tot, ibase, j0, j1, x, y, z, q, eps2, qJ, K);
    else
        pair_split<PREC, P, FORCE, POT, false>(ib, tot, ibase, j0, j1, x, y, z, q, eps2, 1.0, K);

#pragma unroll
    for (int p = 0; p < P; ++p) {
        const int i = ib.i[p];
        if (i < iend) {
            const int r = i - i0;
            if (FORCE) {
                part[(size_t)(s * 3 + 0) * ni + r] = tot.fx[p];
                part[(size_t)(s * 3 + 1) * ni + r] = tot.fy[p];
                part[(size_t)(s * 3 + 2) * ni + r] = tot.fz[p];
            }
            if (POT) ppot[(size_t)s * ni + r] = tot.ph[p];
        }
    }
}

}  // namespace cb
