// Hessian-vector products by Newton's third law: each unordered pair (i, j)
// evaluated once for NV vectors.
//
// With d = r_i - r_j, u = v_i - v_j and y = (|d|^2 + eps2)^{-1/2}, ion i's
// pair term is k_C q_i q_j T_ij with T_ij = 3 d (d . u) y^5 - u y^3
// = y^3 (3 y^2 (d . u) d - u), and T_ji = -T_ij (d and u both change sign).  So, as for the force
// (pair_sym.hpp), a tile of i-block I and j-segment s evaluates T once per
// pair, adds q_i q_j T_ij to i's sums and the wave's sum over i of q_i T_ij
// to j's reaction (the finish scales it by -k_C q_j).  The same tile table,
// partial layout per vector and fixed-order finish as the force stage.
//
// Per lane: P i-particles with their NV vectors' components; per j (uniform,
// one 16-double record of position, charge and vector components read by
// scalar loads, the next j requested before the current is evaluated).  The
// 3 NV reaction values of each j are kept for 4 / NV j's, i.e. 12 values,
// and summed over the wave together by lds_reduce12.  Tiles of one charge per
// side (ions grouped by species) drop q_i and q_j from the pair loop and
// scale the partials when they are stored.
#pragma once
#include <hip/hip_runtime.h>

#include "hvp_kernels.hpp"
#include "pair_sym.hpp"
#include "step_common.hpp"

namespace cb {

constexpr int kHvpRec = 16;  // doubles per packed j record: x, y, z, q, v[b][c] (b < 4)

// J[i] = (x, y, z, q, v[0][0..2], ..., v[nv-1][0..2], 0 ...) for one pass of
// nv <= 4 vectors; pass blockIdx.y takes vectors nv blockIdx.y ... and writes
// its records n kHvpRec doubles further on.  With nG > 0 the launch has one
// more column of blocks, whose first block writes the tile table of nG row
// groups (sym_plan_fill, W = 1) instead, so that the table costs no launch
// of its own.
__global__ void __launch_bounds__(256) k_hvp_pack(int n, int nv, const double* __restrict__ x,
                                                  const double* __restrict__ y, const double* __restrict__ z,
                                                  const double* __restrict__ q, const double* __restrict__ v,
                                                  double* __restrict__ J, int IB, int JL, int nG,
                                                  int* __restrict__ rowstart, int2* __restrict__ tiles) {
    if (nG > 0 && blockIdx.x == gridDim.x - 1) {
        if (blockIdx.y == 0) sym_plan_fill<256>(n, IB, JL, 1, nG, rowstart, tiles);
        return;
    }
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    v += (size_t)blockIdx.y * nv * 3 * n;
    double* r = J + ((size_t)blockIdx.y * n + i) * kHvpRec;
    r[0] = x[i];
    r[1] = y[i];
    r[2] = z[i];
    r[3] = q[i];
#pragma unroll
    for (int k = 0; k < 12; ++k) r[4 + k] = (k / 3) < nv ? v[(size_t)k * n + i] : 0.0;
}

template <int NV>
struct HvpJRec {
    double x, y, z, q, v[NV][3];
};

template <int NV>
__device__ __forceinline__ HvpJRec<NV> load_hvp_j(const double* __restrict__ J, int j) {
    const double* r = J + (size_t)j * kHvpRec;
    HvpJRec<NV> a;
    a.x = r[0];
    a.y = r[1];
    a.z = r[2];
    a.q = r[3];
#pragma unroll
    for (int b = 0; b < NV; ++b)
#pragma unroll
        for (int c = 0; c < 3; ++c) a.v[b][c] = r[4 + 3 * b + c];
    return a;
}

// q y^3 and 3 y^2 from r^2 + eps2 (the refinement of the force, section 4 of
// the paper, with r^-2 = t (1 + e + e^2 + ...) from the same estimate).  The
// pair term is then T = y^3 (w d - u) with w = 3 y^2 (d . u): per vector three
// products fewer than 3 d (d . u) y^5 - u y^3 written out.
template <int PREC>
__device__ __forceinline__ void hvp_scales_w(double r2, double q, const SeriesK& K, double& s3, double& g3) {
    if (PREC == PREC_IEEE) {
        const double r = 1.0 / __builtin_sqrt(r2);
        const double y2 = r * r;
        s3 = y2 * r * q;
        g3 = 3.0 * y2;
    } else if (PREC == PREC_FP32) {
        const double y0 = rsq_seed(r2);
        const double t = y0 * y0;
        s3 = (y0 * q) * t;
        g3 = 3.0 * t;
    } else {
        const double y0 = rsq_seed(r2);
        const double t = y0 * y0;
        const double e = __builtin_fma(-r2, t, 1.0);
        const double w = (y0 * q) * t;
        const double t3 = 3.0 * t;
        if (PREC == PREC_FP64) {
            const double p = __builtin_fma(e, K.c1875, K.c15);
            s3 = __builtin_fma(w, e * p, w);
            g3 = __builtin_fma(t3, __builtin_fma(e, e, e), t3);
        } else {
            s3 = __builtin_fma(w, K.c15 * e, w);
            g3 = __builtin_fma(t3, e, t3);
        }
    }
}

// Pairs of one j with the lane's P ions: i sums into ia[p][b][c] (q_i q_j T,
// or T when UNI), this lane's share of j's reaction (sum over p of q_i T, or
// T) into sh[b][c].
template <int PREC, int P, int NV, bool UNI>
__device__ __forceinline__ void hvp_sym_pair(const HvpJRec<NV>& J, double eps2, const double (&xi)[P],
                                             const double (&yi)[P], const double (&zi)[P], const double (&qi)[P],
                                             const double (&vi)[NV][3][P], double (&ia)[P][NV][3],
                                             double (&sh)[NV][3], const SeriesK& K) {
#pragma unroll
    for (int b = 0; b < NV; ++b) sh[b][0] = sh[b][1] = sh[b][2] = 0.0;
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const double dx = xi[p] - J.x, dy = yi[p] - J.y, dz = zi[p] - J.z;
        const double r2 = __builtin_fma(dx, dx, __builtin_fma(dy, dy, __builtin_fma(dz, dz, eps2)));
        double s3, g3;  // q_i y^3 (y^3 when UNI) and 3 y^2
        hvp_scales_w<PREC>(r2, UNI ? 1.0 : qi[p], K, s3, g3);
        const double a3 = UNI ? s3 : s3 * J.q;  // q_i q_j y^3
#pragma unroll
        for (int b = 0; b < NV; ++b) {
            const double ux = vi[b][0][p] - J.v[b][0];
            const double uy = vi[b][1][p] - J.v[b][1];
            const double uz = vi[b][2][p] - J.v[b][2];
            const double w = __builtin_fma(dx, ux, __builtin_fma(dy, uy, dz * uz)) * g3;
            const double vx = __builtin_fma(w, dx, -ux);  // T / y^3
            const double vy = __builtin_fma(w, dy, -uy);
            const double vz = __builtin_fma(w, dz, -uz);
            ia[p][b][0] = __builtin_fma(a3, vx, ia[p][b][0]);
            ia[p][b][1] = __builtin_fma(a3, vy, ia[p][b][1]);
            ia[p][b][2] = __builtin_fma(a3, vz, ia[p][b][2]);
            sh[b][0] = __builtin_fma(s3, vx, sh[b][0]);
            sh[b][1] = __builtin_fma(s3, vy, sh[b][1]);
            sh[b][2] = __builtin_fma(s3, vz, sh[b][2]);
        }
    }
}

// Waves per SIMD the register budget of k_hvp_sym is sized for (each lane
// holds 6 NV + 4 doubles per i-particle and 3 NV sums; at these targets the
// variants spill at most a few registers).
template <int P, int NV>
constexpr int hvp_sym_waves() {
    return P == 1 ? (NV == 4 ? 3 : 4) : (P == 2 ? (NV == 4 ? 2 : (NV == 2 ? 3 : 4)) : (NV == 1 ? 3 : 2));
}

// The j loop of tile t over [j0, j1) and the stores of its partials:
// Pi[t][NV][3][IB] and R[t][NV][3][JL].
template <int PREC, int P, int NV, bool UNI>
__device__ __forceinline__ void hvp_sym_body(const double* __restrict__ J, double eps2, int JL, int j0, int j1, int t,
                                             const double (&xi)[P], const double (&yi)[P], const double (&zi)[P],
                                             const double (&qi)[P], const double (&vi)[NV][3][P], double qI,
                                             double qJ, double* __restrict__ red, double* __restrict__ Pi,
                                             double* __restrict__ R) {
    constexpr int IB = 64 * P;
    constexpr int GJ = 4 / NV;  // j's whose 3 NV reaction values make one 12-value wave sum
    const int lane = threadIdx.x;
    double ia[P][NV][3];
#pragma unroll
    for (int p = 0; p < P; ++p)
#pragma unroll
        for (int b = 0; b < NV; ++b) ia[p][b][0] = ia[p][b][1] = ia[p][b][2] = 0.0;
    const SeriesK K;
    double* Rt = R + (size_t)t * NV * 3 * JL;
    // one group's wave sums are in flight while the next group is evaluated:
    // the loads of group pjg are requested after its evaluation and added
    // (and stored) after the evaluation of the following group
    double2 a[8];
    int pjg = -1, plive = 0;
    const int v = lane >> 2;  // value v = (g NV + b) 3 + c of quad v
    auto store = [&](int jgs, int lv) {
        const double o = lds_sum12(a);
        if ((lane & 3) == 0 && v < 12) {
            const int g = v / (3 * NV), b = (v / 3) % NV, c = v % 3;
            if (g < lv) Rt[(size_t)(b * 3 + c) * JL + (jgs - j0) + g] = UNI ? o * qI : o;
        }
    };
    HvpJRec<NV> cur = load_hvp_j<NV>(J, j0);
    for (int jg = j0; jg < j1; jg += GJ) {
        const int live = min(GJ, j1 - jg);
        double sh[GJ][NV][3];
#pragma unroll
        for (int g = 0; g < GJ; ++g) {
            // the next j's record is requested before this j is evaluated
            const HvpJRec<NV> nxt = load_hvp_j<NV>(J, min(jg + g + 1, j1 - 1));
            __builtin_amdgcn_sched_barrier(0);
            if (g < live) {
                hvp_sym_pair<PREC, P, NV, UNI>(cur, eps2, xi, yi, zi, qi, vi, ia, sh[g], K);
            } else {
#pragma unroll
                for (int b = 0; b < NV; ++b) sh[g][b][0] = sh[g][b][1] = sh[g][b][2] = 0.0;
            }
            cur = nxt;
        }
        // the empty asm keeps the i sums' updates ahead of the reduction (as in
        // the force tiles: otherwise their operands stay live through it)
#pragma unroll
        for (int p = 0; p < P; ++p)
#pragma unroll
            for (int b = 0; b < NV; ++b) asm volatile("" : "+v"(ia[p][b][0]), "+v"(ia[p][b][1]), "+v"(ia[p][b][2]));
        if (pjg >= 0) store(pjg, plive);
        double v12[12];
#pragma unroll
        for (int k = 0; k < 12; ++k) v12[k] = sh[k / (3 * NV)][(k / 3) % NV][k % 3];
        lds_put12(v12, red, a);
        pjg = jg;
        plive = live;
    }
    if (pjg >= 0) store(pjg, plive);
    const double sc = UNI ? qI * qJ : 1.0;
    double* Pt = Pi + (size_t)t * NV * 3 * IB;
#pragma unroll
    for (int p = 0; p < P; ++p)
#pragma unroll
        for (int b = 0; b < NV; ++b)
#pragma unroll
            for (int c = 0; c < 3; ++c)
                Pt[(size_t)(b * 3 + c) * IB + p * 64 + lane] = UNI ? sc * ia[p][b][c] : ia[p][b][c];
}

// One wave per tile (row I, segment s) of the tile table and pass
// blockIdx.y of the launch.  v: [passes][NV][3][n]; J: each pass's packed j
// records, n kHvpRec doubles apart; the partials of pass u and tile t go to
// slot u T + t (T = gridDim.x tiles).
template <int PREC, int P, int NV>
__global__ void __launch_bounds__(64, (hvp_sym_waves<P, NV>())) k_hvp_sym(int n, const double* __restrict__ x,
                                                                  const double* __restrict__ y,
                                                                  const double* __restrict__ z,
                                                                  const double* __restrict__ q,
                                                                  const double* __restrict__ v,
                                                                  const double* __restrict__ J, double eps2, int JL,
                                                                  const int2* __restrict__ tiles,
                                                                  double* __restrict__ Pi, double* __restrict__ R) {
    __shared__ __align__(16) double red[12 * kRedStride];
    constexpr int IB = 64 * P;
    const int t = blockIdx.x;
    const int2 tl = tiles[t];
    const int lane = threadIdx.x;
    const int slot = blockIdx.y * gridDim.x + t;
    v += (size_t)blockIdx.y * NV * 3 * n;
    J += (size_t)blockIdx.y * n * kHvpRec;
    double xi[P], yi[P], zi[P], qi[P], vi[NV][3][P];
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const int i = tl.x * IB + p * 64 + lane;  // rows with tiles are full blocks
        xi[p] = x[i];
        yi[p] = y[i];
        zi[p] = z[i];
        qi[p] = q[i];
#pragma unroll
        for (int b = 0; b < NV; ++b)
#pragma unroll
            for (int c = 0; c < 3; ++c) vi[b][c][p] = v[(size_t)(b * 3 + c) * n + i];
    }
    const int j0 = (tl.x + 1) * IB + tl.y * JL;
    const int j1 = min(n, j0 + JL);
    double qI, qJ;
    if (tile_charges<P>(qi, q, j0, j1, qI, qJ))
        hvp_sym_body<PREC, P, NV, true>(J, eps2, JL, j0, j1, slot, xi, yi, zi, qi, vi, qI, qJ, red, Pi, R);
    else
        hvp_sym_body<PREC, P, NV, false>(J, eps2, JL, j0, j1, slot, xi, yi, zi, qi, vi, 1.0, 1.0, red, Pi, R);
}

// Per ion k and vector b = blockIdx.y of the launch (pass b / NV, its vector
// b % NV; 64 ions per workgroup, kFinishParts waves each taking a fixed share
// of every sum): the pairs inside k's own i-block (direct, self pair
// skipped), k's i sums over the tiles of its row, minus q_k times its
// reactions from the rows above; hv[b][c][k] = k_C (those) + m_k kk_c v_k (m
// may be NULL).  T: tiles per pass.  The waves' shares are added in wave
// order (deterministic).  One vector per workgroup spreads the partial reads
// of a pass over NV times the workgroups.
template <int PREC, int NV>
__global__ void __launch_bounds__(64 * kFinishParts) k_hvp_sym_finish(
    int n, int IB, int JL, int lgJL, int T, const double* __restrict__ x, const double* __restrict__ y,
    const double* __restrict__ z, const double* __restrict__ q, const double* __restrict__ v, double eps2,
    const int* __restrict__ rowstart, const double* __restrict__ Pi, const double* __restrict__ R,
    const double* __restrict__ m, TrapK kk, double* __restrict__ hv, unsigned* flags) {
    __shared__ double red[kFinishParts][3][64];
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int b = blockIdx.y;
    const size_t pslot = (size_t)(b / NV) * T;  // the pass's first partial slot
    const int bl = b % NV;
    const int k0 = blockIdx.x * 64;
    const int k = k0 + lane;
    const int kc = min(k, n - 1);
    const int Ik = k0 / IB;
    const int b0 = Ik * IB, b1 = min(n, b0 + IB);
    const double xk = x[kc], yk = y[kc], zk = z[kc], qk = q[kc];
    const double* vb = v + (size_t)b * 3 * n;
    const double vk[3] = {vb[kc], vb[n + kc], vb[2 * (size_t)n + kc]};
    const SeriesK K;
    int lo, hi;
    double d[3] = {0.0, 0.0, 0.0}, e[3] = {0.0, 0.0, 0.0}, s[3] = {0.0, 0.0, 0.0};
    share(b0, b1, w, lo, hi);
    // four j's per iteration: their scalar loads are issued together
    // (27.3 -> 22.9 us for 8 vectors at 8192 ions, measured on MI355X)
#pragma unroll 4
    for (int j = lo; j < hi; ++j) {  // q_j T_kj over k's own block
        const double dx = xk - x[j], dy = yk - y[j], dz = zk - z[j];
        const double r2 = __builtin_fma(dx, dx, __builtin_fma(dy, dy, __builtin_fma(dz, dz, eps2)));
        double s3, g3;
        hvp_scales_w<PREC>(r2, q[j], K, s3, g3);
        if (j == kc) s3 = g3 = 0.0;  // the self pair (both scales: they are not finite at r = 0)
        const double ux = vk[0] - vb[j], uy = vk[1] - vb[n + j], uz = vk[2] - vb[2 * (size_t)n + j];
        const double w = __builtin_fma(dx, ux, __builtin_fma(dy, uy, dz * uz)) * g3;
        d[0] = __builtin_fma(s3, __builtin_fma(w, dx, -ux), d[0]);
        d[1] = __builtin_fma(s3, __builtin_fma(w, dy, -uy), d[1]);
        d[2] = __builtin_fma(s3, __builtin_fma(w, dz, -uz), d[2]);
    }
    const int off = kc - b0;
    share(rowstart[Ik], rowstart[Ik + 1], w, lo, hi);
#pragma unroll 4
    for (int t = lo; t < hi; ++t) {  // k's i sums over the tiles of its row
        const double* Pt = Pi + ((pslot + t) * NV + bl) * 3 * IB + off;
        s[0] += Pt[0];
        s[1] += Pt[IB];
        s[2] += Pt[2 * IB];
    }
    share(0, Ik, w, lo, hi);
#pragma unroll 4
    for (int I = lo; I < hi; ++I) {  // k's reactions from the rows above
        const int rel = kc - (I + 1) * IB;
        const int sI = rel >> lgJL;
        const double* Rt = R + ((pslot + rowstart[I] + sI) * NV + bl) * 3 * JL + (rel - (sI << lgJL));
        e[0] += Rt[0];
        e[1] += Rt[JL];
        e[2] += Rt[2 * JL];
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) red[w][c][lane] = s[c] + qk * (d[c] - e[c]);
    __syncthreads();
    if (w != 0 || k >= n) return;
    const double kc3[3] = {kk.kx, kk.ky, kk.kz};
    const double mk = m ? m[k] : 0.0;
    bool ok = true;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        double a = red[0][c][lane];
#pragma unroll
        for (int u = 1; u < kFinishParts; ++u) a += red[u][c][lane];
        const double h = __builtin_fma(mk * kc3[c], vk[c], kCoulomb * a);
        hv[((size_t)b * 3 + c) * n + k] = h;
        ok = ok && __builtin_isfinite(h);
    }
    if (!ok) atomicOr(flags, 1u);
}

}  // namespace cb
