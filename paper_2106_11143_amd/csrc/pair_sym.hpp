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
//   - adds q_i d y^3 over its P ions into a per-j value; after a group of
//     4 j's the 12 per-j values are summed over the wave (wave_reduce.hpp:
//     cross-lane permutes and DPP, or an LDS transpose), giving the reaction
//     on those j (up to -k_C q_j), which one lane per value stores.
// The tile writes its i sums to Pi[tile][3][IB] and its reactions to
// R[tile][3][JL]; nothing is accumulated across workgroups, so results are
// deterministic.  The diagonal i-block (pairs inside one block) is evaluated
// directly by the finish kernel, which then adds, per ion, its i sums over
// the segments of its row and its reactions from every row above, in a
// fixed order.
#pragma once
#include <hip/hip_runtime.h>

#include "internal.hpp"
#include "rsqrt.hpp"
#include "step_common.hpp"
#include "wave_reduce.hpp"

namespace cb {

// Segments of row I: ceil((n - (I+1) IB) / JL), or 0.
__host__ __device__ __forceinline__ int sym_nseg(int n, int IB, int JL, int I) {
    const int a = n - (I + 1) * IB;  // n <= 2^18: no overflow
    return a > 0 ? (a + JL - 1) / JL : 0;
}

// Tile table, by one workgroup of NT threads.  Rows are groups of W i-blocks
// (W = 1: single blocks); group I's segments cut the j's above its first
// block, W I.  rowstart[I] = first tile of group I (exclusive prefix sum over
// groups of their segment counts), rowstart[nI] = tiles T; tiles[t] = (group,
// segment) of tile t.  Each thread sums the segments of a contiguous share of
// groups, the shares are scanned in LDS (Hillis-Steele), the group starts are
// kept in LDS, and each wave then writes whole groups of the table, its lanes
// taking consecutive segments.
constexpr int kPlanMaxRows = 2048;  // n <= 2^18 ions in blocks of >= 128

template <int NT>
__device__ __forceinline__ void sym_plan_fill(int n, int IB, int JL, int W, int nI, int* __restrict__ rowstart,
                                              int2* __restrict__ tiles) {
    __shared__ int sh[NT];
    __shared__ int rs[kPlanMaxRows + 1];
    const int t = threadIdx.x;
    const int per = (nI + NT - 1) / NT;
    const int r0 = min(nI, t * per), r1 = min(nI, r0 + per);
    int mine = 0;
    for (int I = r0; I < r1; ++I) mine += sym_nseg(n, IB, JL, I * W);
    sh[t] = mine;
    __syncthreads();
    for (int w = 1; w < NT; w <<= 1) {
        const int add = t >= w ? sh[t - w] : 0;
        __syncthreads();
        sh[t] += add;
        __syncthreads();
    }
    int acc = sh[t] - mine;  // exclusive prefix of this thread's rows
    for (int I = r0; I < r1; ++I) {
        rs[I] = acc;
        rowstart[I] = acc;
        acc += sym_nseg(n, IB, JL, I * W);
    }
    if (t == NT - 1) {
        rs[nI] = sh[t];
        rowstart[nI] = sh[t];
    }
    __syncthreads();
    const int lane = t & 63;
    for (int I = t >> 6; I < nI; I += NT / 64) {
        const int s0 = rs[I], ns = rs[I + 1] - s0;
        for (int sg = lane; sg < ns; sg += 64) tiles[s0 + sg] = make_int2(I, sg);
    }
}

// s = q r^{-3} refined as in the direct kernel (the series on r^-3).
template <int PREC>
__device__ __forceinline__ double sym_s(double r2, double q, const SeriesK& K) {
    double s, y;
    inv_r<PREC, true, false>(r2, q, K, s, y);
    return s;
}

// Coordinates (and charges, when WQ) of a group of 4 j's.  The j index is
// uniform over the wave, so these are scalar loads into SGPRs (32 of them;
// two groups fit beside the rest of the kernel's scalar registers, eight j's
// do not).  Tiles of one charge on each side need no per-j charge (WQ false).
constexpr int kGroupJ = 4;

template <bool WQ>
struct JGroupT {
    double x[kGroupJ], y[kGroupJ], z[kGroupJ], q[WQ ? kGroupJ : 1];
};
using JGroup = JGroupT<true>;

// Loads j = jg + u for u < 4, with u clamped to last (last >= 0) so that a
// partial group stays in bounds.
template <bool CLAMP, bool WQ>
__device__ __forceinline__ void load_group(JGroupT<WQ>& g, int jg, int last, const double* __restrict__ x,
                                           const double* __restrict__ y, const double* __restrict__ z,
                                           const double* __restrict__ q) {
#pragma unroll
    for (int u = 0; u < kGroupJ; ++u) {
        const int j = CLAMP ? jg + min(u, last) : jg + u;
        g.x[u] = x[j];
        g.y[u] = y[j];
        g.z[u] = z[j];
        if constexpr (WQ) g.q[u] = q[j];
    }
}

// Minimum and maximum of a and b over the wave (every lane gets them).
__device__ __forceinline__ void wave_minmax(double& lo, double& hi) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        lo = fmin(lo, __shfl_xor(lo, o));
        hi = fmax(hi, __shfl_xor(hi, o));
    }
}

// Whether every ion of an i-block (the lane's P charges) and every ion of
// the j range [j0, j1) carry one charge each, and those charges (qI, qJ):
// the tile is then one of the paper's single-species N-body sub-problems
// (section 2), and its pair loop needs no per-pair charge.  Wave-uniform.
// A non-finite charge anywhere makes the answer false (the general loop then
// carries it into the forces).
template <int P>
__device__ __forceinline__ bool tile_charges(const double (&qi)[P], const double* __restrict__ q, int j0, int j1,
                                             double& qI, double& qJ) {
    double ilo = qi[0], ihi = qi[0];
    bool fin = __builtin_isfinite(qi[0]);
#pragma unroll
    for (int p = 1; p < P; ++p) {
        ilo = fmin(ilo, qi[p]);
        ihi = fmax(ihi, qi[p]);
        fin = fin && __builtin_isfinite(qi[p]);
    }
    double jlo = qi[0], jhi = qi[0];  // any finite placeholder: j1 > j0 in every tile
    if (j1 > j0) jlo = jhi = q[j0];
    for (int j = j0 + (int)__lane_id(); j < j1; j += 64) {
        const double v = q[j];
        jlo = fmin(jlo, v);
        jhi = fmax(jhi, v);
        fin = fin && __builtin_isfinite(v);
    }
    wave_minmax(ilo, ihi);
    wave_minmax(jlo, jhi);
    const bool all_fin = __builtin_amdgcn_ballot_w64(!fin) == 0;
    qI = ilo;
    qJ = jlo;
    return all_fin && ilo == ihi && jlo == jhi;
}

// The pairs of one group (only its first `live` j's when TAIL): i sums into
// ia; the reactions on the 4 j's summed over the wave and stored by one lane
// per value to Rt[c][jg - j0 + u].
// RED selects the wave reduction: 0 = cross-lane permutes and DPP, 1 = LDS
// (red, one wave's buffer).
// UNI: a tile of one charge per side.  The pair term is then d r^-3 alone
// (no charge load, no charge multiply); the i sums are scaled by qI qJ when
// stored and the reactions by rscale = qI here, so that the partials hold
// what the general loop stores.
// POT: the pair energies too, into one sum per lane, pe += q_i q_j r^-1
// (r^-1 when UNI), from r^-1 = r^2 r^-3: one or two operations per pair and
// no reaction (each unordered pair's energy is counted once, here).
template <int PREC, int P, int RED, bool TAIL, bool UNI, bool POT>
__device__ __forceinline__ void sym_group(const JGroupT<!UNI>& jd, int jg, int live, int j0, int JL, double eps2,
                                          const double (&xi)[P], const double (&yi)[P], const double (&zi)[P],
                                          const double (&qi)[P], double (&ia)[P][3], double& pe, const SeriesK& K,
                                          double rscale, double* __restrict__ Rt, double* __restrict__ red) {
    double jv[3 * kGroupJ];  // this lane's share of each reaction: sum over its P ions of q_i d r^-3
#pragma unroll
    for (int u = 0; u < kGroupJ; ++u) {
        const double xj = jd.x[u], yj = jd.y[u], zj = jd.z[u];
        double a0 = 0.0, a1 = 0.0, a2 = 0.0;
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const double dx = xi[p] - xj, dy = yi[p] - yj, dz = zi[p] - zj;
            const double r2 = __builtin_fma(dx, dx, __builtin_fma(dy, dy, __builtin_fma(dz, dz, eps2)));
            double s = sym_s<PREC>(r2, UNI ? 1.0 : qi[p], K);  // r^-3 (UNI) or q_i r^-3
            if (TAIL && u >= live) s = 0.0;
            double sq = s;
            if constexpr (!UNI) sq = s * jd.q[u];  // q_i q_j r^-3
            ia[p][0] = __builtin_fma(dx, sq, ia[p][0]);
            ia[p][1] = __builtin_fma(dy, sq, ia[p][1]);
            ia[p][2] = __builtin_fma(dz, sq, ia[p][2]);
            a0 = __builtin_fma(dx, s, a0);
            a1 = __builtin_fma(dy, s, a1);
            a2 = __builtin_fma(dz, s, a2);
            if constexpr (POT) pe = __builtin_fma(r2, sq, pe);  // r^2 (q_i q_j) r^-3
        }
        jv[3 * u + 0] = a0;
        jv[3 * u + 1] = a1;
        jv[3 * u + 2] = a2;
    }
    // The empty asm ties the i sums to this point: without it the compiler
    // defers their updates past the reduction and the conditional store,
    // keeping every pair's dx, dy, dz and s alive through them (about 100
    // more VGPRs, half the occupancy).
#pragma unroll
    for (int p = 0; p < P; ++p) asm volatile("" : "+v"(ia[p][0]), "+v"(ia[p][1]), "+v"(ia[p][2]));
    if constexpr (POT) asm volatile("" : "+v"(pe));
    const int lane = threadIdx.x & 63;
    if constexpr (RED == 0) {
        double o[3];
        reduce_scatter12(jv, o);
        const int g = lane >> 4, c = lane & 15;
        if ((!TAIL || g < live) && c < 3) {
            const double r = (c == 0) ? o[0] : ((c == 1) ? o[1] : o[2]);
            Rt[(size_t)c * JL + (jg - j0) + g] = UNI ? r * rscale : r;
        }
    } else {
        const double o = lds_reduce12(jv, red);
        const int v = lane >> 2;           // value 3 u + c of quad v (v < 12 stores)
        const int u = (v * 11) >> 5, c = v - 3 * u;  // v / 3 and v % 3 for v < 16
        if ((lane & 3) == 0 && v < 12 && (!TAIL || u < live))
            Rt[(size_t)c * JL + (jg - j0) + u] = UNI ? o * rscale : o;
    }
}

// Waves per SIMD the register budget is sized for (no spills at these; the
// IEEE square root and division need more registers).
template <int PREC, int P, bool POT = false>
constexpr int sym_waves() {
    return PREC == PREC_IEEE ? (P <= 4 ? 4 : (P <= 6 ? 3 : 2)) : (P <= 5 ? 4 : 3);
}

// The j loop of a tile over [j0, j1) and the store of its i sums (see
// sym_tile); UNI: a tile of one charge per side, qI and qJ.  With POT the
// tile's pair energy sum_{i, j} q_i q_j r^-1 goes to Et[t].
template <int PREC, int P, int RED, bool UNI, bool POT>
__device__ __forceinline__ void sym_tile_body(const double* __restrict__ x, const double* __restrict__ y,
                                              const double* __restrict__ z, const double* __restrict__ q,
                                              double eps2, int JL, int j0, int j1, int t, const double (&xi)[P],
                                              const double (&yi)[P], const double (&zi)[P], const double (&qi)[P],
                                              double qI, double qJ, double* __restrict__ red,
                                              double* __restrict__ Pi, double* __restrict__ R,
                                              double* __restrict__ Et) {
    constexpr int IB = 64 * P;
    const int lane = threadIdx.x;
    double ia[P][3], pe = 0.0;
#pragma unroll
    for (int p = 0; p < P; ++p) ia[p][0] = ia[p][1] = ia[p][2] = 0.0;
    const SeriesK K;
    const int jfull = j0 + (j1 - j0) / kGroupJ * kGroupJ;
    double* Rt = R + (size_t)t * 3 * JL;
    // Full groups, software-pipelined: the next group's j data is requested
    // before the current group is evaluated, so its load latency overlaps the
    // arithmetic (the last group re-requests itself).
    int jg = j0;
    if (jg < jfull) {
        JGroupT<!UNI> cur;
        load_group<false>(cur, jg, 0, x, y, z, q);
        for (; jg < jfull; jg += kGroupJ) {
            JGroupT<!UNI> nxt;
            const int jn = jg + kGroupJ;
            load_group<false>(nxt, jn < jfull ? jn : jg, 0, x, y, z, q);
            __builtin_amdgcn_sched_barrier(0);  // keep the requests ahead of the arithmetic
            sym_group<PREC, P, RED, false, UNI, POT>(cur, jg, kGroupJ, j0, JL, eps2, xi, yi, zi, qi, ia, pe, K, qI,
                                                     Rt, red);
            cur = nxt;
        }
    }
    if (jg < j1) {  // the last, partial group: j's from j1 on are masked
        JGroupT<!UNI> tail;
        load_group<true>(tail, jg, j1 - jg - 1, x, y, z, q);
        sym_group<PREC, P, RED, true, UNI, POT>(tail, jg, j1 - jg, j0, JL, eps2, xi, yi, zi, qi, ia, pe, K, qI, Rt,
                                                red);
    }
    const double sc = UNI ? qI * qJ : 1.0;
    double* Pt = Pi + (size_t)t * 3 * IB;
#pragma unroll
    for (int p = 0; p < P; ++p)
#pragma unroll
        for (int c = 0; c < 3; ++c) Pt[(size_t)c * IB + p * 64 + lane] = UNI ? sc * ia[p][c] : ia[p][c];
    if constexpr (POT) {
        // the tile's energy: a fixed butterfly over the wave (every run adds
        // in the same order), stored by lane 0
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) pe += __shfl_xor(pe, o);
        if (lane == 0) Et[t] = UNI ? sc * pe : pe;
    }
}

// Tile (row I, segment sg) of a run of n ions at x, y, z, q: i sums to
// Pi[t][3][IB], reactions to R[t][3][JL] (and with POT its pair energy to
// Et[t]).  red: the LDS reduction buffer.  A tile whose i-block and
// j-segment each hold ions of one charge (ions grouped by species) takes the
// charge-free pair loop.
template <int PREC, int P, int RED, bool POT = false>
__device__ __forceinline__ void sym_tile(int n, const double* __restrict__ x, const double* __restrict__ y,
                                         const double* __restrict__ z, const double* __restrict__ q, double eps2,
                                         int JL, int I, int sg, int t, double* __restrict__ red,
                                         double* __restrict__ Pi, double* __restrict__ R,
                                         double* __restrict__ Et = nullptr) {
    constexpr int IB = 64 * P;
    const int lane = threadIdx.x;
    double xi[P], yi[P], zi[P], qi[P];
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const int i = I * IB + p * 64 + lane;  // rows with tiles are full blocks
        xi[p] = x[i];
        yi[p] = y[i];
        zi[p] = z[i];
        qi[p] = q[i];
    }
    const int j0 = (I + 1) * IB + sg * JL;
    const int j1 = min(n, j0 + JL);
    double qI, qJ;
    if (tile_charges<P>(qi, q, j0, j1, qI, qJ))
        sym_tile_body<PREC, P, RED, true, POT>(x, y, z, q, eps2, JL, j0, j1, t, xi, yi, zi, qi, qI, qJ, red, Pi, R,
                                               Et);
    else
        sym_tile_body<PREC, P, RED, false, POT>(x, y, z, q, eps2, JL, j0, j1, t, xi, yi, zi, qi, 1.0, 1.0, red, Pi,
                                                R, Et);
}

template <int PREC, int P, int RED, bool POT>
__global__ void __launch_bounds__(64, (sym_waves<PREC, P, POT>())) k_pair_sym(int n, const double* __restrict__ x,
                                                                 const double* __restrict__ y,
                                                                 const double* __restrict__ z,
                                                                 const double* __restrict__ q, double eps2, int JL,
                                                                 const int2* __restrict__ tiles,
                                                                 double* __restrict__ Pi, double* __restrict__ R,
                                                                 double* __restrict__ Et) {
    __shared__ __align__(16) double red_buf[RED == 1 ? 12 * kRedStride : 2];
    const int t = blockIdx.x;
    const int2 tl = tiles[t];
    sym_tile<PREC, P, RED, POT>(n, x, y, z, q, eps2, JL, tl.x, tl.y, t, red_buf, Pi, R, Et);
}

// ---------------------------------------------------------------- row groups
// Algorithm 4: a workgroup of kSymRows waves takes the i-blocks I = kSymRows G
// + w (w = its waves) of row group G against one j-segment [c0, c0 + JL),
// c0 = (kSymRows G + 1) IB + s JL: each wave evaluates the part of the
// segment above its own diagonal block (j >= (I + 1) IB; segments and blocks
// are multiples of 64 apart, so a wave's part starts on a 64-j boundary).
// The waves' per-j reactions go to one LDS slab per wave, 64 j's at a time;
// after each 64 j's the workgroup adds the slabs in wave order and stores one
// reaction partial R[t][3][JL] for the tile, so the reaction partials are a
// kSymRows-th of one-wave tiles' and the waves share the segment's j data.
// The i sums go to Pi[t][w][3][IB] (zeros from a wave with no pairs), the
// pair energies (POT) to Et[t kSymRows + w].
constexpr int kRowChunk = 64;               // j's per LDS slab
constexpr int kRowStride = kRowChunk + 1;  // doubles per component row of a slab (odd: the rows' stores hit distinct banks)

// The pairs of j in [cs, ce) (whole groups, the last one partial) of one
// wave: reactions into its slab slabw[3][kRowStride] (index j - cs).  cur:
// the chunk's first group, already requested (when the chunk holds a whole
// one); on return it holds the group at jnext (the next chunk's first, when
// jnext >= 0), requested during this chunk's last whole group, so that only
// two groups of j data are held in the loop.
template <int PREC, int P, bool UNI, bool POT>
__device__ __forceinline__ void sym_rows_chunk(const double* __restrict__ x, const double* __restrict__ y,
                                               const double* __restrict__ z, const double* __restrict__ q,
                                               double eps2, int cs, int ce, int jnext, JGroupT<!UNI>& cur,
                                               const double (&xi)[P], const double (&yi)[P], const double (&zi)[P],
                                               const double (&qi)[P], double (&ia)[P][3], double& pe, double qI,
                                               double* __restrict__ slabw, double* __restrict__ red) {
    const SeriesK K;
    const int jfull = cs + (ce - cs) / kGroupJ * kGroupJ;
    int jg = cs;
    for (; jg < jfull; jg += kGroupJ) {
        JGroupT<!UNI> nxt;
        const int jn = jg + kGroupJ;
        load_group<false>(nxt, jn < jfull ? jn : (jnext >= 0 ? jnext : jg), 0, x, y, z, q);
        __builtin_amdgcn_sched_barrier(0);  // keep the requests ahead of the arithmetic
        sym_group<PREC, P, 1, false, UNI, POT>(cur, jg, kGroupJ, cs, kRowStride, eps2, xi, yi, zi, qi, ia, pe, K, qI,
                                               slabw, red);
        cur = nxt;
    }
    if (jg < ce) {  // the last, partial group: j's from ce on are masked
        JGroupT<!UNI> tail;
        load_group<true>(tail, jg, ce - jg - 1, x, y, z, q);
        sym_group<PREC, P, 1, true, UNI, POT>(tail, jg, ce - jg, cs, kRowStride, eps2, xi, yi, zi, qi, ia, pe, K, qI,
                                              slabw, red);
    }
}

// The j loop of a row-group tile (the workgroup's 64-j chunks of [c0, c1),
// each wave's pairs from j0 on) and the stores of its partials.  UNI is
// uniform over the workgroup, so every wave meets every barrier.
template <int PREC, int P, bool UNI, bool POT>
__device__ __forceinline__ void sym_rows_tile(const double* __restrict__ x, const double* __restrict__ y,
                                              const double* __restrict__ z, const double* __restrict__ q,
                                              double eps2, int JL, int t, int w, int c0, int c1, int j0, bool live,
                                              const double (&xi)[P], const double (&yi)[P], const double (&zi)[P],
                                              const double (&qi)[P], double qI, double qJ,
                                              double (*__restrict__ slab)[3 * kRowStride],
                                              double* __restrict__ red, double* __restrict__ Pi,
                                              double* __restrict__ R, double* __restrict__ Et) {
    constexpr int IB = 64 * P;
    const int lane = threadIdx.x & 63;
    double ia[P][3], pe = 0.0;
#pragma unroll
    for (int p = 0; p < P; ++p) ia[p][0] = ia[p][1] = ia[p][2] = 0.0;
    double* slabw = slab[w];
    double* Rt = R + (size_t)t * 3 * JL;
    // the first group of each of the wave's chunks is requested during the
    // chunk before (the first chunk's here), so that its load overlaps the
    // workgroup's slab sums
    JGroupT<!UNI> cur;
    if (live && j0 + kGroupJ <= min(c1, j0 + kRowChunk)) load_group<false>(cur, j0, 0, x, y, z, q);
    for (int cs = c0; cs < c1; cs += kRowChunk) {
        const int ce = min(c1, cs + kRowChunk);
        const int cn = cs + kRowChunk;  // the next chunk, when it holds a whole group
        const int jnext = cn + kGroupJ <= min(c1, cn + kRowChunk) ? cn : -1;
        if (live && cs >= j0)
            sym_rows_chunk<PREC, P, UNI, POT>(x, y, z, q, eps2, cs, ce, jnext, cur, xi, yi, zi, qi, ia, pe,
                                              UNI ? qI : 1.0, slabw, red);
        else
            for (int u = lane; u < 3 * kRowStride; u += 64) slabw[u] = 0.0;
        __syncthreads();
        for (int u = threadIdx.x; u < 3 * kRowChunk; u += 64 * kSymRows) {
            const int c = u / kRowChunk, jj = u - c * kRowChunk, k = c * kRowStride + jj;
            if (cs + jj < ce) {
                double a = slab[0][k];
#pragma unroll
                for (int v = 1; v < kSymRows; ++v) a += slab[v][k];
                Rt[(size_t)c * JL + (cs - c0) + jj] = a;
            }
        }
        __syncthreads();  // the slabs are rewritten by the next 64 j's
    }
    const double sc = UNI ? qI * qJ : 1.0;
    double* Pt = Pi + ((size_t)t * kSymRows + w) * 3 * IB;
#pragma unroll
    for (int p = 0; p < P; ++p)
#pragma unroll
        for (int c = 0; c < 3; ++c) Pt[(size_t)c * IB + p * 64 + lane] = UNI ? sc * ia[p][c] : ia[p][c];
    if constexpr (POT) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) pe += __shfl_xor(pe, o);
        if (lane == 0) Et[(size_t)t * kSymRows + w] = UNI ? sc * pe : pe;
    }
}

template <int PREC, int P, bool POT>
__global__ void __launch_bounds__(64 * kSymRows, (sym_waves<PREC, P, POT>()))
    k_pair_sym_rows(int n, const double* __restrict__ x, const double* __restrict__ y,
                    const double* __restrict__ z, const double* __restrict__ q, double eps2, int JL,
                    const int2* __restrict__ tiles, double* __restrict__ Pi, double* __restrict__ R,
                    double* __restrict__ Et) {
    __shared__ __align__(16) double red_buf[kSymRows][12 * kRedStride];
    __shared__ double slab[kSymRows][3 * kRowStride];
    __shared__ int nonuni;
    constexpr int IB = 64 * P;
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int t = blockIdx.x;
    const int2 tl = tiles[t];
    const int I = tl.x * kSymRows + w;
    const int c0 = (tl.x * kSymRows + 1) * IB + tl.y * JL;
    const int c1 = min(n, c0 + JL);
    const int jr = (I + 1) * IB;  // the first j above this wave's diagonal block
    const int j0 = max(c0, jr);
    const bool live = j0 < c1;    // then block I is a full block
    double xi[P], yi[P], zi[P], qi[P];
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const int i = min(I * IB + p * 64 + lane, n - 1);
        xi[p] = x[i];
        yi[p] = y[i];
        zi[p] = z[i];
        qi[p] = q[i];
    }
    // the charge-free loop when every wave with pairs has one charge on each
    // side (each wave keeps its own qI, qJ)
    double qI = 1.0, qJ = 1.0;
    const bool uni = !live || tile_charges<P>(qi, q, j0, c1, qI, qJ);
    if (threadIdx.x == 0) nonuni = 0;
    __syncthreads();
    if (!uni && lane == 0) nonuni = 1;
    __syncthreads();
    if (nonuni == 0)
        sym_rows_tile<PREC, P, true, POT>(x, y, z, q, eps2, JL, t, w, c0, c1, j0, live, xi, yi, zi, qi, qI, qJ, slab,
                                          red_buf[w], Pi, R, Et);
    else
        sym_rows_tile<PREC, P, false, POT>(x, y, z, q, eps2, JL, t, w, c0, c1, j0, live, xi, yi, zi, qi, qI, qJ,
                                           slab, red_buf[w], Pi, R, Et);
}

// Per ion k: direct pairs inside its own i-block, plus its i sums over the
// segments of its row, minus q_k times its reactions from the rows above;
// writes the finished force F = k_C (...) to F[3][n].  Rows come in groups of
// W i-blocks (W = 1, or kSymRows for the row-group tiles): ion k's block Ik
// is wave Ik % W of group Ik / W, its i sums sit in that wave's slot of each
// tile of the group, and every group whose segments start at or below k
// holds one reaction slot for k.  One workgroup = 64 consecutive ions (one
// i-block holds them all, IB being a multiple of 64) and kFinishParts
// waves; wave w takes the w-th contiguous share of each of the three sums,
// and the shares are added in wave order through LDS, so the result does not
// depend on timing.  All j and row loops are uniform.
constexpr int kFinishParts = 4;

__host__ __device__ __forceinline__ void share(int a, int b, int w, int& lo, int& hi) {
    const int len = (b - a + kFinishParts - 1) / kFinishParts;
    lo = min(b, a + w * len);
    hi = min(b, lo + len);
}

// With POT, phi[k] receives ion k's share of the Coulomb energy, U_C =
// k_C sum_k phi[k]: q_k times its pairs with the later ions of its own block
// (q_j r^-1, j > k), plus the energies of the tiles of its row numbered
// off, off + IB, ... within the row (each tile's energy goes to one ion).
template <int PREC, bool POT>
__global__ void __launch_bounds__(64 * kFinishParts) k_sym_finish(int n, int IB, int JL, int lgJL, int W,
                                                                  const double* __restrict__ x,
                                                                  const double* __restrict__ y,
                                                                  const double* __restrict__ z,
                                                                  const double* __restrict__ q, double eps2,
                                                                  const int* __restrict__ rowstart,
                                                                  const double* __restrict__ Pi,
                                                                  const double* __restrict__ R,
                                                                  const double* __restrict__ Et,
                                                                  double* __restrict__ F, double* __restrict__ phi) {
    constexpr int NS = POT ? 10 : 9;  // per lane: direct 3, i sums 3, reactions 3 (+ the energy share)
    __shared__ double red[kFinishParts][NS][64];
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int k0 = blockIdx.x * 64;
    const int k = k0 + lane;
    const int kc = min(k, n - 1);
    const int Ik = k0 / IB;
    const int Gk = Ik / W, wk = Ik - Gk * W;
    const int b0 = Ik * IB, b1 = min(n, b0 + IB);
    const double xk = x[kc], yk = y[kc], zk = z[kc];
    const SeriesK K;
    int lo, hi;
    double d0 = 0.0, d1 = 0.0, d2 = 0.0, ps = 0.0;
    share(b0, b1, w, lo, hi);
    // four j's per iteration: their scalar loads are issued together (the
    // finish at N = 1e5 with row groups: 95 -> 71 us, measured on MI355X)
#pragma unroll 4
    for (int j = lo; j < hi; ++j) {
        const double dx = xk - x[j], dy = yk - y[j], dz = zk - z[j];
        const double r2 = __builtin_fma(dx, dx, __builtin_fma(dy, dy, __builtin_fma(dz, dz, eps2)));
        double s = sym_s<PREC>(r2, q[j], K);  // q_j r^-3
        if (POT) ps = j > kc ? __builtin_fma(r2, s, ps) : ps;  // q_j r^-1 of the later ions
        if (j == kc) s = 0.0;
        d0 = __builtin_fma(dx, s, d0);
        d1 = __builtin_fma(dy, s, d1);
        d2 = __builtin_fma(dz, s, d2);
    }
    const int off = kc - b0;
    double p0 = 0.0, p1 = 0.0, p2 = 0.0;
    share(rowstart[Gk], rowstart[Gk + 1], w, lo, hi);
#pragma unroll 4
    for (int t = lo; t < hi; ++t) {
        const double* Pt = Pi + ((size_t)t * W + wk) * 3 * IB + off;
        p0 += Pt[0];
        p1 += Pt[IB];
        p2 += Pt[2 * IB];
    }
    double e0 = 0.0, e1 = 0.0, e2 = 0.0;
    // the groups whose segments start at or below k: all above k's group, and
    // k's own group when k is not in its first block
    share(0, Gk + (wk > 0 ? 1 : 0), w, lo, hi);
#pragma unroll 4
    for (int G = lo; G < hi; ++G) {
        const int rel = kc - (G * W + 1) * IB;
        const int sI = rel >> lgJL;
        const double* Rt = R + (size_t)(rowstart[G] + sI) * 3 * JL + (rel - (sI << lgJL));
        e0 += Rt[0];
        e1 += Rt[JL];
        e2 += Rt[2 * JL];
    }
    double es = 0.0;
    if (POT) {
        const double qk = q[kc];
        es = qk * ps;
        if (w == 0)
            for (int t = rowstart[Gk] + off; t < rowstart[Gk + 1]; t += IB) es += Et[(size_t)t * W + wk];
    }
    const double v[10] = {d0, d1, d2, p0, p1, p2, e0, e1, e2, es};
#pragma unroll
    for (int c = 0; c < NS; ++c) red[w][c][lane] = v[c];
    __syncthreads();
    if (w != 0 || k >= n) return;
    double tot[NS];
#pragma unroll
    for (int c = 0; c < NS; ++c) {
        double a = red[0][c][lane];
#pragma unroll
        for (int u = 1; u < kFinishParts; ++u) a += red[u][c][lane];
        tot[c] = a;
    }
    const double qk = q[k];
    F[k] = kCoulomb * (tot[3] + qk * (tot[0] - tot[6]));
    F[(size_t)n + k] = kCoulomb * (tot[4] + qk * (tot[1] - tot[7]));
    F[2 * (size_t)n + k] = kCoulomb * (tot[5] + qk * (tot[2] - tot[8]));
    if (POT) phi[k] = tot[NS - 1];
}

}  // namespace cb
