// Stepped ensemble path of md_run with many runs (the Kibble-Zurek statistics
// use case of the paper's introduction).  Instead of one workgroup per run
// (batched.hip), every velocity-Verlet step is two launches over all runs at
// once, so that no run's size bounds the makespan:
//   1. k_pair_sym_ens: the Newton's-third-law tiles (pair_sym.hpp) of every
//      run, one wave per tile, longest tiles first.  A tile entry holds its
//      run's first ion and size, the slot of its partials, and its row and
//      segment.
//      Each row's first tiles are its diagonal block (the ordered pairs
//      inside the i-block, evaluated directly) cut into j-ranges of 128.
//   2. k_ens_step: per 64 ions of one run, the finish of the force (the i
//      sums of its row and the reactions from the rows above, each summed in
//      a fixed order) fused with the trap, the kick and the next drift.  The drift writes the other of two
//      position buffers: other workgroups of the launch still read the
//      current positions of the same i-block.
// When no run is longer than an i-block there are no tiles, and the second
// launch alone evaluates every pair of each run directly (16 waves per 64
// ions).  md_run_small steps one small run in one launch per step with no
// tables at all (k_small_step: one wave per 64 ions and part of the run, the
// parts added by the last to arrive).
// Energy records add each ion's Coulomb potential (a direct pass over its
// run) on the recording step; the last 64-ion chunk of a run to finish sums
// the run's chunk partials in chunk order.  Results do not depend on timing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "internal.hpp"
#include "pair_sym.hpp"
#include "split_sum.hpp"
#include "step_common.hpp"

namespace cb {

// Diagonal sub-tile d of row I: the ordered pairs (i, j) inside i-block I
// (ions b0 .. b1-1; a run's last block may be short) with j in the d-th
// range of DL, evaluated directly, the self pair skipped, into the i sums
// Pi[t] (q_i q_j d r^-3, as the row's other tiles).  In a small launch a
// block's diagonal is split (DL < IB) so that it takes several waves, not
// one long one; in a large one it stays whole (DL = IB).
// The j data of the next group of 4 are requested before the current group
// is evaluated; at most 4 rows per lane are held at a time, so the tile fits
// the register budget of the symmetric tiles it shares a kernel with.  Lanes beyond the block compute on a clamped ion and their
// sums are never read.
constexpr int kDiagLen = 128;        // j's per diagonal sub-tile when a block's diagonal is split
constexpr int kDiagSplitMax = 4096;  // split only below this many off-diagonal tiles
constexpr int kDiagSeg = 0xffff;     // segment field of diagonal sub-tile d: kDiagSeg - d
constexpr int kDiagMax = 8;          // sub-tiles per block at most (IB <= 1024)

template <int PREC, int P>
__device__ __forceinline__ void diag_tile(int n, const double* __restrict__ x, const double* __restrict__ y,
                                          const double* __restrict__ z, const double* __restrict__ q, double eps2,
                                          int I, int d, int DL, int t, double* __restrict__ Pi) {
    constexpr int IB = 64 * P;
    constexpr int H = P < 4 ? P : 4;  // i rows held per pass: the block in P / H passes over its j's
    const int lane = threadIdx.x;
    const int b0 = I * IB, b1 = min(n, b0 + IB);
    const int j0 = b0 + d * DL, j1 = min(b1, j0 + DL);  // this sub-tile's j's
    double* Pt = Pi + (size_t)t * 3 * IB;
    const SeriesK K;
    const int full = j0 + (j1 - j0) / kGroupJ * kGroupJ;
#pragma unroll 1
    for (int h = 0; h < P / H; ++h) {
        double xi[H], yi[H], zi[H], qi[H], ia[H][3];
        int ii[H];
#pragma unroll
        for (int p = 0; p < H; ++p) {
            ii[p] = b0 + (h * H + p) * 64 + lane;
            const int ic = min(ii[p], b1 - 1);
            xi[p] = x[ic];
            yi[p] = y[ic];
            zi[p] = z[ic];
            qi[p] = q[ic];
            ia[p][0] = ia[p][1] = ia[p][2] = 0.0;
        }
        auto group = [&](const JGroup& g, int jg, int live) {
#pragma unroll
            for (int u = 0; u < kGroupJ; ++u) {
#pragma unroll
                for (int p = 0; p < H; ++p) {
                    const double dx = xi[p] - g.x[u], dy = yi[p] - g.y[u], dz = zi[p] - g.z[u];
                    const double r2 = __builtin_fma(dx, dx, __builtin_fma(dy, dy, __builtin_fma(dz, dz, eps2)));
                    double s = sym_s<PREC>(r2, qi[p], K);  // q_i r^-3
                    if (u >= live || ii[p] == jg + u) s = 0.0;
                    const double sq = s * g.q[u];
                    ia[p][0] = __builtin_fma(dx, sq, ia[p][0]);
                    ia[p][1] = __builtin_fma(dy, sq, ia[p][1]);
                    ia[p][2] = __builtin_fma(dz, sq, ia[p][2]);
                }
                // an empty asm ties each j's updates here, so that only H pairs are in flight
#pragma unroll
                for (int p = 0; p < H; ++p) asm volatile("" : "+v"(ia[p][0]), "+v"(ia[p][1]), "+v"(ia[p][2]));
            }
        };
        int jg = j0;
        if (jg < full) {
            JGroup cur;
            load_group<false>(cur, jg, 0, x, y, z, q);
            for (; jg < full; jg += kGroupJ) {
                JGroup nxt;
                const int jn = jg + kGroupJ;
                load_group<false>(nxt, jn < full ? jn : jg, 0, x, y, z, q);
                __builtin_amdgcn_sched_barrier(0);  // keep the requests ahead of the arithmetic
                group(cur, jg, kGroupJ);
                cur = nxt;
            }
        }
        if (jg < j1) {
            JGroup tail;
            load_group<true>(tail, jg, j1 - jg - 1, x, y, z, q);
            group(tail, jg, j1 - jg);
        }
#pragma unroll
        for (int p = 0; p < H; ++p)
#pragma unroll
            for (int c = 0; c < 3; ++c) Pt[(size_t)c * IB + (h * H + p) * 64 + lane] = ia[p][c];
    }
}

template <int PREC, int P>
__global__ void __launch_bounds__(64, (sym_waves<PREC, P>())) k_pair_sym_ens(const double* __restrict__ x,
                                                                     const double* __restrict__ y,
                                                                     const double* __restrict__ z,
                                                                     const double* __restrict__ q, double eps2,
                                                                     int JL, int DL, const int4* __restrict__ tiles,
                                                                     double* __restrict__ Pi,
                                                                     double* __restrict__ R) {
    __shared__ __align__(16) double red_buf[12 * kRedStride];
    const int4 tl = tiles[blockIdx.x];  // first ion, ions, slot, row << 16 | segment
    const int o = tl.x;
    const int sg = tl.w & 0xffff;
    if (sg > kDiagSeg - kDiagMax)
        diag_tile<PREC, P>(tl.y, x + o, y + o, z + o, q + o, eps2, tl.w >> 16, kDiagSeg - sg, DL, tl.z, Pi);
    else
        sym_tile<PREC, P, 1>(tl.y, x + o, y + o, z + o, q + o, eps2, JL, tl.w >> 16, sg, tl.z, red_buf,
                             Pi, R);
}

struct EnsParams {
    const int2* chunks;    // [nchunk] (run, first ion of the chunk within the run)
    const int4* runs;      // [nrun] (first ion, ions, first row-start entry, first chunk)
    const int* rowstart;   // per run, rows 0..nI: partial slot of (row, segment 0); concatenated
    const cb_trap* traps;  // [nrun]
    const double* Pi;      // [slots][3][IB]
    const double* R;       // [slots][3][JL]
    const double *x, *y, *z;  // positions at this step (read)
    double *xn, *yn, *zn;     // positions after the drift (written)
    const double* q;
    const double* m;
    double *vx, *vy, *vz, *ax, *ay, *az;
    int IB, JL, lgJL;
    int ndiag;  // diagonal sub-tiles (slots) at the head of every full row, 0 without tiles
    double eps2, t0, dt;
    long long step;     // the trap is taken at step_time(t0, dt, step)
    unsigned mode;      // EPI_ACCEL, EPI_KICK, EPI_DRIFT, EPI_ENERGY
    double* echunk;     // [nchunk][3]: K, U_C, U_trap of each chunk (EPI_ENERGY)
    // EPI_ENERGY: the last chunk of a run to finish (counted in ecount[run],
    // zero at launch and left zero) sums the run's chunk partials in chunk
    // order into energies[run][rec][0..3] = K, U_C, U_trap, E.
    unsigned* ecount;   // [nrun]
    double* energies;   // [nrun][nrec][4]
    int nrun, nchunk;
    long long nrec, rec;
    unsigned* flags;
    // k_small_step: the run's size and trap, its j-parts per 64 ions, the
    // parts' sums [nchunk * S][4][64] and the arrival counts [nchunk].
    int n1;
    cb_trap trap1;
    int S;
    double* spart;
    unsigned* scount;
};

// Share w of PARTS of [a, b).
template <int PARTS>
__device__ __forceinline__ void part_of(int a, int b, int w, int& lo, int& hi) {
    const int len = (b - a + PARTS - 1) / PARTS;
    lo = min(b, a + w * len);
    hi = min(b, lo + len);
}

// Direct pairs of ion kc with the j's of [lo, hi): into f the force sums
// q_j d r^-3 (FORCE), into u the potential sum q_j / r (POT); the self pair
// is skipped.  j is uniform over the wave, so the j data are scalar loads,
// and those of the next group of 4 are issued before the current group is
// evaluated (as in the pair kernels).
template <int PREC, bool FORCE, bool POT>
__device__ __forceinline__ void direct_range(int lo, int hi, int kc, double xk, double yk, double zk,
                                             const double* __restrict__ X, const double* __restrict__ Y,
                                             const double* __restrict__ Z, const double* __restrict__ Q,
                                             double eps2, const SeriesK& K, double (&f)[3], double& u) {
    auto pair = [&](double xj, double yj, double zj, double qj, int j) {
        const double dx = xk - xj, dy = yk - yj, dz = zk - zj;
        const double r2 = __builtin_fma(dx, dx, __builtin_fma(dy, dy, __builtin_fma(dz, dz, eps2)));
        double s = 0.0, y = 0.0;
        inv_r<PREC, FORCE, POT>(r2, qj, K, s, y);
        if (j == kc) {
            s = 0.0;
            y = 0.0;
        }
        if (FORCE) {
            f[0] = __builtin_fma(dx, s, f[0]);
            f[1] = __builtin_fma(dy, s, f[1]);
            f[2] = __builtin_fma(dz, s, f[2]);
        }
        if (POT) u = __builtin_fma(qj, y, u);
    };
    const int full = lo + (hi - lo) / kGroupJ * kGroupJ;
    int jg = lo;
    if (jg < full) {
        JGroup cur;
        load_group<false>(cur, jg, 0, X, Y, Z, Q);
        for (; jg < full; jg += kGroupJ) {
            JGroup nxt;
            const int jn = jg + kGroupJ;
            load_group<false>(nxt, jn < full ? jn : jg, 0, X, Y, Z, Q);
            __builtin_amdgcn_sched_barrier(0);  // keep the requests ahead of the arithmetic
#pragma unroll
            for (int t = 0; t < kGroupJ; ++t) pair(cur.x[t], cur.y[t], cur.z[t], cur.q[t], jg + t);
            cur = nxt;
        }
    }
    for (; jg < hi; ++jg) pair(X[jg], Y[jg], Z[jg], Q[jg], jg);
}

// Trap, kick and drift (as P.mode says) of ion i (packed index) at (x, y, z)
// with charge qk, Coulomb force (Fx, Fy, Fz) and pot = sum_j q_j / r; its
// energy terms (EPI_ENERGY) go to eK, eC, eT.  Non-finite results set the
// flag.
__device__ __forceinline__ void step_ion(const EnsParams& P, const cb_trap& tr, int i, double x, double y,
                                         double z, double qk, double Fx, double Fy, double Fz, double pot,
                                         double& eK, double& eC, double& eT) {
    const unsigned mode = P.mode;
    const TrapK kk = trap_k(tr, step_time(P.t0, P.dt, P.step));
    double vx = P.vx[i], vy = P.vy[i], vz = P.vz[i];
    double ax = P.ax[i], ay = P.ay[i], az = P.az[i];
    const double mi = P.m[i];
    bool ok = true;
    if (mode & (EPI_ACCEL | EPI_KICK)) {
        const double anx = Fx / mi - kk.kx * x;
        const double any = Fy / mi - kk.ky * y;
        const double anz = Fz / mi - kk.kz * z;
        if (mode & EPI_KICK) {
            const double h = 0.5 * P.dt;
            if (tr.gamma == 0.0) {
                vx = vx + h * (ax + anx);
                vy = vy + h * (ay + any);
                vz = vz + h * (az + anz);
            } else {  // friction -g v by the trapezoidal rule, g = Gamma / m_i
                const double g = tr.gamma / mi, lo = 1.0 - g * h, hi = 1.0 + g * h;
                vx = (vx * lo + h * (ax + anx)) / hi;
                vy = (vy * lo + h * (ay + any)) / hi;
                vz = (vz * lo + h * (az + anz)) / hi;
            }
            P.vx[i] = vx;
            P.vy[i] = vy;
            P.vz[i] = vz;
        }
        ax = anx;
        ay = any;
        az = anz;
        P.ax[i] = ax;
        P.ay[i] = ay;
        P.az[i] = az;
        ok = finite3(ax, ay, az) && finite3(vx, vy, vz);
    }
    if (mode & EPI_ENERGY) {
        eK = 0.5 * mi * (vx * vx + vy * vy + vz * vz);
        eC = 0.5 * kCoulomb * qk * pot;
        eT = 0.5 * mi * (kk.kx * x * x + kk.ky * y * y + kk.kz * z * z);
        ok = ok && finite3(eK, eC, eT);
    }
    if (mode & EPI_DRIFT) {
        const double dt = P.dt, h2 = 0.5 * dt * dt;
        if (tr.gamma == 0.0) {
            x = x + vx * dt + h2 * ax;
            y = y + vy * dt + h2 * ay;
            z = z + vz * dt + h2 * az;
        } else {  // the drift sees the friction acceleration -g v too
            const double g = tr.gamma / mi;
            x = x + vx * dt + h2 * (ax - g * vx);
            y = y + vy * dt + h2 * (ay - g * vy);
            z = z + vz * dt + h2 * (az - g * vz);
        }
        P.xn[i] = x;
        P.yn[i] = y;
        P.zn[i] = z;
        ok = ok && finite3(x, y, z);
    }
    if (!ok) atomicOr(P.flags, 1u);
}

// Energy record of run r, by one whole wave for chunk cid of the run's
// chunks c0 .. c1-1, with each lane's energy terms: the chunk's sums go to
// P.echunk[cid]; the last chunk of the run to arrive (counted in
// P.ecount[r]) adds the run's chunk sums in chunk order into its record.
__device__ __forceinline__ void energy_arrival(const EnsParams& P, int r, int cid, int c0, int c1, double eK,
                                               double eC, double eT) {
    const int lane = threadIdx.x & 63;
    // fixed butterfly over the wave: every lane ends with the same sums
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) {
        eK += __shfl_xor(eK, d);
        eC += __shfl_xor(eC, d);
        eT += __shfl_xor(eT, d);
    }
    int last = 0;
    if (lane == 0) {
        P.echunk[(size_t)cid * 3 + 0] = eK;
        P.echunk[(size_t)cid * 3 + 1] = eC;
        P.echunk[(size_t)cid * 3 + 2] = eT;
        __threadfence();  // this chunk's sums before its arrival
        last = atomicAdd(&P.ecount[r], 1u) == (unsigned)(c1 - c0 - 1);
    }
    last = __shfl(last, 0);
    if (!last) return;
    __threadfence();  // every chunk's sums of this run are visible
    double a = 0.0, b = 0.0, c = 0.0;
    for (int u = c0 + lane; u < c1; u += 64) {
        a += P.echunk[(size_t)u * 3 + 0];
        b += P.echunk[(size_t)u * 3 + 1];
        c += P.echunk[(size_t)u * 3 + 2];
    }
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) {
        a += __shfl_xor(a, d);
        b += __shfl_xor(b, d);
        c += __shfl_xor(c, d);
    }
    if (lane == 0) {
        double* e = P.energies + ((size_t)r * P.nrec + P.rec) * 4;
        e[0] = a;
        e[1] = b;
        e[2] = c;
        e[3] = a + b + c;
        P.ecount[r] = 0u;
    }
}

// PARTS waves per 64 ions.  With WHOLE every run is a single i-block (no
// tiles): only the direct sums and the potential are reduced, which lets
// 16 waves share a chunk's pairs within the static LDS limit.
template <int PREC, int PARTS, bool WHOLE>
__global__ void __launch_bounds__(64 * PARTS) k_ens_step(EnsParams P) {
    constexpr int kVals = WHOLE ? 4 : 10;  // direct (3), [row i sums (3), reactions (3)], potential
    constexpr int kPot = kVals - 1;
    __shared__ double red[PARTS][kVals][64];
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int2 ch = P.chunks[blockIdx.x];
    const int4 ru = P.runs[ch.x];
    const int o = ru.x, n = ru.y;
    const double *X = P.x + o, *Y = P.y + o, *Z = P.z + o, *Q = P.q + o;
    const int* rowstart = WHOLE ? nullptr : P.rowstart + ru.z;
    const int k0 = ch.y, k = k0 + lane, kc = min(k, n - 1);
    const unsigned mode = P.mode;
    const double xk = X[kc], yk = Y[kc], zk = Z[kc];
    const SeriesK K;
    double v[kVals];
#pragma unroll
    for (int c = 0; c < kVals; ++c) v[c] = 0.0;
    const bool need_f = (mode & (EPI_ACCEL | EPI_KICK)) != 0, need_p = (mode & EPI_ENERGY) != 0;
    double f[3] = {0.0, 0.0, 0.0}, u = 0.0;
    if (WHOLE) {  // the run is one block: force and potential in one pass over it
        int lo, hi;
        part_of<PARTS>(0, n, w, lo, hi);
        if (need_f && need_p) direct_range<PREC, true, true>(lo, hi, kc, xk, yk, zk, X, Y, Z, Q, P.eps2, K, f, u);
        else if (need_f) direct_range<PREC, true, false>(lo, hi, kc, xk, yk, zk, X, Y, Z, Q, P.eps2, K, f, u);
        else if (need_p) direct_range<PREC, false, true>(lo, hi, kc, xk, yk, zk, X, Y, Z, Q, P.eps2, K, f, u);
    } else {
        // (the pairs inside the ion's own i-block come from the row's diagonal sub-tiles)
        if (need_p) {  // potential over the whole run
            int lo, hi;
            part_of<PARTS>(0, n, w, lo, hi);
            direct_range<PREC, false, true>(lo, hi, kc, xk, yk, zk, X, Y, Z, Q, P.eps2, K, f, u);
        }
    }
    v[0] = f[0];
    v[1] = f[1];
    v[2] = f[2];
    v[kPot] = u;
    if (!WHOLE && need_f) {  // i sums of the ion's row (diagonal sub-tiles first), reactions from the rows above
        const int IB = P.IB, JL = P.JL, lgJL = P.lgJL;
        const int Ik = k0 / IB;
        const int off = kc - Ik * IB;
        int lo, hi;
        // partials of 4 tiles (rows) requested before their sums, added in order
        constexpr int U = 4;
        part_of<PARTS>(rowstart[Ik], rowstart[Ik + 1], w, lo, hi);
        for (int t = lo; t < hi; t += U) {
            double a[U][3];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const double* Pt = P.Pi + (size_t)min(t + u, hi - 1) * 3 * IB + off;
                a[u][0] = Pt[0];
                a[u][1] = Pt[IB];
                a[u][2] = Pt[2 * IB];
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (t + u < hi) {
                    v[3] += a[u][0];
                    v[4] += a[u][1];
                    v[5] += a[u][2];
                }
        }
        part_of<PARTS>(0, Ik, w, lo, hi);
        for (int I = lo; I < hi; I += U) {
            int slot[U];
#pragma unroll
            for (int u = 0; u < U; ++u) slot[u] = rowstart[min(I + u, hi - 1)];
            double a[U][3];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int rel = kc - (min(I + u, hi - 1) + 1) * IB;
                const int sI = rel >> lgJL;
                const double* Rt = P.R + (size_t)(slot[u] + P.ndiag + sI) * 3 * JL + (rel - (sI << lgJL));
                a[u][0] = Rt[0];
                a[u][1] = Rt[JL];
                a[u][2] = Rt[2 * JL];
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (I + u < hi) {
                    v[kVals - 4] += a[u][0];
                    v[kVals - 3] += a[u][1];
                    v[kVals - 2] += a[u][2];
                }
        }
    }
#pragma unroll
    for (int c = 0; c < kVals; ++c) red[w][c][lane] = v[c];
    __syncthreads();
    if (w != 0) return;
    // the wave shares in wave order (one wave's values at a time, which keeps
    // the 16-wave form within its 128 VGPRs)
    double acc[kVals];
#pragma unroll
    for (int c = 0; c < kVals; ++c) acc[c] = red[0][c][lane];
#pragma unroll 1
    for (int u = 1; u < PARTS; ++u)
#pragma unroll
        for (int c = 0; c < kVals; ++c) acc[c] += red[u][c][lane];
    double tot[10];
#pragma unroll
    for (int c = 0; c < 10; ++c) tot[c] = 0.0;
#pragma unroll
    for (int c = 0; c < kVals; ++c) tot[WHOLE && c == kPot ? 9 : c] = acc[c];
    double eK = 0.0, eC = 0.0, eT = 0.0;
    if (k < n) {
        const double qk = Q[k];
        step_ion(P, P.traps[ch.x], o + k, xk, yk, zk, qk, kCoulomb * (tot[3] + qk * (tot[0] - tot[6])),
                 kCoulomb * (tot[4] + qk * (tot[1] - tot[7])), kCoulomb * (tot[5] + qk * (tot[2] - tot[8])), tot[9],
                 eK, eC, eT);
    }
    if (mode & EPI_ENERGY)
        energy_arrival(P, ch.x, blockIdx.x, ru.w, ch.x + 1 < P.nrun ? P.runs[ch.x + 1].w : P.nchunk, eK, eC, eT);
}

// Direct pairs of ion kc with the nt j's of an LDS tile (first j = j0), as
// direct_range; the tile entries are read at a uniform address (broadcast).
template <int PREC, bool FORCE, bool POT>
__device__ __forceinline__ void direct_tile(const double4* __restrict__ jt, int nt, int j0, int kc, double xk,
                                            double yk, double zk, double eps2, const SeriesK& K, double (&f)[3],
                                            double& u) {
#pragma unroll 4
    for (int t = 0; t < nt; ++t) {
        const double4 r = jt[t];
        const double dx = xk - r.x, dy = yk - r.y, dz = zk - r.z;
        const double r2 = __builtin_fma(dx, dx, __builtin_fma(dy, dy, __builtin_fma(dz, dz, eps2)));
        double s = 0.0, y = 0.0;
        inv_r<PREC, FORCE, POT>(r2, r.w, K, s, y);
        if (j0 + t == kc) {
            s = 0.0;
            y = 0.0;
        }
        if (FORCE) {
            f[0] = __builtin_fma(dx, s, f[0]);
            f[1] = __builtin_fma(dy, s, f[1]);
            f[2] = __builtin_fma(dz, s, f[2]);
        }
        if (POT) u = __builtin_fma(r.w, y, u);
    }
}

constexpr int kSmallTile = 256;  // j's per LDS tile of k_small_step (8 KB)

// One run of P.n1 ions with trap P.trap1, one launch per step.  Workgroup
// b = one wave: ions 64 c .. 64 c + 63 (c = b / S) against the s-th of S
// parts of the run (s = b % S), whose j data are staged through LDS in
// tiles of kSmallTile (coalesced loads, one memory round trip per tile).
// It stores its sums, and the last of the chunk's S workgroups to arrive
// (counted in P.scount[c], zero at launch and left zero) adds them in part
// order and applies trap, kick and drift.
template <int PREC>
__global__ void __launch_bounds__(64) k_small_step(EnsParams P) {
    __shared__ double4 jt[kSmallTile];
    const int S = P.S;
    const int c = blockIdx.x / S, s = blockIdx.x - c * S;
    const int n = P.n1, lane = threadIdx.x;
    const int k = c * 64 + lane, kc = min(k, n - 1);
    const unsigned mode = P.mode;
    const bool need_f = (mode & (EPI_ACCEL | EPI_KICK)) != 0, need_p = (mode & EPI_ENERGY) != 0;
    const double xk = P.x[kc], yk = P.y[kc], zk = P.z[kc];
    const SeriesK K;
    double f[3] = {0.0, 0.0, 0.0}, u = 0.0;
    const int len = (n + S - 1) / S;
    const int lo = min(n, s * len), hi = min(n, lo + len);
    if (need_f || need_p)
        for (int t0 = lo; t0 < hi; t0 += kSmallTile) {
            const int nt = min(hi - t0, kSmallTile);
            for (int t = lane; t < nt; t += 64) jt[t] = make_double4(P.x[t0 + t], P.y[t0 + t], P.z[t0 + t], P.q[t0 + t]);
            __syncthreads();
            if (need_f && need_p) direct_tile<PREC, true, true>(jt, nt, t0, kc, xk, yk, zk, P.eps2, K, f, u);
            else if (need_f) direct_tile<PREC, true, false>(jt, nt, t0, kc, xk, yk, zk, P.eps2, K, f, u);
            else direct_tile<PREC, false, true>(jt, nt, t0, kc, xk, yk, zk, P.eps2, K, f, u);
            __syncthreads();
        }
    double* mine = P.spart + (size_t)blockIdx.x * 4 * 64;
    mine[lane] = f[0];
    mine[64 + lane] = f[1];
    mine[128 + lane] = f[2];
    mine[192 + lane] = u;
    __threadfence();  // these sums before the arrival
    int last = 0;
    if (lane == 0) last = atomicAdd(&P.scount[c], 1u) == (unsigned)(S - 1);
    last = __shfl(last, 0);
    if (!last) return;
    __threadfence();  // every part of this chunk is visible
    double t[4];
    const double* pc = P.spart + (size_t)c * S * 4 * 64 + lane;
    const double* ps[4] = {pc, pc + 64, pc + 128, pc + 192};
    const size_t st[4] = {4 * 64, 4 * 64, 4 * 64, 4 * 64};
    split_sums<4>(ps, st, S, t);  // the four sums' loads together, each in part order
    if (lane == 0) P.scount[c] = 0u;
    double eK = 0.0, eC = 0.0, eT = 0.0;
    if (k < n) {
        const double cq = kCoulomb * P.q[k];
        step_ion(P, P.trap1, k, xk, yk, zk, P.q[k], cq * t[0], cq * t[1], cq * t[2], t[3], eK, eC, eT);
    }
    if (mode & EPI_ENERGY) energy_arrival(P, 0, c, 0, P.nchunk, eK, eC, eT);
}

__global__ void k_zero_counts(unsigned* __restrict__ c, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) c[i] = 0u;
}

// ----------------------------------------------------------------- host

static size_t al(size_t b) { return (b + 255) / 256 * 256; }

bool ens_cfg_ok(int p, int jl) { return (p == 4 || p == 8) && (jl == 256 || jl == 512); }

// Tables of one ensemble at (P, JL): what the workspace must hold.
struct EnsTables {
    std::vector<int4> tiles, runs;
    std::vector<int> rowstart;
    std::vector<int2> chunks;
    int ndiag = 0;  // diagonal sub-tiles of a full row (0: no tiles)
    int dl = 0;     // j's per diagonal sub-tile
    size_t bytes = 0;
};

// IB: i-block length (64 P; or a multiple of 64 no smaller than any run,
// which makes every run one block and leaves no tiles).
static EnsTables ens_tables(int nrun, const int64_t* offsets, int IB, int JL) {
    EnsTables E;
    struct Tile {
        int4 t;
        int len;
    };
    std::vector<Tile> tl;
    int slot = 0;
    // With any run longer than one i-block, every row starts with its
    // diagonal sub-tiles (one slot each, ceil(rows / DL) of them);
    // otherwise there are no tiles at all.
    bool diag = false;
    size_t noff = 0;
    for (int r = 0; r < nrun; ++r) {
        const int n = (int)(offsets[r + 1] - offsets[r]);
        diag = diag || n > IB;
        for (int I = 0; I * IB < n; ++I) noff += sym_nseg(n, IB, JL, I);
    }
    E.dl = noff < (size_t)kDiagSplitMax ? std::min(IB, kDiagLen) : IB;
    E.ndiag = diag ? (IB + E.dl - 1) / E.dl : 0;
    E.runs.resize(nrun);
    for (int r = 0; r < nrun; ++r) {
        const int o = (int)offsets[r], n = (int)(offsets[r + 1] - offsets[r]);
        const int nI = (n + IB - 1) / IB;
        E.runs[r] = make_int4(o, n, (int)E.rowstart.size(), (int)E.chunks.size());
        for (int I = 0; I < nI; ++I) {
            E.rowstart.push_back(slot);
            if (diag) {
                const int rows = std::min(IB, n - I * IB);
                for (int d = 0; d * E.dl < rows; ++d) {
                    tl.push_back({make_int4(o, n, slot, (I << 16) | (kDiagSeg - d)),
                                  std::min(E.dl, rows - d * E.dl)});
                    ++slot;
                }
            }
            const int ns = sym_nseg(n, IB, JL, I);
            for (int sg = 0; sg < ns; ++sg) {
                const int j0 = (I + 1) * IB + sg * JL;
                tl.push_back({make_int4(o, n, slot, (I << 16) | sg), std::min(JL, n - j0)});
                ++slot;
            }
        }
        E.rowstart.push_back(slot);
        for (int k0 = 0; k0 < n; k0 += 64) E.chunks.push_back(make_int2(r, k0));
    }
    // longest tiles first, so that the short ones fill the end of the launch
    std::stable_sort(tl.begin(), tl.end(), [](const Tile& a, const Tile& b) { return a.len > b.len; });
    E.tiles.reserve(tl.size());
    for (const Tile& t : tl) E.tiles.push_back(t.t);
    const size_t T = E.tiles.size(), nch = E.chunks.size(), ntot = (size_t)offsets[nrun];
    E.bytes = al(sizeof(int4) * (T + 1)) + al(sizeof(int4) * nrun) + al(sizeof(int) * E.rowstart.size()) +
              al(sizeof(int2) * nch) + al(sizeof(cb_trap) * nrun) + al(sizeof(double) * 3 * IB * T) +
              al(sizeof(double) * 3 * (size_t)JL * T) + al(sizeof(double) * 3 * ntot) +
              al(sizeof(double) * 3 * nch) + al(sizeof(unsigned) * nrun);
    return E;
}

// From this many 64-ion chunks on, the finish gives each chunk 2 waves
// instead of 4 (kz512, 16 700 chunks: 1.31-1.34 against 1.33-1.37 ms per
// step; 1 wave measured the same as 2, 8 waves 1.41).
constexpr unsigned kFinishTwoWaves = 4096;

static int whole_ib(int64_t nmax) { return (int)((nmax + 63) / 64 * 64); }

// Upper bound of ens_tables(...).bytes over every ensemble of ntot ions in
// nrun runs of at most kMaxBatchIons, for every allowed (P, JL).  A run of n
// ions has at most n^2 / (2 IB JL) + n / IB off-diagonal tiles and, over
// its ceil(n / IB) <= n / IB + 1 rows, at most n / kDiagLen + n / IB + 1
// diagonal sub-tiles.
size_t ens_ws_bound(int64_t ntot, int32_t nrun) {
    size_t best = 0;
    const double N = (double)ntot;
    for (int P : {4, 8})
        for (int JL : {256, 512}) {
            const int IB = 64 * P;
            const size_t T =
                (size_t)std::ceil(N * (0.5 * kMaxBatchIons / ((double)IB * JL) + 2.0 / IB + 1.0 / kDiagLen)) +
                3 * (size_t)nrun;
            const size_t rows = (size_t)std::ceil(N / IB) + 2 * (size_t)nrun;
            const size_t nch = (size_t)std::ceil(N / 64) + nrun;
            const size_t b = al(sizeof(int4) * (T + 1)) + al(sizeof(int4) * nrun) + al(sizeof(int) * rows) +
                             al(sizeof(int2) * nch) + al(sizeof(cb_trap) * nrun) + al(sizeof(double) * 3 * IB * T) +
                             al(sizeof(double) * 3 * (size_t)JL * T) + al(sizeof(double) * 3 * (size_t)ntot) +
                             al(sizeof(double) * 3 * nch) + al(sizeof(unsigned) * nrun);
            best = std::max(best, b);
        }
    return best;
}

template <int PREC, int P>
static void go_ens_pair(unsigned T, const double* x, const double* y, const double* z, const double* q, double eps2,
                        int JL, int DL, const int4* tiles, double* Pi, double* R, hipStream_t st) {
    k_pair_sym_ens<PREC, P><<<T, 64, 0, st>>>(x, y, z, q, eps2, JL, DL, tiles, Pi, R);
}

template <int PREC>
static void go_ens_pair_p(int P, unsigned T, const double* x, const double* y, const double* z, const double* q,
                          double eps2, int JL, int DL, const int4* tiles, double* Pi, double* R, hipStream_t st) {
    if (P == 8) go_ens_pair<PREC, 8>(T, x, y, z, q, eps2, JL, DL, tiles, Pi, R, st);
    else go_ens_pair<PREC, 4>(T, x, y, z, q, eps2, JL, DL, tiles, Pi, R, st);
}

cb_status md_run_ensemble(int32_t nrun, const int64_t* offsets, const cb_state* s, const double* q,
                          const double* m, const cb_trap* traps, double t0, double dt, int64_t nsteps, double eps2,
                          int32_t prec, uint32_t flags, double* energies, int64_t every, int P, int JL, void* ws,
                          size_t ws_bytes, hipStream_t st) {
    if (P != 0 && !ens_cfg_ok(P, JL))
        return fail(CB_EINVAL, "md_run: ensemble configuration p=%d JL=%d not supported", P, JL);
    int64_t nmax = 0;
    for (int r = 0; r < nrun; ++r) nmax = std::max<int64_t>(nmax, offsets[r + 1] - offsets[r]);
    const int IB = P == 0 ? whole_ib(nmax) : 64 * P;
    if (P == 0) JL = 256;
    const EnsTables E = ens_tables(nrun, offsets, IB, JL);
    if (ws_bytes < E.bytes)
        return fail(CB_ENOWS, "md_run: the ensemble path needs %zu workspace bytes, has %zu", E.bytes, ws_bytes);
    unsigned* fl = flags_ptr();
    if (!fl) return fail(CB_EHIP, "md_run: device flag symbol not found");
    const size_t T = E.tiles.size(), nch = E.chunks.size(), ntot = (size_t)offsets[nrun];

    char* base = static_cast<char*>(ws);
    auto carve = [&](size_t bytes) {
        char* p = base;
        base += al(bytes);
        return p;
    };
    int4* d_tiles = reinterpret_cast<int4*>(carve(sizeof(int4) * (T + 1)));
    int4* d_runs = reinterpret_cast<int4*>(carve(sizeof(int4) * nrun));
    int* d_rows = reinterpret_cast<int*>(carve(sizeof(int) * E.rowstart.size()));
    int2* d_chunks = reinterpret_cast<int2*>(carve(sizeof(int2) * nch));
    cb_trap* d_traps = reinterpret_cast<cb_trap*>(carve(sizeof(cb_trap) * nrun));
    double* Pi = reinterpret_cast<double*>(carve(sizeof(double) * 3 * IB * T));
    double* R = reinterpret_cast<double*>(carve(sizeof(double) * 3 * (size_t)JL * T));
    double* pos2 = reinterpret_cast<double*>(carve(sizeof(double) * 3 * ntot));
    double* echunk = reinterpret_cast<double*>(carve(sizeof(double) * 3 * nch));
    unsigned* ecount = reinterpret_cast<unsigned*>(carve(sizeof(unsigned) * nrun));

    HostUpload up;
    up.add(d_tiles, E.tiles.data(), sizeof(int4) * T);
    up.add(d_runs, E.runs.data(), sizeof(int4) * nrun);
    up.add(d_rows, E.rowstart.data(), sizeof(int) * E.rowstart.size());
    up.add(d_chunks, E.chunks.data(), sizeof(int2) * nch);
    up.add(d_traps, traps, sizeof(cb_trap) * nrun);
    if (cb_status urc = up.run(st, "md_run")) return urc;

    double* bufA[3] = {s->x, s->y, s->z};
    double* bufB[3] = {pos2, pos2 + ntot, pos2 + 2 * ntot};
    double** cur = bufA;
    double** nxt = bufB;

    EnsParams EP{};
    EP.chunks = d_chunks;
    EP.runs = d_runs;
    EP.rowstart = d_rows;
    EP.traps = d_traps;
    EP.Pi = Pi;
    EP.R = R;
    EP.q = q;
    EP.m = m;
    EP.vx = s->vx; EP.vy = s->vy; EP.vz = s->vz;
    EP.ax = s->ax; EP.ay = s->ay; EP.az = s->az;
    EP.IB = IB;
    EP.JL = JL;
    int lgJL = 0;
    while ((1 << lgJL) < JL) ++lgJL;
    EP.lgJL = lgJL;
    EP.ndiag = E.ndiag;
    EP.eps2 = eps2;
    EP.t0 = t0;
    EP.dt = dt;
    EP.echunk = echunk;
    EP.ecount = ecount;
    EP.energies = energies;
    EP.nrun = nrun;
    EP.nchunk = (int)nch;
    EP.nrec = energies ? nsteps / every + 1 : 0;
    EP.flags = fl;
    if (energies) {
        k_zero_counts<<<(nrun + 255) / 256, 256, 0, st>>>(ecount, nrun);
        cb_status rc = check_launch("k_zero_counts");
        if (rc) return rc;
    }

    auto pair_stage = [&]() -> cb_status {
        if (T == 0) return CB_OK;
        switch (prec) {
            case CB_FP64: go_ens_pair_p<PREC_FP64>(P, (unsigned)T, cur[0], cur[1], cur[2], q, eps2, JL, E.dl, d_tiles, Pi, R, st); break;
            case CB_MIXED: go_ens_pair_p<PREC_MIXED>(P, (unsigned)T, cur[0], cur[1], cur[2], q, eps2, JL, E.dl, d_tiles, Pi, R, st); break;
            case CB_FP64_IEEE: go_ens_pair_p<PREC_IEEE>(P, (unsigned)T, cur[0], cur[1], cur[2], q, eps2, JL, E.dl, d_tiles, Pi, R, st); break;
            default: go_ens_pair_p<PREC_FP32>(P, (unsigned)T, cur[0], cur[1], cur[2], q, eps2, JL, E.dl, d_tiles, Pi, R, st); break;
        }
        return check_launch("k_pair_sym_ens");
    };
    // Finish + trap + kick / drift of step `step`.  A launch that reads other
    // ions' positions and drifts writes the other buffer and swaps; a drift
    // alone works in place.  Without tiles every run is one i-block, and 16
    // waves share each chunk.
    const bool whole = T == 0;
    auto step_launch = [&](long long step, unsigned mode, long long rec) -> cb_status {
        const bool reads = (mode & (EPI_ACCEL | EPI_KICK | EPI_ENERGY)) != 0;
        double** out = reads ? nxt : cur;
        EP.x = cur[0]; EP.y = cur[1]; EP.z = cur[2];
        EP.xn = out[0]; EP.yn = out[1]; EP.zn = out[2];
        EP.step = step;
        EP.mode = mode;
        EP.rec = rec;
        const unsigned g = (unsigned)nch;
        if (whole) {
            switch (prec) {
                case CB_FP64: k_ens_step<PREC_FP64, 16, true><<<g, 1024, 0, st>>>(EP); break;
                case CB_MIXED: k_ens_step<PREC_MIXED, 16, true><<<g, 1024, 0, st>>>(EP); break;
                case CB_FP64_IEEE: k_ens_step<PREC_IEEE, 16, true><<<g, 1024, 0, st>>>(EP); break;
                default: k_ens_step<PREC_FP32, 16, true><<<g, 1024, 0, st>>>(EP); break;
            }
        } else if (g < kFinishTwoWaves) {  // few chunks: 4 waves share each
            switch (prec) {
                case CB_FP64: k_ens_step<PREC_FP64, 4, false><<<g, 256, 0, st>>>(EP); break;
                case CB_MIXED: k_ens_step<PREC_MIXED, 4, false><<<g, 256, 0, st>>>(EP); break;
                case CB_FP64_IEEE: k_ens_step<PREC_IEEE, 4, false><<<g, 256, 0, st>>>(EP); break;
                default: k_ens_step<PREC_FP32, 4, false><<<g, 256, 0, st>>>(EP); break;
            }
        } else {  // many chunks fill the chip with 2 waves each
            switch (prec) {
                case CB_FP64: k_ens_step<PREC_FP64, 2, false><<<g, 128, 0, st>>>(EP); break;
                case CB_MIXED: k_ens_step<PREC_MIXED, 2, false><<<g, 128, 0, st>>>(EP); break;
                case CB_FP64_IEEE: k_ens_step<PREC_IEEE, 2, false><<<g, 128, 0, st>>>(EP); break;
                default: k_ens_step<PREC_FP32, 2, false><<<g, 128, 0, st>>>(EP); break;
            }
        }
        cb_status rc = check_launch("k_ens_step");
        if (rc) return rc;
        if ((mode & EPI_DRIFT) && reads) std::swap(cur, nxt);
        return CB_OK;
    };

    cb_status rc;
    const bool rec0 = energies != nullptr;
    const bool init = (flags & CB_INIT_ACCEL) != 0;
    const unsigned mode0 = (init ? EPI_ACCEL : 0u) | (rec0 ? EPI_ENERGY : 0u) | (nsteps > 0 ? EPI_DRIFT : 0u);
    if (init && (rc = pair_stage())) return rc;
    if (mode0 && (rc = step_launch(0, mode0, 0))) return rc;
    for (long long k = 1; k <= nsteps; ++k) {
        const bool rec = rec0 && (k % every == 0);
        if ((rc = pair_stage())) return rc;
        if ((rc = step_launch(k, EPI_KICK | (rec ? EPI_ENERGY : 0u) | (k < nsteps ? EPI_DRIFT : 0u), rec ? k / every : 0)))
            return rc;
    }
    if (cur != bufA)
        for (int c = 0; c < 3; ++c)
            if (hipMemcpyAsync(bufA[c], cur[c], sizeof(double) * ntot, hipMemcpyDeviceToDevice, st) != hipSuccess)
                return fail(CB_EHIP, "md_run: copy of the final positions failed");
    return ok();
}

size_t md_small_ws_bytes(int64_t n, int S) {
    const size_t nch = (size_t)((n + 63) / 64);
    return al(sizeof(double) * 3 * (size_t)n) + al(sizeof(double) * 3 * nch) + al(sizeof(unsigned)) +
           al(sizeof(double) * 4 * 64 * nch * (size_t)S) + al(sizeof(unsigned) * nch);
}

// Parts of at least 32 j's, at most 8 of them (measured on MI355X at
// 256 and 1024 ions).
int small_parts(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>(n / 32, 8)); }

// One run of n <= kSmallRunMax ions, one launch per step (k_small_step).
// Kernels and device-to-device copies only (nothing from the host), so a
// caller may capture it in a graph.
cb_status md_run_small(int64_t n, const cb_state* s, const double* q, const double* m, const cb_trap* trap,
                       double t0, double dt, int64_t nsteps, double eps2, int32_t prec, uint32_t flags,
                       double* energies, int64_t every, int S, void* ws, size_t ws_bytes, hipStream_t st) {
    if (S < 1 || S > kSmallPartsMax) return fail(CB_EINVAL, "md_run: %d j-parts per 64 ions not supported", S);
    if (ws_bytes < md_small_ws_bytes(n, S))
        return fail(CB_ENOWS, "md_run: workspace too small for the one-launch step");
    unsigned* fl = flags_ptr();
    if (!fl) return fail(CB_EHIP, "md_run: device flag symbol not found");
    const size_t N = (size_t)n, nch = (N + 63) / 64;
    char* base = static_cast<char*>(ws);
    auto carve = [&](size_t bytes) {
        char* p = base;
        base += al(bytes);
        return p;
    };
    double* pos2 = reinterpret_cast<double*>(carve(sizeof(double) * 3 * N));
    double* echunk = reinterpret_cast<double*>(carve(sizeof(double) * 3 * nch));
    unsigned* ecount = reinterpret_cast<unsigned*>(carve(sizeof(unsigned)));
    double* spart = reinterpret_cast<double*>(carve(sizeof(double) * 4 * 64 * nch * (size_t)S));
    unsigned* scount = reinterpret_cast<unsigned*>(carve(sizeof(unsigned) * nch));

    double* bufA[3] = {s->x, s->y, s->z};
    double* bufB[3] = {pos2, pos2 + N, pos2 + 2 * N};
    double** cur = bufA;
    double** nxt = bufB;
    EnsParams EP{};
    EP.q = q;
    EP.m = m;
    EP.vx = s->vx; EP.vy = s->vy; EP.vz = s->vz;
    EP.ax = s->ax; EP.ay = s->ay; EP.az = s->az;
    EP.eps2 = eps2;
    EP.t0 = t0;
    EP.dt = dt;
    EP.echunk = echunk;
    EP.ecount = ecount;
    EP.energies = energies;
    EP.nrun = 1;
    EP.nchunk = (int)nch;
    EP.nrec = energies ? nsteps / every + 1 : 0;
    EP.flags = fl;
    EP.n1 = (int)n;
    EP.trap1 = *trap;
    EP.S = S;
    EP.spart = spart;
    EP.scount = scount;
    k_zero_counts<<<(unsigned)((nch + 1 + 255) / 256), 256, 0, st>>>(scount, (int)nch);
    cb_status rc = check_launch("k_zero_counts");
    if (rc) return rc;
    k_zero_counts<<<1, 64, 0, st>>>(ecount, 1);
    if ((rc = check_launch("k_zero_counts"))) return rc;
    // A launch that reads other ions' positions and drifts writes the other
    // buffer and swaps; a drift alone works in place.
    auto step_launch = [&](long long step, unsigned mode, long long rec) -> cb_status {
        const bool reads = (mode & (EPI_ACCEL | EPI_KICK | EPI_ENERGY)) != 0;
        double** out = reads ? nxt : cur;
        EP.x = cur[0]; EP.y = cur[1]; EP.z = cur[2];
        EP.xn = out[0]; EP.yn = out[1]; EP.zn = out[2];
        EP.step = step;
        EP.mode = mode;
        EP.rec = rec;
        const unsigned g = (unsigned)(nch * (size_t)S);
        switch (prec) {
            case CB_FP64: k_small_step<PREC_FP64><<<g, 64, 0, st>>>(EP); break;
            case CB_MIXED: k_small_step<PREC_MIXED><<<g, 64, 0, st>>>(EP); break;
            case CB_FP64_IEEE: k_small_step<PREC_IEEE><<<g, 64, 0, st>>>(EP); break;
            default: k_small_step<PREC_FP32><<<g, 64, 0, st>>>(EP); break;
        }
        cb_status r = check_launch("k_small_step");
        if (r) return r;
        if ((mode & EPI_DRIFT) && reads) std::swap(cur, nxt);
        return CB_OK;
    };
    const bool rec0 = energies != nullptr;
    const bool init = (flags & CB_INIT_ACCEL) != 0;
    const unsigned mode0 = (init ? EPI_ACCEL : 0u) | (rec0 ? EPI_ENERGY : 0u) | (nsteps > 0 ? EPI_DRIFT : 0u);
    if (mode0 && (rc = step_launch(0, mode0, 0))) return rc;
    for (long long k = 1; k <= nsteps; ++k) {
        const bool rec = rec0 && (k % every == 0);
        if ((rc = step_launch(k, EPI_KICK | (rec ? EPI_ENERGY : 0u) | (k < nsteps ? EPI_DRIFT : 0u), rec ? k / every : 0)))
            return rc;
    }
    if (cur != bufA)
        for (int c = 0; c < 3; ++c)
            if (hipMemcpyAsync(bufA[c], cur[c], sizeof(double) * N, hipMemcpyDeviceToDevice, st) != hipSuccess)
                return fail(CB_EHIP, "md_run: copy of the final positions failed");
    return ok();
}

}  // namespace cb
