// Batched persistent velocity-Verlet kernel: many independent runs of uneven
// size (the paper's Kibble-Zurek statistics use case, introduction) in one
// launch, one workgroup per run at a time.
//
// Layout: each workgroup keeps its run's positions and charges in LDS as
// {x, y, z, q} per ion (32 B; 4096 ions = 128 KB), read with broadcast
// ds_read_b128 in the pair loop; velocities and accelerations stay in the
// caller's arrays (each thread reads and writes only its own ions, L2
// resident).  A thread owns P ions per register group (ions g*P*WG + p*WG +
// tid); the self pair is masked only in the 64-wide j chunks that hold the
// wave's own ions.  Runs are taken from an atomic queue in largest-N^2-first
// order so that the long runs start first.  Per step: drift (own ions, LDS),
// barrier, pair loop over LDS, kick, optional energy record, barrier.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

#include "internal.hpp"
#include "rsqrt.hpp"
#include "step_common.hpp"
#include "wave_reduce.hpp"

namespace cb {

// Newton's-third-law pass for the largest runs (the ones that bound the
// launch's makespan): blocks of kSymBS ions (one wave, kSymBP per lane), every
// unordered pair of blocks once in a round-robin schedule in which the eight
// waves hold disjoint pairs of blocks, so each block's force accumulator is
// touched by one wave per round.  The accumulators (force / k_C, [3][4096] per
// workgroup) live in the workspace and stay in L2.  Runs of at most
// kSymBatchMin ions (fewer than 13 blocks would leave waves idle) and
// energy-recording steps take the direct pass.
constexpr int kSymBP = 4;
constexpr int kSymBS = 64 * kSymBP;
constexpr int kSymBatchMin = 3072;

struct BatchParams {
    int nrun;
    const int64_t* offsets;  // [nrun+1]
    const int* order;        // [nrun] runs, longest first
    const cb_trap* traps;    // [nrun]
    int* queue;              // one counter, zero on entry
    double *x, *y, *z, *vx, *vy, *vz, *ax, *ay, *az;
    const double* q;
    const double* m;
    double t0, dt, eps2;
    long long nsteps, every;
    int init;
    double* energies;  // [nrun][nsteps/every+1][4] or null
    unsigned* flags;
    double* facc;  // [gridDim.x][3][kMaxBatchIons]: force / k_C of the Newton's-third-law pass
};

template <int PREC, bool POT>
__device__ __forceinline__ void batch_pairs(const double4* __restrict__ sh, int n, int gbase, int tid,
                                            double eps2, const SeriesK& K, double (&fx)[kBatchP],
                                            double (&fy)[kBatchP], double (&fz)[kBatchP], double (&ph)[kBatchP]) {
    double xi[kBatchP], yi[kBatchP], zi[kBatchP];
    int ii[kBatchP];
#pragma unroll
    for (int p = 0; p < kBatchP; ++p) {
        ii[p] = gbase + p * kBatchWG + tid;
        const double4 r = sh[min(ii[p], n - 1)];
        xi[p] = r.x;
        yi[p] = r.y;
        zi[p] = r.z;
        fx[p] = fy[p] = fz[p] = ph[p] = 0.0;
    }
    const int wbase = gbase + (tid & ~63);  // first ion of this wave in slot p = 0
    for (int c0 = 0; c0 < n; c0 += 64) {
        const int c1 = min(n, c0 + 64);
        bool diag = false;
#pragma unroll
        for (int p = 0; p < kBatchP; ++p) diag |= (c0 == wbase + p * kBatchWG);
        double ax[kBatchP], ay[kBatchP], az[kBatchP], ap[kBatchP];
#pragma unroll
        for (int p = 0; p < kBatchP; ++p) ax[p] = ay[p] = az[p] = ap[p] = 0.0;
        for (int j = c0; j < c1; ++j) {
            const double4 rj = sh[j];
#pragma unroll
            for (int p = 0; p < kBatchP; ++p) {
                const double dx = xi[p] - rj.x, dy = yi[p] - rj.y, dz = zi[p] - rj.z;
                const double r2 = __builtin_fma(dx, dx, __builtin_fma(dy, dy, __builtin_fma(dz, dz, eps2)));
                double s, y;
                inv_r<PREC, true, POT>(r2, rj.w, K, s, y);
                if (diag && ii[p] == j) {
                    s = 0.0;
                    y = 0.0;
                }
                ax[p] = __builtin_fma(dx, s, ax[p]);
                ay[p] = __builtin_fma(dy, s, ay[p]);
                az[p] = __builtin_fma(dz, s, az[p]);
                if (POT) ap[p] = __builtin_fma(rj.w, y, ap[p]);
            }
        }
#pragma unroll
        for (int p = 0; p < kBatchP; ++p) {
            fx[p] += ax[p];
            fy[p] += ay[p];
            fz[p] += az[p];
            if (POT) ph[p] += ap[p];
        }
    }
}

// Round r of the circle method over Bp (even) blocks: slot k pairs (a, b).
__device__ __forceinline__ void rr_pair(int Bp, int r, int k, int& a, int& b) {
    if (k == 0) {
        a = r;
        b = Bp - 1;
    } else {
        a = (r + k) % (Bp - 1);
        b = (r - k + Bp - 1) % (Bp - 1);
    }
}

// Pairs between block I (i's, one per lane and slot) and block J > I (j's):
// i sums into F[I] (q_i q_j d r^-3), reactions -q_j sum_i q_i d r^-3 into F[J].
// F is [3][kMaxBatchIons].  Block I is full; J may be the run's ragged last.
template <int PREC>
__device__ __forceinline__ void sym_block_pair(const double4* __restrict__ sh, int n, int I, int J, double eps2,
                                               const SeriesK& K, double* __restrict__ F) {
    const int lane = threadIdx.x & 63;
    double xi[kSymBP], yi[kSymBP], zi[kSymBP], qi[kSymBP], ia[kSymBP][3];
#pragma unroll
    for (int p = 0; p < kSymBP; ++p) {
        const double4 r = sh[I * kSymBS + p * 64 + lane];
        xi[p] = r.x;
        yi[p] = r.y;
        zi[p] = r.z;
        qi[p] = r.w;
        ia[p][0] = ia[p][1] = ia[p][2] = 0.0;
    }
    const int j0 = J * kSymBS, j1 = min(n, j0 + kSymBS);
    for (int jg = j0; jg < j1; jg += 4) {
        const int live = min(4, j1 - jg);
        double jv[12];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const double4 rj = sh[jg + min(u, live - 1)];
            double a0 = 0.0, a1 = 0.0, a2 = 0.0;
#pragma unroll
            for (int p = 0; p < kSymBP; ++p) {
                const double dx = xi[p] - rj.x, dy = yi[p] - rj.y, dz = zi[p] - rj.z;
                const double r2 = __builtin_fma(dx, dx, __builtin_fma(dy, dy, __builtin_fma(dz, dz, eps2)));
                double s, y;
                inv_r<PREC, true, false>(r2, qi[p], K, s, y);  // q_i r^-3
                if (u >= live) s = 0.0;
                const double sq = s * rj.w;
                ia[p][0] = __builtin_fma(dx, sq, ia[p][0]);
                ia[p][1] = __builtin_fma(dy, sq, ia[p][1]);
                ia[p][2] = __builtin_fma(dz, sq, ia[p][2]);
                a0 = __builtin_fma(dx, s, a0);
                a1 = __builtin_fma(dy, s, a1);
                a2 = __builtin_fma(dz, s, a2);
            }
            jv[3 * u + 0] = a0;
            jv[3 * u + 1] = a1;
            jv[3 * u + 2] = a2;
        }
        // keep the i-sum updates ahead of the reduction (register pressure)
#pragma unroll
        for (int p = 0; p < kSymBP; ++p) asm volatile("" : "+v"(ia[p][0]), "+v"(ia[p][1]), "+v"(ia[p][2]));
        double o[3];
        reduce_scatter12(jv, o);
        const int g = lane >> 4, c = lane & 15;
        if (g < live && c < 3) {
            const int j = jg + g;
            F[c * kMaxBatchIons + j] -= sh[j].w * ((c == 0) ? o[0] : ((c == 1) ? o[1] : o[2]));
        }
    }
#pragma unroll
    for (int p = 0; p < kSymBP; ++p) {
        const int i = I * kSymBS + p * 64 + lane;
#pragma unroll
        for (int c = 0; c < 3; ++c) F[c * kMaxBatchIons + i] += ia[p][c];
    }
}

// Pairs inside block I (each ordered pair, the self pair masked): into F[I].
template <int PREC>
__device__ __forceinline__ void sym_block_diag(const double4* __restrict__ sh, int n, int I, double eps2,
                                               const SeriesK& K, double* __restrict__ F) {
    const int lane = threadIdx.x & 63;
    const int b0 = I * kSymBS, b1 = min(n, b0 + kSymBS);
    double xi[kSymBP], yi[kSymBP], zi[kSymBP], acc[kSymBP][3];
    int ii[kSymBP];
#pragma unroll
    for (int p = 0; p < kSymBP; ++p) {
        ii[p] = b0 + p * 64 + lane;
        const double4 r = sh[min(ii[p], b1 - 1)];
        xi[p] = r.x;
        yi[p] = r.y;
        zi[p] = r.z;
        acc[p][0] = acc[p][1] = acc[p][2] = 0.0;
    }
    for (int j = b0; j < b1; ++j) {
        const double4 rj = sh[j];
#pragma unroll
        for (int p = 0; p < kSymBP; ++p) {
            const double dx = xi[p] - rj.x, dy = yi[p] - rj.y, dz = zi[p] - rj.z;
            const double r2 = __builtin_fma(dx, dx, __builtin_fma(dy, dy, __builtin_fma(dz, dz, eps2)));
            double s, y;
            inv_r<PREC, true, false>(r2, rj.w, K, s, y);  // q_j r^-3
            if (ii[p] == j) s = 0.0;
            acc[p][0] = __builtin_fma(dx, s, acc[p][0]);
            acc[p][1] = __builtin_fma(dy, s, acc[p][1]);
            acc[p][2] = __builtin_fma(dz, s, acc[p][2]);
        }
    }
#pragma unroll
    for (int p = 0; p < kSymBP; ++p)
        if (ii[p] < b1) {
            const double qi = sh[ii[p]].w;
#pragma unroll
            for (int c = 0; c < 3; ++c) F[c * kMaxBatchIons + ii[p]] += qi * acc[p][c];
        }
}

// Forces / k_C of every ion of the run into F, Newton's third law.  Called by
// the whole workgroup; every thread reaches every barrier.
template <int PREC>
__device__ void sym_run_forces(const double4* __restrict__ sh, int n, double eps2, const SeriesK& K,
                               double* __restrict__ F) {
    const int tid = threadIdx.x, w = tid >> 6;
    constexpr int kWaves = kBatchWG / 64;
    const int B = (n + kSymBS - 1) / kSymBS;  // <= 16
    const int Bp = B + (B & 1);
    for (int i = tid; i < n; i += kBatchWG) F[i] = F[kMaxBatchIons + i] = F[2 * kMaxBatchIons + i] = 0.0;
    __syncthreads();
    for (int I = w; I < B; I += kWaves) sym_block_diag<PREC>(sh, n, I, eps2, K, F);
    __syncthreads();
    for (int r = 0; r < Bp - 1; ++r) {
        if (w < Bp / 2) {
            int a, b;
            rr_pair(Bp, r, w, a, b);
            if (a < B && b < B) sym_block_pair<PREC>(sh, n, min(a, b), max(a, b), eps2, K, F);
        }
        __syncthreads();
    }
}

__device__ __forceinline__ void block_sum3_wg(double& a, double& b, double& c, double* red) {
    // fixed-order tree over kBatchWG threads, red: 3*kBatchWG doubles of LDS
    const int t = threadIdx.x;
    red[t] = a;
    red[kBatchWG + t] = b;
    red[2 * kBatchWG + t] = c;
    __syncthreads();
    for (int w = kBatchWG / 2; w > 0; w >>= 1) {
        if (t < w) {
            red[t] += red[t + w];
            red[kBatchWG + t] += red[kBatchWG + t + w];
            red[2 * kBatchWG + t] += red[2 * kBatchWG + t + w];
        }
        __syncthreads();
    }
    a = red[0];
    b = red[kBatchWG];
    c = red[2 * kBatchWG];
    __syncthreads();
}

// One pass of the pair loop over every ion group of the run, then `op` on
// each owned ion with its force sums (before the k_C q_i factor) and potential.
template <int PREC, bool POT, class Op>
__device__ __forceinline__ void for_groups(const double4* sh, int n, double eps2, const SeriesK& K, Op op) {
    const int tid = threadIdx.x;
    for (int gbase = 0; gbase < n; gbase += kBatchP * kBatchWG) {
        double fx[kBatchP], fy[kBatchP], fz[kBatchP], ph[kBatchP];
        batch_pairs<PREC, POT>(sh, n, gbase, tid, eps2, K, fx, fy, fz, ph);
#pragma unroll
        for (int p = 0; p < kBatchP; ++p) {
            const int i = gbase + p * kBatchWG + tid;
            if (i < n) op(i, fx[p], fy[p], fz[p], ph[p]);
        }
    }
}

template <int PREC>
__global__ void __launch_bounds__(kBatchWG) k_batched(BatchParams B) {
    extern __shared__ double4 sh[];  // run positions + charges, then 3*kBatchWG doubles of reduction space
    __shared__ int s_slot;
    const int tid = threadIdx.x;
    const SeriesK K;
    for (;;) {
        if (tid == 0) s_slot = atomicAdd(B.queue, 1);
        __syncthreads();
        const int slot = s_slot;
        __syncthreads();
        if (slot >= B.nrun) break;
        const int run = B.order[slot];
        const int64_t o = B.offsets[run];
        const int n = (int)(B.offsets[run + 1] - o);
        const cb_trap tr = B.traps[run];
        double* red = reinterpret_cast<double*>(sh + n);
        double *X = B.x + o, *Y = B.y + o, *Z = B.z + o;
        double *VX = B.vx + o, *VY = B.vy + o, *VZ = B.vz + o;
        double *AX = B.ax + o, *AY = B.ay + o, *AZ = B.az + o;
        const double *Q = B.q + o, *M = B.m + o;
        for (int i = tid; i < n; i += kBatchWG) sh[i] = make_double4(X[i], Y[i], Z[i], Q[i]);
        __syncthreads();
        const double dt = B.dt, hdt = 0.5 * dt, hdt2 = 0.5 * dt * dt, eps2 = B.eps2;
        const double Gam = tr.gamma;  // friction coefficient Gamma (kg/s), uniform over the run
        bool bad = false;
        const long long nrec = B.energies ? B.nsteps / B.every + 1 : 0;
        double* Erun = B.energies ? B.energies + (size_t)run * nrec * 4 : nullptr;

        // step 0: initial acceleration and/or energies
        const bool rec0 = Erun != nullptr;
        if (B.init || rec0) {
            const TrapK k = trap_k(tr, step_time(B.t0, dt, 0));
            double eK = 0.0, eC = 0.0, eT = 0.0;
            auto op0 = [&](int i, double fx, double fy, double fz, double ph) {
                const double c = kCoulomb * Q[i];
                const double mi = M[i];
                const double4 r = sh[i];
                if (B.init) {
                    AX[i] = c * fx / mi - k.kx * r.x;
                    AY[i] = c * fy / mi - k.ky * r.y;
                    AZ[i] = c * fz / mi - k.kz * r.z;
                }
                if (rec0) {
                    const double vx = VX[i], vy = VY[i], vz = VZ[i];
                    eK += 0.5 * mi * (vx * vx + vy * vy + vz * vz);
                    eC += 0.5 * c * ph;
                    eT += 0.5 * mi * (k.kx * r.x * r.x + k.ky * r.y * r.y + k.kz * r.z * r.z);
                }
            };
            if (rec0) for_groups<PREC, true>(sh, n, eps2, K, op0);
            else for_groups<PREC, false>(sh, n, eps2, K, op0);
            if (rec0) {
                block_sum3_wg(eK, eC, eT, red);
                if (tid == 0) {
                    Erun[0] = eK;
                    Erun[1] = eC;
                    Erun[2] = eT;
                    Erun[3] = eK + eC + eT;
                }
            }
        }
        __syncthreads();
        for (long long s = 1; s <= B.nsteps; ++s) {
            // drift of the owned ions
            for (int i = tid; i < n; i += kBatchWG) {
                double4 r = sh[i];
                if (Gam == 0.0) {
                    r.x = r.x + VX[i] * dt + hdt2 * AX[i];
                    r.y = r.y + VY[i] * dt + hdt2 * AY[i];
                    r.z = r.z + VZ[i] * dt + hdt2 * AZ[i];
                } else {  // the drift sees the friction acceleration -g v too
                    const double g = Gam / M[i];
                    r.x = r.x + VX[i] * dt + hdt2 * (AX[i] - g * VX[i]);
                    r.y = r.y + VY[i] * dt + hdt2 * (AY[i] - g * VY[i]);
                    r.z = r.z + VZ[i] * dt + hdt2 * (AZ[i] - g * VZ[i]);
                }
                sh[i] = r;
            }
            __syncthreads();
            const TrapK k = trap_k(tr, step_time(B.t0, dt, s));
            const bool rec = Erun && (s % B.every == 0);
            double eK = 0.0, eC = 0.0, eT = 0.0;
            // kick of ion i with its Coulomb force (Fx, Fy, Fz)
            auto kick = [&](int i, double Fx, double Fy, double Fz) {
                const double mi = M[i];
                const double4 r = sh[i];
                const double anx = Fx / mi - k.kx * r.x;
                const double any = Fy / mi - k.ky * r.y;
                const double anz = Fz / mi - k.kz * r.z;
                double vx, vy, vz;
                if (Gam == 0.0) {
                    vx = VX[i] + hdt * (AX[i] + anx);
                    vy = VY[i] + hdt * (AY[i] + any);
                    vz = VZ[i] + hdt * (AZ[i] + anz);
                } else {  // friction -g v by the trapezoidal rule, g = Gamma / m_i
                    const double g = Gam / mi, lo = 1.0 - g * hdt, hi = 1.0 + g * hdt;
                    vx = (VX[i] * lo + hdt * (AX[i] + anx)) / hi;
                    vy = (VY[i] * lo + hdt * (AY[i] + any)) / hi;
                    vz = (VZ[i] * lo + hdt * (AZ[i] + anz)) / hi;
                }
                VX[i] = vx;
                VY[i] = vy;
                VZ[i] = vz;
                AX[i] = anx;
                AY[i] = any;
                AZ[i] = anz;
                bad |= !(__builtin_isfinite(anx) && __builtin_isfinite(any) && __builtin_isfinite(anz));
                if (rec) {
                    eK += 0.5 * mi * (vx * vx + vy * vy + vz * vz);
                    eT += 0.5 * mi * (k.kx * r.x * r.x + k.ky * r.y * r.y + k.kz * r.z * r.z);
                }
            };
            auto op = [&](int i, double fx, double fy, double fz, double ph) {
                const double c = kCoulomb * Q[i];
                kick(i, c * fx, c * fy, c * fz);
                if (rec) eC += 0.5 * c * ph;
            };
            if (rec) {
                for_groups<PREC, true>(sh, n, eps2, K, op);
            } else if (n > kSymBatchMin) {
                double* F = B.facc + (size_t)blockIdx.x * 3 * kMaxBatchIons;
                sym_run_forces<PREC>(sh, n, eps2, K, F);
                for (int i = tid; i < n; i += kBatchWG)
                    kick(i, kCoulomb * F[i], kCoulomb * F[kMaxBatchIons + i], kCoulomb * F[2 * kMaxBatchIons + i]);
            } else {
                for_groups<PREC, false>(sh, n, eps2, K, op);
            }
            if (rec) {
                block_sum3_wg(eK, eC, eT, red);
                if (tid == 0) {
                    double* e = Erun + (s / B.every) * 4;
                    e[0] = eK;
                    e[1] = eC;
                    e[2] = eT;
                    e[3] = eK + eC + eT;
                }
            }
            __syncthreads();
        }
        for (int i = tid; i < n; i += kBatchWG) {
            const double4 r = sh[i];
            X[i] = r.x;
            Y[i] = r.y;
            Z[i] = r.z;
        }
        if (bad) atomicOr(B.flags, 1u);
        __syncthreads();
    }
}

__global__ void k_zero_int(int* p) { *p = 0; }

}  // namespace cb

namespace cb {

cb_status md_run_batched(int32_t nrun, const int64_t* offsets, const cb_state* s, const double* q,
                         const double* m, const cb_trap* traps, double t0, double dt, int64_t nsteps,
                         double eps2, int32_t prec, uint32_t flags, double* energies, int64_t every, void* ws,
                         size_t ws_bytes, hipStream_t st) {
    int nmax = 0;
    for (int r = 0; r < nrun; ++r) nmax = std::max<int>(nmax, (int)(offsets[r + 1] - offsets[r]));
    if (nmax > kMaxBatchIons)
        return fail(CB_EUNSUPPORTED, "md_run: batched runs hold at most %d ions (largest run has %d)", kMaxBatchIons,
                    nmax);
    if (prec != CB_FP64 && prec != CB_MIXED && prec != CB_FP64_IEEE && prec != CB_FP32_RSQ)
        return fail(CB_EINVAL, "md_run: unknown precision %d", prec);
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return fail(CB_EHIP, "md_run: device query failed");
    // Path.  A forced or tuned entry decides.  Otherwise estimate the time of
    // one step on each path from rates measured on MI355X: this kernel runs
    // a small run at about 1.6e9 ordered pairs/s per CU (its runs are spread
    // over the CUs, the largest bounding the step); the stepped path costs
    // about 40 us of launch latency per step plus the pairs at 1.8e12/s.
    // The stepped path uses 256-ion i-blocks, with 512-ion j-segments when
    // the ensemble holds 2^30 or more ordered pairs (4096 or more tiles) and
    // 256-ion ones below (measured on MI355X, ms per step with JL 256 / 512:
    // kz512's 512 runs of 64-4096 ions 1.211 / 1.182; 1024 runs of
    // 1024-4096 3.189 / 3.144; 256 of 2048-4096 1.024 / 1.004; but 128 runs
    // of 64-2048, 1.9e8 pairs, 0.137 / 0.185).  Eight ions per lane were
    // slower for each of these mixes.
    LaunchCfg ec = get_cfg(CB_OP_MD_ENSEMBLE, offsets[nrun], prec);
    if (!ec.tuned) {
        double pairs = 0.0;
        for (int r = 0; r < nrun; ++r)
            pairs += (double)(offsets[r + 1] - offsets[r]) * (double)(offsets[r + 1] - offsets[r]);
        const double t_persistent = std::ceil((double)nrun / ncu) * (double)nmax * nmax / 1.6e9;
        const double t_stepped = 40e-6 + pairs / 1.8e12;
        ec.algo = t_stepped < t_persistent ? ALGO_SYM_LDS : ALGO_DIRECT;
        ec.p = 4;
        ec.splits = pairs >= 1073741824.0 ? 512 : 256;
    }
    if (ec.algo == ALGO_SYM_LDS) {
        const WsLayout LE = ws_layout(CB_OP_MD_RUN, offsets[nrun], nrun, 1, prec);
        return md_run_ensemble(nrun, offsets, s, q, m, traps, t0, dt, nsteps, eps2, prec, flags, energies, every, ec.p,
                               ec.splits, static_cast<char*>(ws) + LE.aux, ws_bytes - LE.aux, st);
    }
    unsigned* fl = flags_ptr();
    if (!fl) return fail(CB_EHIP, "md_run: device flag symbol not found");

    // run table in the workspace: offsets, order, traps, queue counter
    const WsLayout L = ws_layout(CB_OP_MD_RUN, offsets[nrun], nrun, 1, prec);
    char* base = static_cast<char*>(ws) + L.batch;
    int64_t* d_off = reinterpret_cast<int64_t*>(base);
    int* d_order = reinterpret_cast<int*>(d_off + (nrun + 1));
    int* d_queue = d_order + nrun;
    size_t trap_off = (reinterpret_cast<char*>(d_queue + 1) - base + 63) / 64 * 64;
    cb_trap* d_traps = reinterpret_cast<cb_trap*>(base + trap_off);

    std::vector<int> order(nrun);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        return (offsets[a + 1] - offsets[a]) > (offsets[b + 1] - offsets[b]);
    });
    HostUpload up;
    up.add(d_off, offsets, sizeof(int64_t) * (nrun + 1));
    up.add(d_order, order.data(), sizeof(int) * nrun);
    up.add(d_traps, traps, sizeof(cb_trap) * nrun);
    cb_status rc = up.run(st, "md_run");
    if (rc) return rc;
    k_zero_int<<<1, 1, 0, st>>>(d_queue);
    rc = check_launch("k_zero_int");
    if (rc) return rc;

    BatchParams B{};
    B.nrun = nrun;
    B.offsets = d_off;
    B.order = d_order;
    B.traps = d_traps;
    B.queue = d_queue;
    B.x = s->x; B.y = s->y; B.z = s->z;
    B.vx = s->vx; B.vy = s->vy; B.vz = s->vz;
    B.ax = s->ax; B.ay = s->ay; B.az = s->az;
    B.q = q;
    B.m = m;
    B.t0 = t0;
    B.dt = dt;
    B.eps2 = eps2;
    B.nsteps = nsteps;
    B.every = energies ? every : 1;
    B.init = (flags & CB_INIT_ACCEL) ? 1 : 0;
    B.energies = energies;
    B.flags = fl;
    B.facc = reinterpret_cast<double*>(static_cast<char*>(ws) + L.aux);

    const size_t lds = sizeof(double4) * (size_t)nmax + sizeof(double) * 3 * kBatchWG;
    const int per_cu = std::max(1, (int)((160 * 1024) / lds));
    const int grid = std::min(std::min(nrun, ncu * std::min(per_cu, 2)), kBatchGridMax);
    auto launch = [&](auto kern) -> cb_status {
        if (hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)lds) != hipSuccess)
            return fail(CB_EHIP, "md_run: cannot reserve %zu bytes of LDS", lds);
        kern<<<grid, kBatchWG, lds, st>>>(B);
        return CB_OK;
    };
    switch (prec) {
        case CB_FP64: rc = launch(k_batched<PREC_FP64>); break;
        case CB_MIXED: rc = launch(k_batched<PREC_MIXED>); break;
        case CB_FP64_IEEE: rc = launch(k_batched<PREC_IEEE>); break;
        default: rc = launch(k_batched<PREC_FP32>); break;
    }
    if (rc) return rc;
    if ((rc = check_launch("k_batched"))) return rc;
    return ok();
}

}  // namespace cb
