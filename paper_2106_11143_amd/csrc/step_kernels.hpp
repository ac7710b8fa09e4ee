// Element-wise kernels around the pair loop: fixed-order sum of the j-split
// partials, scaling to forces, trap, velocity-Verlet kick and drift (paper,
// section 2), per-ion energy terms and their deterministic reduction.
#pragma once
#include <hip/hip_runtime.h>

#include "split_sum.hpp"
#include "step_common.hpp"

namespace cb {

struct EpiParams {
    int n, S;
    const double* part;  // [S][3][n]
    const double* ppot;  // [S][n]
    const double* q;
    const double* m;
    double *x, *y, *z, *vx, *vy, *vz, *ax, *ay, *az;
    double *fx, *fy, *fz;
    cb_trap trap;
    double t0, dt;
    long long step;  // the trap is taken at step_time(t0, dt, step)
    unsigned mode;
    double* eblk;  // [gridDim.x][3]
    unsigned* flags;
    // With EPI_ENERGY and efinal set, the last block to finish sums the block
    // partials (in block order, so the result does not depend on timing)
    // into efinal: K, U_C, U_trap, E (U_C alone with EPI_UC_ONLY).  ecount
    // is zero at launch and is left zero.
    double* efinal;
    unsigned* ecount;
    // Deferred finish of an earlier energy record (md_run; not together
    // with efinal): with eprev set, one extra block after the ions' blocks
    // sums the nprev block partials at eprev, written by an earlier launch
    // on the stream and so complete, in block order into eprev_out (K, U_C,
    // U_trap, E).  The sum is the one the last-arriving block would form.
    const double* eprev;
    double* eprev_out;
    int nprev;
};

// a, b, c summed over the block (every thread gets the sums): a butterfly of
// cross-lane exchanges within each wave (lanes exchanging the same two values
// add them in either order to the same result), then the waves' sums in wave
// order.  One barrier pair instead of a tree through LDS.
__device__ __forceinline__ void block_sum3_waves(double& a, double& b, double& c) {
    constexpr int kWaves = kEpiThreads / 64;
    __shared__ double sh[3][kWaves];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_xor(a, o);
        b += __shfl_xor(b, o);
        c += __shfl_xor(c, o);
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sh[0][w] = a;
        sh[1][w] = b;
        sh[2][w] = c;
    }
    __syncthreads();
    a = sh[0][0];
    b = sh[1][0];
    c = sh[2][0];
#pragma unroll
    for (int k = 1; k < kWaves; ++k) {
        a += sh[0][k];
        b += sh[1][k];
        c += sh[2][k];
    }
    __syncthreads();  // sh may be reused by a later call
}

// Sums nb block partials [nb][3] in a fixed order into out: with what =
// REC_UC, out[0] = U_C; with REC_UPOT, out[0] = U_C + U_trap; with REC_ALL,
// out[0..3] = K, U_C, U_trap, K + U_C + U_trap.  Called by every thread of
// one block.
__device__ __forceinline__ void sum_record(int nb, const double* __restrict__ eblk, double* __restrict__ out,
                                           int what) {
    double a = 0.0, b = 0.0, c = 0.0;
    for (int k = threadIdx.x; k < nb; k += kEpiThreads) {
        a += eblk[k * 3 + 0];
        b += eblk[k * 3 + 1];
        c += eblk[k * 3 + 2];
    }
    block_sum3_waves(a, b, c);
    if (threadIdx.x == 0) {
        if (what == REC_UC) {
            out[0] = b;
        } else if (what == REC_UPOT) {
            out[0] = b + c;
        } else {
            out[0] = a;
            out[1] = b;
            out[2] = c;
            out[3] = a + b + c;
        }
    }
}

__global__ void k_zero_u32(unsigned* p) { *p = 0u; }

// T threads per ion (T = 1, 2, 4, 8 or 16; kEpiThreads / T ions per block): with
// T > 1 thread t of an ion sums the t-th contiguous share of the S splits in
// split order and the shares are added in share order through LDS, so that a
// few hundred ions with many splits take T times the CUs and 1/T of the
// dependent loads per thread.  The sum does not depend on timing.
template <int T = 1>
__global__ void __launch_bounds__(kEpiThreads) k_epilogue(EpiParams P) {
    static_assert(T == 1 || T == 2 || T == 4 || T == 8 || T == 16, "threads per ion");
    constexpr int IPB = kEpiThreads / T;  // ions per block
    if (P.eprev && blockIdx.x == gridDim.x - 1) {  // the extra block: an earlier record's sum
        sum_record(P.nprev, P.eprev, P.eprev_out, REC_ALL);
        return;
    }
    const int il = T == 1 ? (int)threadIdx.x : (int)threadIdx.x % IPB;
    const int share = T == 1 ? 0 : (int)threadIdx.x / IPB;
    const int i = blockIdx.x * IPB + il;
    double eK = 0.0, eC = 0.0, eT = 0.0;
    const unsigned mode = P.mode;
    const int n = P.n;
    const bool need_f = (mode & (EPI_FORCES | EPI_ACCEL | EPI_KICK | EPI_GRAD)) != 0;
    const bool need_p = (mode & EPI_ENERGY) && P.ppot != nullptr;
    // the ion's state, requested before the partials so that both round
    // trips overlap (only share 0 of ion i touches it)
    const bool need_s =
        (mode & (EPI_ACCEL | EPI_KICK | EPI_DRIFT | EPI_ENERGY)) && !(mode & (EPI_UC_ONLY | EPI_UPOT | EPI_GRAD));
    const bool own = i < n && share == 0;
    double x = 0.0, y = 0.0, z = 0.0, vx = 0.0, vy = 0.0, vz = 0.0, ax = 0.0, ay = 0.0, az = 0.0, mi = 1.0;
    if (own && need_s) {
        x = P.x[i];
        y = P.y[i];
        z = P.z[i];
        vx = P.vx[i];
        vy = P.vy[i];
        vz = P.vz[i];
        ax = P.ax[i];
        ay = P.ay[i];
        az = P.az[i];
        mi = P.m[i];
    }
    double sx = 0.0, sy = 0.0, sz = 0.0, sp = 0.0;
    {
        int s0 = 0, ns = P.S;  // this thread's splits s0 .. s0 + ns - 1
        if (T > 1) {
            const int len = (P.S + T - 1) / T;
            s0 = min(P.S, share * len);
            ns = min(P.S, s0 + len) - s0;
        }
        const size_t n3 = 3 * (size_t)n;
        if (i < n) {
            if (need_f && need_p) {  // the four arrays' loads together
                const double* ps[4] = {P.part + s0 * n3 + i, P.part + s0 * n3 + n + i,
                                       P.part + s0 * n3 + 2 * (size_t)n + i, P.ppot + (size_t)s0 * n + i};
                const size_t st[4] = {n3, n3, n3, (size_t)n};
                double o[4];
                split_sums<4, 16>(ps, st, ns, o);
                sx = o[0];
                sy = o[1];
                sz = o[2];
                sp = o[3];
            } else if (need_f) {
                const double* ps[3] = {P.part + s0 * n3 + i, P.part + s0 * n3 + n + i,
                                       P.part + s0 * n3 + 2 * (size_t)n + i};
                const size_t st[3] = {n3, n3, n3};
                double o[3];
                split_sums<3, 16>(ps, st, ns, o);
                sx = o[0];
                sy = o[1];
                sz = o[2];
            } else if (need_p) {
                sp = split_sum(P.ppot + (size_t)s0 * n + i, (size_t)n, ns);
            }
        }
        if constexpr (T > 1) {  // the shares in share order
            __shared__ double red[4][T][IPB];
            red[0][share][il] = sx;
            red[1][share][il] = sy;
            red[2][share][il] = sz;
            red[3][share][il] = sp;
            __syncthreads();
            if (share == 0) {
#pragma unroll
                for (int u = 1; u < T; ++u) {
                    sx += red[0][u][il];
                    sy += red[1][u][il];
                    sz += red[2][u][il];
                    sp += red[3][u][il];
                }
            }
        }
    }
    if (own) {
        const double qi = P.q[i];
        const double c = kCoulomb * qi;
        const double cf = (mode & EPI_PRESCALED) ? 1.0 : c;
        // U_C of the ion: half its potential sum times k_C q_i, or its share
        const double cu = (mode & EPI_POT_SHARE) ? kCoulomb : 0.5 * c;
        const double Fx = cf * sx, Fy = cf * sy, Fz = cf * sz;
        bool ok = true;
        if (mode & EPI_FORCES) {
            P.fx[i] = Fx;
            P.fy[i] = Fy;
            P.fz[i] = Fz;
            ok = finite3(Fx, Fy, Fz);
        }
        if (mode & (EPI_GRAD | EPI_UPOT)) {
            // gradient of U_C + U_trap(t0) and/or those two energies: the
            // trap enters only through m (none when m is NULL)
            double xi = 0.0, yi = 0.0, zi = 0.0, mi = 0.0;
            TrapK k{0.0, 0.0, 0.0};
            if (P.m) {
                xi = P.x[i];
                yi = P.y[i];
                zi = P.z[i];
                mi = P.m[i];
                k = trap_k(P.trap, P.t0);
            }
            if (mode & EPI_GRAD) {
                const double gx = __builtin_fma(mi * k.kx, xi, -Fx);
                const double gy = __builtin_fma(mi * k.ky, yi, -Fy);
                const double gz = __builtin_fma(mi * k.kz, zi, -Fz);
                P.fx[i] = gx;
                P.fy[i] = gy;
                P.fz[i] = gz;
                ok = finite3(gx, gy, gz);
            }
            if (mode & EPI_ENERGY) {
                eC = cu * sp;
                eT = 0.5 * mi * (k.kx * xi * xi + k.ky * yi * yi + k.kz * zi * zi);
                ok = ok && __builtin_isfinite(eC) && __builtin_isfinite(eT);
            }
        } else if (mode & EPI_UC_ONLY) {
            eC = cu * sp;
            ok = ok && __builtin_isfinite(eC);
        } else if (mode & (EPI_ACCEL | EPI_KICK | EPI_DRIFT | EPI_ENERGY)) {
            const double t = step_time(P.t0, P.dt, P.step);
            const TrapK k = trap_k(P.trap, t);
            if (mode & (EPI_ACCEL | EPI_KICK)) {
                const double anx = Fx / mi - k.kx * x;
                const double any = Fy / mi - k.ky * y;
                const double anz = Fz / mi - k.kz * z;
                if (mode & EPI_KICK) {
                    const double h = 0.5 * P.dt;
                    if (P.trap.gamma == 0.0) {
                        vx = vx + h * (ax + anx);
                        vy = vy + h * (ay + any);
                        vz = vz + h * (az + anz);
                    } else {  // friction -g v by the trapezoidal rule, g = Gamma / m_i
                        const double g = P.trap.gamma / mi, lo = 1.0 - g * h, hi = 1.0 + g * h;
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
                ok = ok && finite3(ax, ay, az) && finite3(vx, vy, vz);
            }
            if (mode & EPI_ENERGY) {
                eK = 0.5 * mi * (vx * vx + vy * vy + vz * vz);
                eC = cu * sp;
                eT = 0.5 * mi * (k.kx * x * x + k.ky * y * y + k.kz * z * z);
                ok = ok && finite3(eK, eC, eT);
            }
            if (mode & EPI_DRIFT) {
                const double dt = P.dt, h2 = 0.5 * dt * dt;
                if (P.trap.gamma == 0.0) {
                    x = x + vx * dt + h2 * ax;
                    y = y + vy * dt + h2 * ay;
                    z = z + vz * dt + h2 * az;
                } else {  // the drift sees the friction acceleration -g v too
                    const double g = P.trap.gamma / mi;
                    x = x + vx * dt + h2 * (ax - g * vx);
                    y = y + vy * dt + h2 * (ay - g * vy);
                    z = z + vz * dt + h2 * (az - g * vz);
                }
                P.x[i] = x;
                P.y[i] = y;
                P.z[i] = z;
                ok = ok && finite3(x, y, z);
            }
        }
        if (!ok) atomicOr(P.flags, 1u);
    }
    if (mode & EPI_ENERGY) {
        block_sum3_waves(eK, eC, eT);
        if (threadIdx.x == 0) {
            P.eblk[blockIdx.x * 3 + 0] = eK;
            P.eblk[blockIdx.x * 3 + 1] = eC;
            P.eblk[blockIdx.x * 3 + 2] = eT;
        }
        if (P.efinal) {
            __shared__ int last;
            if (threadIdx.x == 0) {
                __threadfence();  // this block's partials before its arrival
                last = atomicAdd(P.ecount, 1u) == gridDim.x - 1;
            }
            __syncthreads();
            if (last) {
                __threadfence();  // every block's partials are visible
                double a = 0.0, b = 0.0, c = 0.0;
                for (int k = threadIdx.x; k < (int)gridDim.x; k += kEpiThreads) {
                    a += P.eblk[k * 3 + 0];
                    b += P.eblk[k * 3 + 1];
                    c += P.eblk[k * 3 + 2];
                }
                block_sum3_waves(a, b, c);
                if (threadIdx.x == 0) {
                    if (mode & EPI_UC_ONLY) {
                        P.efinal[0] = b;
                    } else {
                        P.efinal[0] = a;
                        P.efinal[1] = b;
                        P.efinal[2] = c;
                        P.efinal[3] = a + b + c;
                    }
                    *P.ecount = 0u;
                }
            }
        }
    }
}

// One block: sum_record of nb block partials.
__global__ void __launch_bounds__(kEpiThreads) k_energy_final(int nb, const double* __restrict__ eblk,
                                                             double* __restrict__ out, int what) {
    sum_record(nb, eblk, out, what);
}

}  // namespace cb
