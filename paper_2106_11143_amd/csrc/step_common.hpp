// Device helpers shared by the element-wise kernels: physical constants, trap
// spring constants (paper, section 2, eq. (1)), step times and fixed-order
// block sums.
#pragma once
#include <hip/hip_runtime.h>

#include "coulomb.h"

namespace cb {

// k_C = 1 / (4 pi eps0), CODATA 2018 vacuum permittivity.
constexpr double kPi = 3.14159265358979323846;
constexpr double kEps0 = 8.8541878128e-12;
constexpr double kCoulomb = 1.0 / (4.0 * kPi * kEps0);

constexpr int kEpiThreads = 256;

// What one element-wise launch does per ion.
enum : unsigned {
    EPI_FORCES = 1u,   // write F to fx, fy, fz
    EPI_ACCEL = 2u,    // a <- F/m + trap (initial acceleration)
    EPI_KICK = 4u,     // a_new = F/m + trap; v += dt/2 (a + a_new); a <- a_new
    EPI_DRIFT = 8u,    // r += v dt + a dt^2/2 (after any kick)
    EPI_ENERGY = 16u,  // per-block sums of K, U_C, U_trap of the resulting state
    EPI_UC_ONLY = 32u,    // energy: only U_C (no m, v, trap)
    EPI_PRESCALED = 64u,  // part holds finished forces [3][n] (S = 1), not sums to scale by k_C q_i
    EPI_GRAD = 128u,      // write g = -F + m k(t0) r (m NULL: -F) to fx, fy, fz
    EPI_UPOT = 256u,      // energy: U_C and U_trap(t0) only (no velocities; U_trap = 0 when m is NULL)
    EPI_POT_SHARE = 512u  // the potential partials hold energy shares (U_C = k_C sum), S = 1
};

// What sum_record writes: the whole record, U_C alone, or U_C + U_trap alone.
enum : int { REC_ALL = 0, REC_UC = 1, REC_UPOT = 2 };

struct TrapK {
    double kx, ky, kz;
};

// Spring constants per unit mass of the trap at time t (see cb_trap): the
// pseudo-potential's (wx^2, wy^2, wz^2), linearly ramped in (wx, wy); or the
// RF drive of eq. (1) in Mathieu form.  Host and device use this one
// function (cb_trap_k exports the host side).
__host__ __device__ __forceinline__ TrapK trap_k(const cb_trap& tr, double t) {
    TrapK k;
    if (tr.kind == 1) {
        const double w2 = tr.rf_omega * tr.rf_omega;
        const double kx = tr.rf_a * w2 * 0.25 + tr.rf_q * w2 * 0.5 * cos(tr.rf_omega * t + tr.rf_phase);
        k.kx = kx;
        k.ky = -kx;
        k.kz = tr.wz * tr.wz;
        return k;
    }
    double wx = tr.wx, wy = tr.wy;
    if (tr.t_ramp1 > tr.t_ramp0) {
        double s = (t - tr.t_ramp0) / (tr.t_ramp1 - tr.t_ramp0);
        s = fmin(fmax(s, 0.0), 1.0);
        wx = tr.wx + s * (tr.wx1 - tr.wx);
        wy = tr.wy + s * (tr.wy1 - tr.wy);
    }
    k.kx = wx * wx;
    k.ky = wy * wy;
    k.kz = tr.wz * tr.wz;
    return k;
}

// Time of step `step` of a run started at t0 (one rounding per operation,
// never contracted, so every kernel computes the same value).
__device__ __forceinline__ double step_time(double t0, double dt, long long step) {
    return __dadd_rn(t0, __dmul_rn(static_cast<double>(step), dt));
}

// Fixed-order tree sum of three values over the 256 threads of a block; the
// result is valid in thread 0.
__device__ __forceinline__ void block_sum3(double& a, double& b, double& c) {
    __shared__ double sh[3][kEpiThreads];
    const int t = threadIdx.x;
    sh[0][t] = a;
    sh[1][t] = b;
    sh[2][t] = c;
    __syncthreads();
    for (int w = kEpiThreads / 2; w > 0; w >>= 1) {
        if (t < w) {
            sh[0][t] += sh[0][t + w];
            sh[1][t] += sh[1][t + w];
            sh[2][t] += sh[2][t + w];
        }
        __syncthreads();
    }
    a = sh[0][0];
    b = sh[1][0];
    c = sh[2][0];
}

__device__ __forceinline__ bool finite3(double a, double b, double c) {
    return __builtin_isfinite(a) && __builtin_isfinite(b) && __builtin_isfinite(c);
}

}  // namespace cb
