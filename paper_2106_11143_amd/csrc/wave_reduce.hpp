// Wave-wide reduce-scatter of 12 doubles per lane on gfx950 (wave64), two
// ways: through cross-lane permutes and DPP (reduce_scatter12), or through LDS
// (lds_reduce12, for workgroups of one wave).
#pragma once
#include <hip/hip_runtime.h>

namespace cb {

__device__ __forceinline__ double pack_d(unsigned lo, unsigned hi) {
    return __builtin_bit_cast(double, (static_cast<unsigned long long>(hi) << 32) | lo);
}
__device__ __forceinline__ unsigned lo_u(double d) {
    return static_cast<unsigned>(__builtin_bit_cast(unsigned long long, d));
}
__device__ __forceinline__ unsigned hi_u(double d) {
    return static_cast<unsigned>(__builtin_bit_cast(unsigned long long, d) >> 32);
}

// lanes 0-31 return a(l) + a(l+32); lanes 32-63 return b(l-32) + b(l).
__device__ __forceinline__ double swap32_add(double a, double b) {
    const auto lo = __builtin_amdgcn_permlane32_swap(lo_u(a), lo_u(b), false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap(hi_u(a), hi_u(b), false, false);
    return pack_d(lo[0], hi[0]) + pack_d(lo[1], hi[1]);
}

// rows 0 and 2 return a(l) + a(l+16); rows 1 and 3 return b(l-16) + b(l).
__device__ __forceinline__ double swap16_add(double a, double b) {
    const auto lo = __builtin_amdgcn_permlane16_swap(lo_u(a), lo_u(b), false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap(hi_u(a), hi_u(b), false, false);
    return pack_d(lo[0], hi[0]) + pack_d(lo[1], hi[1]);
}

template <int CTRL>
__device__ __forceinline__ double dpp_d(double x) {
    const unsigned lo = __builtin_amdgcn_mov_dpp(static_cast<int>(lo_u(x)), CTRL, 0xf, 0xf, false);
    const unsigned hi = __builtin_amdgcn_mov_dpp(static_cast<int>(hi_u(x)), CTRL, 0xf, 0xf, false);
    return pack_d(lo, hi);
}

constexpr int kDppRowRor8 = 0x128;
constexpr int kDppRowHalfMirror = 0x141;
constexpr int kDppQuadXor2 = 0x4E;  // quad_perm [2,3,0,1]
constexpr int kDppQuadXor1 = 0xB1;  // quad_perm [1,0,3,2]

// Input: every lane holds v[jj*3 + c] for jj < 4, c < 3.  Output: every lane
// of the 16-lane group g = lane >> 4 holds in out[c] the sum over all 64
// lanes of v[g*3 + c].  Two halving steps, each exchanging with a partner
// lane and keeping half of the remaining values:
//   lanes 0-31 / 32-63   v_permlane32_swap (keep indices 0-5 / 6-11)
//   rows 0,2 / rows 1,3  v_permlane16_swap (keep 0-2 / 3-5 of those)
// then an all-reduce of the 3 survivors over the 16 lanes of the group (DPP
// row_ror:8, row_half_mirror, quad_perm [2,3,0,1], quad_perm [1,0,3,2]).
// The swaps move 32-bit halves, so each 64-bit value takes two swaps.  All
// lanes of a group end with the same sum up to the order of the last
// additions; callers store it from one lane.
__device__ __forceinline__ void reduce_scatter12(const double (&v)[12], double (&out)[3]) {
    double u[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) u[k] = swap32_add(v[k], v[k + 6]);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        double x = swap16_add(u[c], u[c + 3]);
        x += dpp_d<kDppRowRor8>(x);
        x += dpp_d<kDppRowHalfMirror>(x);
        x += dpp_d<kDppQuadXor2>(x);
        x += dpp_d<kDppQuadXor1>(x);
        out[c] = x;
    }
}

// The same sums through LDS, for a workgroup of one wave.  Every lane writes
// its NV (12 or 16) values value-major into red: row k of kRedStride doubles
// holds value k of lanes 0-63, each run of 16 lanes followed by 2 doubles of
// padding.  Lane L then reads value vi = min(L / 4, NV - 1) of lanes
// 16 g .. 16 g + 15 (g = L % 4, one contiguous run) as eight 16-byte loads,
// adds them in a fixed tree, and the four lanes of each quad add their
// partial sums by DPP.  The result, the sum over all 64 lanes of value vi, is
// returned in every lane of quad vi (with 12 values lanes 48-63 repeat value
// 11).  The padding puts the four runs a quad reads 144 bytes apart (distinct
// banks) and the row stride of 576 bytes puts neighbouring quads' rows half a
// bank cycle apart, so the loads are free of bank conflicts.
// One wave's LDS instructions are performed in issue order, so the reads see
// the writes and the next call's writes follow these reads without a
// barrier; the wavefront-scope fences only keep the compiler from moving the
// accesses across each other.  red holds NV kRedStride doubles, 16-byte
// aligned, and is used by one wave only.
constexpr int kRedStride = 72;

template <int NV>
__device__ __forceinline__ double lds_reduce(const double (&v)[NV], double* __restrict__ red) {
    static_assert(NV == 12 || NV == 16, "12 or 16 values per lane");
    const int lane = __lane_id();
    const int wpos = lane + 2 * (lane >> 4);
#pragma unroll
    for (int k = 0; k < NV; ++k) red[k * kRedStride + wpos] = v[k];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int vi = min(lane >> 2, NV - 1);
    const double2* src = reinterpret_cast<const double2*>(red + vi * kRedStride + (lane & 3) * 18);
    double2 a[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) a[k] = src[k];
    double s4[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) s4[k] = (a[2 * k].x + a[2 * k].y) + (a[2 * k + 1].x + a[2 * k + 1].y);
    double x = (s4[0] + s4[1]) + (s4[2] + s4[3]);
    x += dpp_d<kDppQuadXor1>(x);
    x += dpp_d<kDppQuadXor2>(x);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");  // these reads before the next call's writes
    return x;
}

__device__ __forceinline__ double lds_reduce12(const double (&v)[12], double* __restrict__ red) {
    return lds_reduce<12>(v, red);
}

// lds_reduce<12> in two halves, for a loop that evaluates the next j while
// one j's sums are in flight: lds_put12 writes the values and requests this
// lane's eight loads into a; lds_sum12 (after independent work) adds them.
// The next lds_put12 on the same buffer follows the reads in the wave's
// issue order, so one buffer serves every round.
__device__ __forceinline__ void lds_put12(const double (&v)[12], double* __restrict__ red, double2 (&a)[8]) {
    const int lane = __lane_id();
    const int wpos = lane + 2 * (lane >> 4);
#pragma unroll
    for (int k = 0; k < 12; ++k) red[k * kRedStride + wpos] = v[k];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int vi = min(lane >> 2, 11);
    const double2* src = reinterpret_cast<const double2*>(red + vi * kRedStride + (lane & 3) * 18);
#pragma unroll
    for (int k = 0; k < 8; ++k) a[k] = src[k];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");  // these reads before the next round's writes
}

__device__ __forceinline__ double lds_sum12(const double2 (&a)[8]) {
    double s4[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) s4[k] = (a[2 * k].x + a[2 * k].y) + (a[2 * k + 1].x + a[2 * k + 1].y);
    double x = (s4[0] + s4[1]) + (s4[2] + s4[3]);
    x += dpp_d<kDppQuadXor1>(x);
    x += dpp_d<kDppQuadXor2>(x);
    return x;
}

}  // namespace cb
