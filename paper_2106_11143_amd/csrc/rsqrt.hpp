// Inverse-square-root arithmetic of the pair loop (device code, gfx950).
//
// The paper (sections 2 and 4) finds 1/sqrt(r^2) to be the single largest
// cost of the pair interaction and replaces SQRT+DIV by a hardware estimate
// refined with Newton-Raphson steps, each doubling the correct bits.  On
// gfx950 the cheapest estimate is v_rsq_f32 (about 2^-23 relative error; it
// overlaps with FP64 VALU work, whereas v_rsq_f64 is no more accurate and runs
// at quarter rate), so every fast variant starts from the FP32 estimate y0 of
// the FP32-rounded r^2 and refines in FP64.
//
// The force needs s = q r^{-3}, not r^{-1}, so the refinement is applied to s
// directly.  With t = y0^2 (exact in FP64: y0 has 24 significant bits) and
// e = 1 - r^2 t (one FMA, rounded once),
//   r^{-3} = y0^3 (1 - e)^{-3/2} = y0^3 (1 + 3/2 e + 15/8 e^2 + O(e^3)).
// Keeping the e term is one Newton-Raphson step for the root of
// s^{-2/3} = r^2 (s1 = s0 (1 + 3/2 e)); keeping e^2 as well is the next
// (Householder) order.  With |e| <= 2^-22 the first leaves a relative error
// of about 2 e^2 (~1e-13) and the second about 2 e^3 (below double rounding).
// The potential uses the same e:  r^{-1} = y0 (1 + e/2 + 3/8 e^2 + O(e^3)).
#pragma once
#include <hip/hip_runtime.h>

namespace cb {

// PREC_F32D: the mixed refinement on displacements rounded to FP32 (an
// ablation; the rounding happens where the displacement is formed).
enum : int { PREC_FP64 = 0, PREC_MIXED = 1, PREC_IEEE = 2, PREC_FP32 = 3, PREC_F32D = 4 };

__device__ __forceinline__ double rsq_seed(double r2) {
    return static_cast<double>(__builtin_amdgcn_rsqf(static_cast<float>(r2)));
}

// Series coefficients held in VGPRs for the whole kernel: gfx950 has no
// 64-bit literal operand and reads at most one SGPR per VALU instruction, so
// without this the compiler re-materialises fma(e, 15/8, 3/2)'s constants
// with two v_mov_b32 per pair.  The empty asm makes them opaque values.
struct SeriesK {
    double c15, c1875, c0375;
    __device__ __forceinline__ SeriesK() : c15(1.5), c1875(1.875), c0375(0.375) {
        asm volatile("" : "+v"(c15), "+v"(c1875), "+v"(c0375));
    }
};

// s = q (r^2)^{-3/2} when FORCE, y = (r^2)^{-1/2} when POT.
template <int PREC, bool FORCE, bool POT>
__device__ __forceinline__ void inv_r(double r2, double q, const SeriesK& K, double& s, double& y) {
    if (PREC == PREC_IEEE) {
        // SQRT+DIV: correctly rounded square root, then correctly rounded division.
        const double r = 1.0 / __builtin_sqrt(r2);
        if (FORCE) s = r * r * r * q;
        if (POT) y = r;
    } else if (PREC == PREC_FP32) {
        const double y0 = rsq_seed(r2);
        if (FORCE) s = y0 * y0 * (y0 * q);
        if (POT) y = y0;
    } else {
        const double y0 = rsq_seed(r2);
        const double t = y0 * y0;
        const double e = __builtin_fma(-r2, t, 1.0);
        if (FORCE) {
            const double w = (y0 * q) * t;
            if (PREC == PREC_FP64) {
                const double p = __builtin_fma(e, K.c1875, K.c15);
                s = __builtin_fma(w, e * p, w);
            } else {
                s = __builtin_fma(w, K.c15 * e, w);
            }
        }
        if (POT) {
            const double ye = y0 * e;
            if (PREC == PREC_FP64) {
                const double p = __builtin_fma(e, K.c0375, 0.5);
                y = __builtin_fma(ye, p, y0);
            } else {
                y = __builtin_fma(ye, 0.5, y0);
            }
        }
    }
}

}  // namespace cb
