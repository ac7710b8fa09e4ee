// Launch sequence of the Newton's-third-law force stage (tile table, pair
// kernel, finish) for every precision, i-particles-per-lane count and
// reaction-sum variant.
#include <hip/hip_runtime.h>

#include "internal.hpp"
#include "pair_sym.hpp"

namespace cb {

constexpr int kPlanThreads = 1024;

// Tile table, one workgroup (sym_plan_fill in pair_sym.hpp).
__global__ void __launch_bounds__(kPlanThreads) k_sym_plan(int n, int IB, int JL, int W, int nI,
                                                           int* __restrict__ rowstart, int2* __restrict__ tiles) {
    sym_plan_fill<kPlanThreads>(n, IB, JL, W, nI, rowstart, tiles);
}

static size_t al256(size_t b) { return (b + 255) / 256 * 256; }

static int sym_groups(int64_t n, int IB, int W) {
    const int nI = (int)((n + IB - 1) / IB);
    return (nI + W - 1) / W;
}

int64_t sym_tiles(int64_t n, int IB, int JL, int W) {
    const int nG = sym_groups(n, IB, W);
    int64_t T = 0;
    for (int G = 0; G < nG; ++G) T += sym_nseg((int)n, IB, JL, G * W);
    return T;
}

// Workspace carve-up: rowstart[nG+1] | tiles[T] | Pi[T][W][3][IB] |
// R[T][3][JL] (| Et[T][W], the tiles' pair energies, with the energy)
size_t sym_ws_bytes(int64_t n, int p, int jl, bool pot, int W) {
    const int IB = 64 * p;
    const int64_t T = sym_tiles(n, IB, jl, W);
    const size_t TW = (size_t)W * T;
    return sym_plan_bytes(n, IB, jl, W) + al256(sizeof(double) * 3 * IB * (TW + 1)) +
           al256(sizeof(double) * 3 * (size_t)jl * (T + 1)) + (pot ? al256(sizeof(double) * (TW + 1)) : 0);
}

template <int PREC, int P, int RED, bool POT>
static void go_sym(int n, int JL, int64_t T, const double* x, const double* y, const double* z, const double* q,
                   double eps2, const int2* tiles, double* Pi, double* R, double* Et, hipStream_t st) {
    k_pair_sym<PREC, P, RED, POT><<<(unsigned)T, 64, 0, st>>>(n, x, y, z, q, eps2, JL, tiles, Pi, R, Et);
}

template <int PREC, int RED, bool POT>
static bool go_sym_p(int P, int n, int JL, int64_t T, const double* x, const double* y, const double* z,
                     const double* q, double eps2, const int2* tiles, double* Pi, double* R, double* Et,
                     hipStream_t st) {
    switch (P) {
        case 2: go_sym<PREC, 2, RED, POT>(n, JL, T, x, y, z, q, eps2, tiles, Pi, R, Et, st); return true;
        case 3: go_sym<PREC, 3, RED, POT>(n, JL, T, x, y, z, q, eps2, tiles, Pi, R, Et, st); return true;
        case 4: go_sym<PREC, 4, RED, POT>(n, JL, T, x, y, z, q, eps2, tiles, Pi, R, Et, st); return true;
        case 5: go_sym<PREC, 5, RED, POT>(n, JL, T, x, y, z, q, eps2, tiles, Pi, R, Et, st); return true;
        case 6: go_sym<PREC, 6, RED, POT>(n, JL, T, x, y, z, q, eps2, tiles, Pi, R, Et, st); return true;
        case 8: go_sym<PREC, 8, RED, POT>(n, JL, T, x, y, z, q, eps2, tiles, Pi, R, Et, st); return true;
        default: return false;
    }
}

// red: 1 = reactions summed through LDS, 0 = by permutes; the energy's
// variant sums them through LDS.
template <int PREC>
static bool go_sym_pr(int P, int red, bool pot, int n, int JL, int64_t T, const double* x, const double* y,
                      const double* z, const double* q, double eps2, const int2* tiles, double* Pi, double* R,
                      double* Et, hipStream_t st) {
    if (pot) return go_sym_p<PREC, 1, true>(P, n, JL, T, x, y, z, q, eps2, tiles, Pi, R, Et, st);
    return red ? go_sym_p<PREC, 1, false>(P, n, JL, T, x, y, z, q, eps2, tiles, Pi, R, Et, st)
               : go_sym_p<PREC, 0, false>(P, n, JL, T, x, y, z, q, eps2, tiles, Pi, R, Et, st);
}

// The row-group kernel (kSymRows i-blocks per workgroup), for P = 4, 6, 8.
template <int PREC, bool POT>
static bool go_sym_rows(int P, int n, int JL, int64_t T, const double* x, const double* y, const double* z,
                        const double* q, double eps2, const int2* tiles, double* Pi, double* R, double* Et,
                        hipStream_t st) {
    const unsigned g = (unsigned)T, b = 64 * kSymRows;
    switch (P) {
        case 4: k_pair_sym_rows<PREC, 4, POT><<<g, b, 0, st>>>(n, x, y, z, q, eps2, JL, tiles, Pi, R, Et); return true;
        case 6: k_pair_sym_rows<PREC, 6, POT><<<g, b, 0, st>>>(n, x, y, z, q, eps2, JL, tiles, Pi, R, Et); return true;
        case 8: k_pair_sym_rows<PREC, 8, POT><<<g, b, 0, st>>>(n, x, y, z, q, eps2, JL, tiles, Pi, R, Et); return true;
        default: return false;
    }
}

template <int PREC>
static bool go_sym_rows_p(int P, bool pot, int n, int JL, int64_t T, const double* x, const double* y,
                          const double* z, const double* q, double eps2, const int2* tiles, double* Pi, double* R,
                          double* Et, hipStream_t st) {
    return pot ? go_sym_rows<PREC, true>(P, n, JL, T, x, y, z, q, eps2, tiles, Pi, R, Et, st)
               : go_sym_rows<PREC, false>(P, n, JL, T, x, y, z, q, eps2, tiles, Pi, R, Et, st);
}

template <int PREC>
static void go_finish(bool pot, unsigned nb, int n, int IB, int JL, int lgJL, int W, const double* x,
                      const double* y, const double* z, const double* q, double eps2, const int* rowstart,
                      const double* Pi, const double* R, const double* Et, double* F, double* phi, hipStream_t st) {
    if (pot)
        k_sym_finish<PREC, true><<<nb, 64 * kFinishParts, 0, st>>>(n, IB, JL, lgJL, W, x, y, z, q, eps2, rowstart,
                                                                   Pi, R, Et, F, phi);
    else
        k_sym_finish<PREC, false><<<nb, 64 * kFinishParts, 0, st>>>(n, IB, JL, lgJL, W, x, y, z, q, eps2, rowstart,
                                                                    Pi, R, Et, F, phi);
}

size_t sym_plan_bytes(int64_t n, int IB, int JL, int W) {
    const int64_t nG = sym_groups(n, IB, W);
    return al256(sizeof(int) * (nG + 1)) + al256(sizeof(int2) * (sym_tiles(n, IB, JL, W) + 1));
}

cb_status sym_plan(int n, int IB, int JL, void* ws, SymPlan* out, hipStream_t st, int W, bool filled) {
    const int nI = (n + IB - 1) / IB;
    if (nI > kPlanMaxRows) return fail(CB_EINVAL, "sym_plan: n = %d is too large for the symmetric kernels", n);
    const int nG = sym_groups(n, IB, W);
    out->T = sym_tiles(n, IB, JL, W);
    char* base = static_cast<char*>(ws);
    out->rowstart = reinterpret_cast<int*>(base);
    base += al256(sizeof(int) * (nG + 1));
    out->tiles = reinterpret_cast<int2*>(base);
    out->bytes = sym_plan_bytes(n, IB, JL, W);
    if (filled) return CB_OK;
    k_sym_plan<<<1, kPlanThreads, 0, st>>>(n, IB, JL, W, nG, out->rowstart, out->tiles);
    return check_launch("k_sym_plan");
}

cb_status launch_pair_sym(int prec, const LaunchCfg& c, int n, const double* x, const double* y, const double* z,
                          const double* q, double eps2, void* ws, double* F, hipStream_t st, double* phi,
                          bool plan_filled) {
    const int P = c.p, JL = c.splits, IB = 64 * P, W = sym_rows(c.algo);
    if (!is_sym(c.algo) || !sym_cfg_ok(P, c.wg, JL) || (W > 1 && !sym_rows_p_ok(P)))
        return fail(CB_EINVAL, "launch_pair_sym: bad configuration");
    const int red = c.algo == ALGO_SYM ? 0 : 1;
    SymPlan plan;
    cb_status rc = sym_plan(n, IB, JL, ws, &plan, st, W, plan_filled);
    if (rc) return rc;
    const int64_t T = plan.T;
    int* rowstart = plan.rowstart;
    const int2* tiles = plan.tiles;
    const bool pot = phi != nullptr;
    char* base = static_cast<char*>(ws) + plan.bytes;
    double* Pi = reinterpret_cast<double*>(base);
    base += al256(sizeof(double) * 3 * IB * ((size_t)W * T + 1));
    double* R = reinterpret_cast<double*>(base);
    base += al256(sizeof(double) * 3 * (size_t)JL * (T + 1));
    double* Et = pot ? reinterpret_cast<double*>(base) : nullptr;
    if (T > 0 && W > 1) {
        bool okk = false;
        switch (prec) {
            case PREC_FP64: okk = go_sym_rows_p<PREC_FP64>(P, pot, n, JL, T, x, y, z, q, eps2, tiles, Pi, R, Et, st); break;
            case PREC_MIXED: okk = go_sym_rows_p<PREC_MIXED>(P, pot, n, JL, T, x, y, z, q, eps2, tiles, Pi, R, Et, st); break;
            case PREC_IEEE: okk = go_sym_rows_p<PREC_IEEE>(P, pot, n, JL, T, x, y, z, q, eps2, tiles, Pi, R, Et, st); break;
            case PREC_FP32: okk = go_sym_rows_p<PREC_FP32>(P, pot, n, JL, T, x, y, z, q, eps2, tiles, Pi, R, Et, st); break;
            default: break;
        }
        if (!okk) return fail(CB_EINVAL, "launch_pair_sym: unsupported precision %d / p %d", prec, P);
        if ((rc = check_launch("k_pair_sym_rows"))) return rc;
    } else if (T > 0) {
        bool okk = false;
        switch (prec) {
            case PREC_FP64: okk = go_sym_pr<PREC_FP64>(P, red, pot, n, JL, T, x, y, z, q, eps2, tiles, Pi, R, Et, st); break;
            case PREC_MIXED: okk = go_sym_pr<PREC_MIXED>(P, red, pot, n, JL, T, x, y, z, q, eps2, tiles, Pi, R, Et, st); break;
            case PREC_IEEE: okk = go_sym_pr<PREC_IEEE>(P, red, pot, n, JL, T, x, y, z, q, eps2, tiles, Pi, R, Et, st); break;
            case PREC_FP32: okk = go_sym_pr<PREC_FP32>(P, red, pot, n, JL, T, x, y, z, q, eps2, tiles, Pi, R, Et, st); break;
            default: break;
        }
        if (!okk) return fail(CB_EINVAL, "launch_pair_sym: unsupported precision %d / p %d", prec, P);
        if ((rc = check_launch("k_pair_sym"))) return rc;
    }
    const unsigned nb = (unsigned)((n + 63) / 64);
    int lgJL = 0;
    while ((1 << lgJL) < JL) ++lgJL;
    switch (prec) {
        case PREC_FP64: go_finish<PREC_FP64>(pot, nb, n, IB, JL, lgJL, W, x, y, z, q, eps2, rowstart, Pi, R, Et, F, phi, st); break;
        case PREC_MIXED: go_finish<PREC_MIXED>(pot, nb, n, IB, JL, lgJL, W, x, y, z, q, eps2, rowstart, Pi, R, Et, F, phi, st); break;
        case PREC_IEEE: go_finish<PREC_IEEE>(pot, nb, n, IB, JL, lgJL, W, x, y, z, q, eps2, rowstart, Pi, R, Et, F, phi, st); break;
        default: go_finish<PREC_FP32>(pot, nb, n, IB, JL, lgJL, W, x, y, z, q, eps2, rowstart, Pi, R, Et, F, phi, st); break;
    }
    return check_launch("k_sym_finish");
}

}  // namespace cb
