// Instantiation and launch of the direct all-pairs kernel for every
// precision, i-particles-per-lane count and output kind.
#include <hip/hip_runtime.h>

#include "internal.hpp"
#include "pair_kernels.hpp"

namespace cb {

struct PairArgs {
    int n, i0, ni;
    const double *x, *y, *z, *q;
    double eps2;
    int jlen;
    double *part, *ppot;
};

template <int PREC, int P, bool FORCE, bool POT>
static void go(dim3 grid, dim3 block, hipStream_t st, const PairArgs& a) {
    k_pair<PREC, P, FORCE, POT><<<grid, block, 0, st>>>(a.n, a.i0, a.ni, a.x, a.y, a.z, a.q, a.eps2, a.jlen, a.part,
                                                        a.ppot);
}

template <int PREC, int P>
static bool go_kind(bool force, bool pot, dim3 g, dim3 b, hipStream_t st, const PairArgs& a) {
    if (force && pot) go<PREC, P, true, true>(g, b, st, a);
    else if (force) go<PREC, P, true, false>(g, b, st, a);
    else if (pot) go<PREC, P, false, true>(g, b, st, a);
    else return false;
    return true;
}

template <int PREC>
static bool go_p(int p, bool force, bool pot, dim3 g, dim3 b, hipStream_t st, const PairArgs& a) {
    switch (p) {
        case 1: return go_kind<PREC, 1>(force, pot, g, b, st, a);
        case 2: return go_kind<PREC, 2>(force, pot, g, b, st, a);
        case 4: return go_kind<PREC, 4>(force, pot, g, b, st, a);
        default: return false;
    }
}

cb_status launch_pair_range(int prec, const LaunchCfg& c, bool force, bool pot, int n, int i0, int ni,
                            const double* x, const double* y, const double* z, const double* q, double eps2,
                            int jlen, double* part, double* ppot, hipStream_t st) {
    if (i0 < 0 || ni < 1 || i0 + ni > n) return fail(CB_EINVAL, "launch_pair: bad i-range");
    const int S = n_splits(n, jlen);
    const int ipb = 64 * c.p * (c.wg / 64);  // i-particles per workgroup
    dim3 grid((ni + ipb - 1) / ipb, S);
    dim3 block(c.wg);
    const PairArgs a{n, i0, ni, x, y, z, q, eps2, jlen, part, ppot};
    bool okk = false;
    switch (prec) {
        case PREC_FP64: okk = go_p<PREC_FP64>(c.p, force, pot, grid, block, st, a); break;
        case PREC_MIXED: okk = go_p<PREC_MIXED>(c.p, force, pot, grid, block, st, a); break;
        case PREC_IEEE: okk = go_p<PREC_IEEE>(c.p, force, pot, grid, block, st, a); break;
        case PREC_FP32: okk = go_p<PREC_FP32>(c.p, force, pot, grid, block, st, a); break;
        case PREC_F32D: okk = force && !pot && go_p<PREC_F32D>(c.p, force, pot, grid, block, st, a); break;
        default: break;
    }
    if (!okk) return fail(CB_EINVAL, "launch_pair: unsupported precision %d / p %d", prec, c.p);
    return check_launch("k_pair");
}

cb_status launch_pair(int prec, const LaunchCfg& c, bool force, bool pot, int n, const double* x,
                      const double* y, const double* z, const double* q, double eps2, int jlen, double* part,
                      double* ppot, hipStream_t st) {
    return launch_pair_range(prec, c, force, pot, n, 0, n, x, y, z, q, eps2, jlen, part, ppot, st);
}

}  // namespace cb
