// Instantiation and launch of the all-pairs kernels for every precision,
// i-particles-per-lane count and output kind.
#include <hip/hip_runtime.h>

#include "internal.hpp"
#include "pair_kernels.hpp"

namespace cb {

template <int PREC, int P, bool FORCE, bool POT>
static void go(dim3 grid, dim3 block, hipStream_t st, int n, const double* x, const double* y, const double* z,
               const double* q, double eps2, int jlen, double* part, double* ppot) {
    k_pair<PREC, P, FORCE, POT><<<grid, block, 0, st>>>(n, x, y, z, q, eps2, jlen, part, ppot);
}

template <int PREC, int P>
static bool go_kind(bool force, bool pot, dim3 g, dim3 b, hipStream_t st, int n, const double* x,
                    const double* y, const double* z, const double* q, double eps2, int jlen, double* part,
                    double* ppot) {
    if (force && pot) go<PREC, P, true, true>(g, b, st, n, x, y, z, q, eps2, jlen, part, ppot);
    else if (force) go<PREC, P, true, false>(g, b, st, n, x, y, z, q, eps2, jlen, part, ppot);
    else if (pot) go<PREC, P, false, true>(g, b, st, n, x, y, z, q, eps2, jlen, part, ppot);
    else return false;
    return true;
}

template <int PREC>
static bool go_p(int p, bool force, bool pot, dim3 g, dim3 b, hipStream_t st, int n, const double* x,
                 const double* y, const double* z, const double* q, double eps2, int jlen, double* part,
                 double* ppot) {
    switch (p) {
        case 1: return go_kind<PREC, 1>(force, pot, g, b, st, n, x, y, z, q, eps2, jlen, part, ppot);
        case 2: return go_kind<PREC, 2>(force, pot, g, b, st, n, x, y, z, q, eps2, jlen, part, ppot);
        case 4: return go_kind<PREC, 4>(force, pot, g, b, st, n, x, y, z, q, eps2, jlen, part, ppot);
        default: return false;
    }
}

cb_status launch_pair(int prec, const LaunchCfg& c, bool force, bool pot, int n, const double* x,
                      const double* y, const double* z, const double* q, double eps2, int jlen, double* part,
                      double* ppot, hipStream_t st) {
    const int S = n_splits(n, jlen);
    const int ipb = 64 * c.p * (c.wg / 64);  // i-particles per workgroup
    dim3 grid((n + ipb - 1) / ipb, S);
    dim3 block(c.wg);
    bool okk = false;
    switch (prec) {
        case PREC_FP64: okk = go_p<PREC_FP64>(c.p, force, pot, grid, block, st, n, x, y, z, q, eps2, jlen, part, ppot); break;
        case PREC_MIXED: okk = go_p<PREC_MIXED>(c.p, force, pot, grid, block, st, n, x, y, z, q, eps2, jlen, part, ppot); break;
        case PREC_IEEE: okk = go_p<PREC_IEEE>(c.p, force, pot, grid, block, st, n, x, y, z, q, eps2, jlen, part, ppot); break;
        case PREC_FP32: okk = go_p<PREC_FP32>(c.p, force, pot, grid, block, st, n, x, y, z, q, eps2, jlen, part, ppot); break;
        default: break;
    }
    if (!okk) return fail(CB_EINVAL, "launch_pair: unsupported precision %d / p %d", prec, c.p);
    return check_launch("k_pair");
}

}  // namespace cb
