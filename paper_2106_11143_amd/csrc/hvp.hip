// Hessian-vector products and the adjoint velocity-Verlet step.
#include <hip/hip_runtime.h>

#include "internal.hpp"

using namespace cb;

extern "C" {

cb_status coulomb_hvp(int64_t n, const double* x, const double* y, const double* z, const double* q, int32_t nvec,
                      const double* v, double* hv, const double* m, const cb_trap* trap, double t, double eps2,
                      int32_t prec, void* ws, size_t ws_bytes, void* stream) {
    (void)n; (void)x; (void)y; (void)z; (void)q; (void)nvec; (void)v; (void)hv; (void)m; (void)trap; (void)t;
    (void)eps2; (void)prec; (void)ws; (void)ws_bytes; (void)stream;
    return fail(CB_EUNSUPPORTED, "coulomb_hvp: not built yet");
}

cb_status md_adjoint_step(int64_t n, const double* x, const double* y, const double* z, const double* q,
                          const double* m, const cb_trap* trap, double dt, double eps2, int32_t prec, uint32_t flags,
                          double* lam, double* dldw, void* ws, size_t ws_bytes, void* stream) {
    (void)n; (void)x; (void)y; (void)z; (void)q; (void)m; (void)trap; (void)dt; (void)eps2; (void)prec; (void)flags;
    (void)lam; (void)dldw; (void)ws; (void)ws_bytes; (void)stream;
    return fail(CB_EUNSUPPORTED, "md_adjoint_step: not built yet");
}

}  // extern "C"
