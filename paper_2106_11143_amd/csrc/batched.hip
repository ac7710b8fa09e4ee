// Batched persistent velocity-Verlet kernel (one workgroup per run).
#include <hip/hip_runtime.h>

#include "internal.hpp"

namespace cb {

cb_status md_run_batched(int32_t nrun, const int64_t* offsets, const cb_state* s, const double* q,
                         const double* m, const cb_trap* traps, double t0, double dt, int64_t nsteps,
                         double eps2, int32_t prec, uint32_t flags, double* energies, int64_t every, void* ws,
                         size_t ws_bytes, hipStream_t st) {
    (void)nrun; (void)offsets; (void)s; (void)q; (void)m; (void)traps; (void)t0; (void)dt; (void)nsteps;
    (void)eps2; (void)prec; (void)flags; (void)energies; (void)every; (void)ws; (void)ws_bytes; (void)st;
    return fail(CB_EUNSUPPORTED, "md_run: batched runs are not built yet");
}

}  // namespace cb
