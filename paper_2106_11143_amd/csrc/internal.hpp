// Host-side declarations shared by the translation units of the library.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <cstring>

#include "coulomb.h"

namespace cb {

constexpr int kMaxSplits = 64;       // j-splits per launch
constexpr int kMaxVec = 8;           // HVP vectors per call
constexpr int kMaxBatchIons = 4096;  // ions per run in the batched kernel (LDS bound)
constexpr int kBatchGridMax = 2048;  // workgroups of one batched launch (force accumulator slots)
constexpr int kBatchWG = 512;        // threads per workgroup of the persistent batched kernel
constexpr int kBatchP = 4;           // ions per thread and register group in that kernel
constexpr int kEpiBlock = 256;       // threads per element-wise block
constexpr int kEpiMinIons = kEpiBlock / 16;  // ions per block of the widest epilogue (16 threads per ion)
// Threads per ion of the epilogue (k_epilogue<T>) of the all-pairs kernel's
// calls (forces, energy, gradient, md_step, md_run): in a run of at most
// 8192 ions whose pair launch leaves 16 or more j-split partials per ion, 8
// or 16 threads share each ion's sums, over 8 or 16 times the CUs (md_run
// with energies every step on MI355X: 1024 ions 14.5 -> 11.0 us per step,
// 2048 17.4 -> 14.3, 4096 28.5 -> 24.9, with 64 splits).
constexpr int epi_parts(int64_t n, int S) { return n > 8192 ? 1 : (S >= 32 ? 16 : (S >= 16 ? 8 : 1)); }
constexpr int64_t kMaxIons = int64_t(1) << 28;  // largest n any entry point accepts
constexpr int64_t kSymMaxN = int64_t(1) << 18;  // largest n for the symmetric kernel (partials grow as n^2)
constexpr int kMaxDevices = 64;      // GPUs per process the per-device symbol tables hold

// ALGO_SYM and ALGO_SYM_LDS differ only in how the per-j reactions are summed
// over the wave (cross-lane permutes and DPP, or LDS).  ALGO_SYM_ROWS: as
// ALGO_SYM_LDS with kSymRows consecutive i-blocks per workgroup sharing each
// j-segment, their reactions added in LDS before one store.
// ALGO_SMALL (md_step / md_run of one run of at most kSmallRunMax ions):
// one launch per step, every pair direct (md_run_small).
enum : int { ALGO_DIRECT = 0, ALGO_SYM = 1, ALGO_SYM_LDS = 2, ALGO_SMALL = 3, ALGO_SYM_ROWS = 4 };

constexpr bool is_sym(int algo) { return algo == ALGO_SYM || algo == ALGO_SYM_LDS || algo == ALGO_SYM_ROWS; }

// i-blocks per workgroup of the row-group variant, and of the others.
constexpr int kSymRows = 4;
constexpr int sym_rows(int algo) { return algo == ALGO_SYM_ROWS ? kSymRows : 1; }
constexpr bool sym_rows_p_ok(int p) { return p == 4 || p == 6 || p == 8; }
constexpr int64_t kSymRowsMinN = 81920;  // the row-group tiles are the default from here

// Operations whose pair stage may take the Newton's-third-law kernels.
constexpr bool sym_op(int op) {
    return op == CB_OP_FORCES || op == CB_OP_ENERGY || op == CB_OP_MD_STEP || op == CB_OP_MD_RUN;
}

// Symmetric path launch parameters: i-particles per lane, j's per reaction
// group, segment lengths (powers of two).
constexpr int kSymP[] = {2, 3, 4, 5, 6, 8};
constexpr int kSymGroup = 4;
constexpr int kSymJL[] = {256, 512, 1024, 2048};

// Newton's-third-law Hessian-vector products (hvp.hip): i-particles per
// lane, segment lengths, the smallest n of the default, the largest n a
// tile table holds, and the workspace of the configuration.
constexpr int kHvpSymP[] = {1, 2, 4};
constexpr int kHvpSymJL[] = {64, 128, 256, 512};
constexpr int64_t kHvpSymMinN = 4096;
constexpr bool hvp_sym_cfg_ok(int p, int jl) {
    bool pk = false, jk = false;
    for (int v : kHvpSymP) pk = pk || v == p;
    for (int v : kHvpSymJL) jk = jk || v == jl;
    return pk && jk;
}
constexpr int64_t hvp_sym_max_n(int p) { return int64_t(2048) * 64 * p; }
// Passes of nvmax vectors that one launch evaluates together (more waves in
// flight than one pass of a small problem gives), and the passes a
// workspace for nvec vectors holds.
constexpr int kHvpSymPasses = 2;
constexpr int hvp_sym_passes(int nvec, int nvmax) {
    return nvec / nvmax < 1 ? 1 : (nvec / nvmax > kHvpSymPasses ? kHvpSymPasses : nvec / nvmax);
}
size_t hvp_sym_ws_bytes(int64_t n, int p, int jl, int npass);

constexpr bool sym_cfg_ok(int p, int g, int jl) {
    bool pk = false, jk = false;
    for (int v : kSymP) pk = pk || v == p;
    for (int v : kSymJL) jk = jk || v == jl;
    return pk && jk && g == kSymGroup;
}

struct LaunchCfg {
    int p;       // i-particles per lane
    int wg;      // direct: threads per workgroup; symmetric: j's per reaction group (4)
    int splits;  // direct: requested j-splits; symmetric: segment length JL
    int tuned;   // 1 if set by tuning or cb_set_config
    int algo;    // ALGO_DIRECT, ALGO_SYM or ALGO_SYM_LDS
};

struct WsLayout {
    size_t part, ppot, eblk, aux, batch, total;
};

cb_status fail(cb_status st, const char* fmt, ...);
cb_status ok();
cb_status check_launch(const char* what);
unsigned* flags_ptr();

// Host-to-device copies of tables a call builds on the host (run tables,
// traps).  On a stream that is not capturing, each copy reads its source
// directly (HIP consumes pageable sources before hipMemcpyAsync returns).
// On a capturing stream the sources are first copied into one host block
// that the graph under construction owns (a user object the graph retains,
// freed after the graph is destroyed), so every replay copies the same
// bytes again.  Sources must stay valid until run() returns.
class HostUpload {
  public:
    void add(void* dst, const void* src, size_t bytes);
    cb_status run(hipStream_t st, const char* what);

  private:
    struct Item {
        void* dst;
        const void* src;
        size_t bytes;
    };
    Item items_[8];
    int count_ = 0;
};

int n_bucket(int64_t n);
LaunchCfg default_cfg(int op, int64_t n, int prec);
LaunchCfg direct_cfg(int op, int64_t n, int prec);
LaunchCfg get_cfg(int op, int64_t n, int prec);
void put_cfg(int op, int64_t n, int prec, LaunchCfg c);
void drop_cfg(int op, int64_t n, int prec);
bool valid_cfg(int op, const LaunchCfg& c);
int split_len(int64_t n, int splits);
int n_splits(int64_t n, int jlen);
// Workspace carve-up of an entry point; sized for the launch configuration
// get_cfg picks for (op, n, prec) at the time of the call.
WsLayout ws_layout(int op, int64_t n, int32_t nrun, int32_t nvec, int32_t prec);

bool trap_ok(const cb_trap* t, const char* who, cb_status* st);

// Tile table of the Newton's-third-law kernels (pair_sym.hip): row groups of
// W consecutive i-blocks of IB ions (W = 1: single rows), the j's above the
// group's first block cut into j-segments of JL.  sym_plan carves
// rowstart[nG+1] and tiles[T] (tile = (group, segment)) from the start of ws
// (sym_plan_bytes of it) and enqueues the kernel that fills them (unless
// filled: the same table is already in ws, written by an earlier call on the
// stream with the same n, IB, JL and W).
struct SymPlan {
    int* rowstart;
    int2* tiles;
    int64_t T;
    size_t bytes;
};
int64_t sym_tiles(int64_t n, int IB, int JL, int W = 1);
size_t sym_plan_bytes(int64_t n, int IB, int JL, int W = 1);
cb_status sym_plan(int n, int IB, int JL, void* ws, SymPlan* out, hipStream_t st, int W = 1, bool filled = false);

// Symmetric (Newton's third law) force path (pair_sym.hip): workspace bytes
// for (n, p, JL) and W rows per workgroup (pot: with the tiles' pair
// energies), and the launch sequence ending with finished forces F[3][n]
// and, when phi is set, each ion's share of the Coulomb energy, U_C = k_C
// sum_k phi[k].  plan_filled: ws already holds the tile table of (n, c), from
// an earlier launch on the stream (md_run's later steps).
size_t sym_ws_bytes(int64_t n, int p, int jl, bool pot = false, int W = 1);
cb_status launch_pair_sym(int prec, const LaunchCfg& c, int n, const double* x, const double* y, const double* z,
                          const double* q, double eps2, void* ws, double* F, hipStream_t st, double* phi = nullptr,
                          bool plan_filled = false);

// Launches of the pair kernels (pair.hip).  The _range form evaluates the
// forces / potentials of the ions i0 .. i0 + ni - 1 only (partials indexed by
// i - i0); launch_pair is the whole range.
cb_status launch_pair_range(int prec, const LaunchCfg& c, bool force, bool pot, int n, int i0, int ni,
                            const double* x, const double* y, const double* z, const double* q, double eps2,
                            int jlen, double* part, double* ppot, hipStream_t st);
cb_status launch_pair(int prec, const LaunchCfg& c, bool force, bool pot, int n, const double* x,
                      const double* y, const double* z, const double* q, double eps2, int jlen, double* part,
                      double* ppot, hipStream_t st);
cb_status launch_hvp(int prec, const LaunchCfg& c, int nvec, int n, const double* x, const double* y,
                     const double* z, const double* q, const double* v, double eps2, int jlen, double* part,
                     hipStream_t st);

// Stepped ensemble md_run (ensemble.hip): supported (p, JL), a workspace
// bound over every split of ntot ions into nrun runs of at most
// kMaxBatchIons, and the driver.
bool ens_cfg_ok(int p, int jl);
size_t ens_ws_bound(int64_t ntot, int32_t nrun);
cb_status md_run_ensemble(int32_t nrun, const int64_t* offsets, const cb_state* s, const double* q,
                          const double* m, const cb_trap* traps, double t0, double dt, int64_t nsteps, double eps2,
                          int32_t prec, uint32_t flags, double* energies, int64_t every, int P, int JL, void* ws,
                          size_t ws_bytes, hipStream_t st);

// One run of at most kSmallRunMax ions in one launch per step
// (ensemble.hip), with S j-parts per 64 ions (1..kSmallPartsMax): workspace
// bytes, the default S and the driver.
constexpr int64_t kSmallRunMax = 8192;
constexpr int64_t kSmallRunDefault = 256;  // largest run that takes it by default
constexpr int kSmallPartsMax = 32;
size_t md_small_ws_bytes(int64_t n, int S);
int small_parts(int64_t n);
cb_status md_run_small(int64_t n, const cb_state* s, const double* q, const double* m, const cb_trap* trap,
                       double t0, double dt, int64_t nsteps, double eps2, int32_t prec, uint32_t flags,
                       double* energies, int64_t every, int S, void* ws, size_t ws_bytes, hipStream_t st);

// Batched md_run (batched.hip): picks the persistent kernel or the stepped
// ensemble path.
cb_status md_run_batched(int32_t nrun, const int64_t* offsets, const cb_state* s, const double* q,
                         const double* m, const cb_trap* traps, double t0, double dt, int64_t nsteps,
                         double eps2, int32_t prec, uint32_t flags, double* energies, int64_t every, void* ws,
                         size_t ws_bytes, hipStream_t st);

}  // namespace cb
