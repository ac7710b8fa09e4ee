// Host side of libcoulomb_mi355x.so: argument checking, workspace layout,
// launch-configuration table, kernel dispatch.  Declarations and the contract
// of every entry point are in include/coulomb.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>

#include "coulomb.h"
#include "internal.hpp"
#include "step_common.hpp"

__device__ unsigned int g_cb_flags;

namespace cb {

// ------------------------------------------------------------------ errors
static thread_local std::string t_err;

cb_status fail(cb_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    t_err = buf;
    return st;
}

cb_status ok() {
    t_err.clear();
    return CB_OK;
}

cb_status check_launch(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(CB_EHIP, "%s: %s", what, hipGetErrorString(e));
    return CB_OK;
}

// Device address of this GPU's flag word, looked up once per device (a fixed
// table, so that no call allocates host memory for it).
unsigned* flags_ptr() {
    static std::mutex mu;
    static unsigned* per_dev[kMaxDevices];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(mu);
    if (per_dev[dev]) return per_dev[dev];
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(g_cb_flags)) != hipSuccess) return nullptr;
    per_dev[dev] = static_cast<unsigned*>(p);
    return per_dev[dev];
}

// ------------------------------------------------------- configurations
static std::mutex g_cfg_mu;
static std::map<long long, LaunchCfg> g_cfg;

int n_bucket(int64_t n) {
    int b = 0;
    while (b < 62 && (int64_t(1) << b) < n) ++b;
    return (int64_t(1) << b) < n ? 63 : b;
}

// (op, precision, size bucket) -> table key; op and precision are taken as
// unsigned fields, so an out-of-range value from a caller or a tuning file
// gives a key of its own rather than an undefined shift
static long long cfg_key(int op, int prec, int64_t n) {
    const unsigned long long k = ((unsigned long long)(uint16_t)op << 40) | ((unsigned long long)(uint8_t)prec << 32) |
                                 (unsigned long long)n_bucket(n);
    return (long long)k;
}

// Heuristic default (measured on MI355X at n = 1e5): one i-particle per
// lane and many short waves -- about 64 waves per SIMD over the launch, by
// j-splits -- so that the last waves of the launch leave little of the chip
// idle; ILP comes from the independent FMA chains within a pair.
LaunchCfg default_cfg(int op, int64_t n, int prec) {
    LaunchCfg c;
    c.tuned = 0;
    c.algo = ALGO_DIRECT;
    (void)prec;
    if (op == CB_OP_MD_ENSEMBLE) {
        // Stepped ensemble path (ensemble.hip).  While this entry is untuned,
        // md_run_batched picks the path and (p, JL) from the run sizes.
        c.algo = ALGO_SYM_LDS;
        c.p = 4;
        c.wg = kSymGroup;
        c.splits = 256;
        return c;
    }
    const bool force_op = sym_op(op);
    if ((op == CB_OP_MD_STEP || op == CB_OP_MD_RUN) && n <= kSmallRunDefault) {
        // One launch per step: for the smallest runs the two-launch step is
        // bound by the latency of its second launch (measured on MI355X,
        // per step without / with energy records: 6.8 / 9.0 us against 7.7 /
        // 9.0 at 128 ions, 7.1 / 9.5 against 7.5 / 8.6 at 256; from 384 ions
        // the two-launch step with its 16-thread epilogue is faster, 8.4 /
        // 9.6 against 8.7 / 11.3).
        c.algo = ALGO_SMALL;
        c.p = 1;
        c.wg = 64;
        c.splits = small_parts(n);
        return c;
    }
    if (force_op && n >= 16384 && n <= kSymMaxN) {
        // Newton's third law: each pair once (see pair_sym.hpp), reactions
        // summed through LDS.  Eight ions per lane amortise the per-j wave
        // reduction best; below 32768 ions smaller tiles keep enough of them
        // in flight; below 16384 the direct kernel is faster (measured on
        // MI355X).  The energy takes the same stage, with the potential as a
        // fourth component of the sums.  From 81920 ions the row-group tiles
        // (four i-blocks per workgroup) take the same time or less -- 0.98 to
        // 1.006 of the one-wave tiles' time from 81920 to 262144 ions, 0.96
        // for the energy at 100000 -- while writing and reading back 0.89 GB
        // of partial sums per evaluation at 100000 ions instead of 1.30;
        // below that the workgroups are too few to share out evenly (1.08x
        // the time at 65536 ions, 1.35x at 32768).
        c.algo = n >= kSymRowsMinN ? ALGO_SYM_ROWS : ALGO_SYM_LDS;
        c.wg = kSymGroup;
        c.p = n >= 32768 ? 8 : (n >= 24576 ? 6 : 4);
        c.splits = n >= 32768 ? 512 : 256;
        return c;
    }
    if ((op == CB_OP_HVP || op == CB_OP_ADJOINT) && n >= kHvpSymMinN && n <= hvp_sym_max_n(2)) {
        // Hessian-vector products by Newton's third law (hvp_sym.hpp): two
        // ions per lane (the four-vector pass keeps 24 vector components and
        // 24 sums per lane), up to four vectors per pass (wg), short segments
        // for enough tiles at 8192 ions
        c.algo = ALGO_SYM_LDS;
        c.wg = 4;
        c.p = 2;
        c.splits = 128;
        return c;
    }
    return direct_cfg(op, n, prec);
}

// The all-pairs kernel's default shape for op at n.
LaunchCfg direct_cfg(int op, int64_t n, int prec) {
    LaunchCfg c;
    c.tuned = 0;
    c.algo = ALGO_DIRECT;
    (void)prec;
    c.wg = 64;
    c.p = 1;
    const int64_t waves = (n + 64 * c.p - 1) / (64 * c.p);
    // HVP-shaped work (more registers per lane, fewer waves per SIMD) runs
    // best with longer j-ranges per wave: about 3072 waves over the launch
    // in 256-thread workgroups (measured on MI355X at n = 8192: 24 splits,
    // 0.41 ms for 8 vectors against 0.53 with 16 splits of 64 threads).
    // Below 16384 ions the force kernel, too, prefers about 4096 waves in
    // 256-thread workgroups (md steps at 4096 and 8192 ions).
    const bool hv = (op == CB_OP_HVP || op == CB_OP_ADJOINT);
    const bool small = n < 16384;
    if (hv || small) c.wg = 256;
    int64_t s = ((hv ? 3072 : (small ? 4096 : 65536)) + waves - 1) / waves;
    s = std::max<int64_t>(1, std::min<int64_t>(s, kMaxSplits));
    // j-ranges of at least 64, or 32 for the force kernel up to 1024 ions
    // (with one epilogue thread per ion, md_run at 1024 ions with energies
    // every step took 16.5 us per step at 32 splits of 32 j's, 17.2 at 16
    // splits and 21 at 64; measured on MI355X)
    s = std::min<int64_t>(s, std::max<int64_t>(1, n / (hv || n > 1024 ? 64 : 32)));
    // md_step / md_run up to 4096 ions: j-ranges of 16, at most 64 of them,
    // whose sums the epilogue spreads over 16 threads per ion (with energies
    // every step: 11.0 us per step at 1024 ions against 11.8-12.0 with 32 or
    // 48 splits; 14.3 at 2048 against 15.3; 24.9 at 4096 against 25.2-26.7)
    if ((op == CB_OP_MD_STEP || op == CB_OP_MD_RUN) && n <= 4096)
        s = std::min<int64_t>(kMaxSplits, std::max<int64_t>(1, n / 16));
    c.splits = (int)s;
    return c;
}

LaunchCfg get_cfg(int op, int64_t n, int prec) {
    std::lock_guard<std::mutex> lk(g_cfg_mu);
    auto it = g_cfg.find(cfg_key(op, prec, n));
    if (it != g_cfg.end()) return it->second;
    return default_cfg(op, n, prec);
}

void put_cfg(int op, int64_t n, int prec, LaunchCfg c) {
    std::lock_guard<std::mutex> lk(g_cfg_mu);
    g_cfg[cfg_key(op, prec, n)] = c;
}

void drop_cfg(int op, int64_t n, int prec) {
    std::lock_guard<std::mutex> lk(g_cfg_mu);
    g_cfg.erase(cfg_key(op, prec, n));
}

bool valid_cfg(int op, const LaunchCfg& c) {
    if (c.algo == ALGO_SMALL)
        return (op == CB_OP_MD_STEP || op == CB_OP_MD_RUN) && c.p == 1 && c.wg == 64 && c.splits >= 1 &&
               c.splits <= kSmallPartsMax;
    if (op == CB_OP_MD_ENSEMBLE)
        return (c.algo == ALGO_DIRECT && c.p == kBatchP && c.wg == kBatchWG && c.splits == 1) ||
               (c.algo == ALGO_SYM_LDS && c.wg == kSymGroup && ens_cfg_ok(c.p, c.splits));
    const bool force_op = sym_op(op);
    const bool hv_op = (op == CB_OP_HVP || op == CB_OP_ADJOINT);
    if (c.algo == ALGO_SYM_ROWS) return force_op && sym_cfg_ok(c.p, c.wg, c.splits) && sym_rows_p_ok(c.p);
    if (is_sym(c.algo))
        return (force_op && sym_cfg_ok(c.p, c.wg, c.splits)) ||
               (hv_op && c.algo == ALGO_SYM_LDS && (c.wg == 1 || c.wg == 2 || c.wg == 4) &&
                hvp_sym_cfg_ok(c.p, c.splits));
    if (c.algo != ALGO_DIRECT) return false;
    const bool p_ok = (op == CB_OP_HVP || op == CB_OP_ADJOINT) ? (c.p == 1 || c.p == 2)
                                                                 : (c.p == 1 || c.p == 2 || c.p == 4);
    return p_ok && (c.wg == 64 || c.wg == 128 || c.wg == 256) && c.splits >= 1 && c.splits <= kMaxSplits;
}

// Actual j-range per split for a requested split count (multiple of 8).
int split_len(int64_t n, int splits) {
    int64_t len = (n + splits - 1) / splits;
    len = (len + 7) / 8 * 8;
    return (int)std::max<int64_t>(len, 8);
}

int n_splits(int64_t n, int jlen) { return (int)((n + jlen - 1) / jlen); }

// ------------------------------------------------------------- workspace
static size_t al(size_t b) { return (b + 255) / 256 * 256; }

WsLayout ws_layout(int op, int64_t n, int32_t nrun, int32_t nvec, int32_t prec) {
    WsLayout L{};
    // entry points size the workspace before they check n: keep the sizing
    // arithmetic in range for any n (the call then fails on n itself)
    n = std::min<int64_t>(std::max<int64_t>(n, 1), kMaxIons);
    const size_t N = (size_t)n;
    const size_t nv = (size_t)std::max(1, (int)nvec);
    size_t off = 0;
    // the configuration whose Newton's-third-law partials the buffer must hold
    // (coulomb_trap_grad's force stage follows the forces' configuration, or
    // the energy's when it also returns the energy: the larger of the two)
    const int cfg_op = op == CB_OP_GRAD ? CB_OP_ENERGY : op;
    // the tiles' pair energies too: energies, energy records, the gradient's energy
    const bool pot = (op == CB_OP_ENERGY || op == CB_OP_MD_RUN || op == CB_OP_GRAD);
    if (op == CB_OP_GRAD) op = CB_OP_MD_STEP;  // the same buffers: force stage, potential partials, energy blocks
    const bool batched = (op == CB_OP_MD_RUN && nrun > 1);
    const bool hv = (op == CB_OP_HVP || op == CB_OP_ADJOINT);
    if (!batched) {
        L.part = off;
        size_t part = sizeof(double) * (size_t)kMaxSplits * 3 * (hv ? nv : 1) * N;
        const bool force_op = sym_op(op);
        LaunchCfg c = get_cfg(cfg_op, n, prec);
        if (cfg_op == CB_OP_ENERGY) {  // coulomb_trap_grad: the forces' stage too
            const LaunchCfg f = get_cfg(CB_OP_FORCES, n, prec);
            if (is_sym(f.algo) && sym_cfg_ok(f.p, f.wg, f.splits) &&
                (!is_sym(c.algo) || sym_ws_bytes(n, f.p, f.splits, true, sym_rows(f.algo)) >
                                        sym_ws_bytes(n, c.p, c.splits, true, sym_rows(c.algo))))
                c = f;
        }
        if (force_op && n <= kSymMaxN && is_sym(c.algo) && sym_cfg_ok(c.p, c.wg, c.splits))
            // the configured symmetric stage: finished forces [3][n] then its tiles and partials
            part = std::max(part, al(sizeof(double) * 3 * N) + sym_ws_bytes(n, c.p, c.splits, pot, sym_rows(c.algo)));
        if (hv && is_sym(c.algo) && hvp_sym_cfg_ok(c.p, c.splits))  // (the adjoint's product [3][n] first)
            part = std::max(part, (op == CB_OP_ADJOINT ? al(sizeof(double) * 3 * N) : 0) +
                                      hvp_sym_ws_bytes(n, c.p, c.splits, hvp_sym_passes((int)nv, c.wg)));
        off += al(part);
        L.ppot = off;
        if (op == CB_OP_ENERGY || op == CB_OP_MD_STEP || op == CB_OP_MD_RUN)
            off += al(sizeof(double) * (size_t)kMaxSplits * N);
        L.eblk = off;  // two sets of block partials (md_run alternates them) and a counter
        off += al(sizeof(double) * 6 * (N / kEpiMinIons + 2));
        L.aux = off;
        if (op == CB_OP_ADJOINT) off += al(sizeof(double) * 3 * N);
    } else {
        L.batch = off;
        off += al((sizeof(int64_t) * 2 + sizeof(cb_trap) + sizeof(int)) * (size_t)nrun + 64);
        // Persistent kernel: force accumulators of its Newton's-third-law pass.
        // Stepped path: its tables, partials and second position buffer.
        L.aux = off;
        off += al(std::max(sizeof(double) * 3 * (size_t)kMaxBatchIons * (size_t)std::min<int32_t>(nrun, kBatchGridMax),
                           ens_ws_bound(n, nrun)));
    }
    L.total = off + 256;
    return L;
}

bool trap_ok(const cb_trap* t, const char* who, cb_status* st) {
    if (!t) {
        *st = fail(CB_EINVAL, "%s: trap is NULL", who);
        return false;
    }
    const double v[] = {t->wx, t->wy, t->wz, t->rf_a, t->rf_q, t->rf_omega, t->rf_phase, t->gamma,
                        t->wx1, t->wy1, t->t_ramp0, t->t_ramp1};
    for (double d : v)
        if (!std::isfinite(d)) {
            *st = fail(CB_EINVAL, "%s: non-finite trap parameter", who);
            return false;
        }
    if (t->kind != 0 && t->kind != 1) {
        *st = fail(CB_EINVAL, "%s: trap kind must be 0 or 1", who);
        return false;
    }
    if (t->gamma < 0.0) {
        *st = fail(CB_EINVAL, "%s: friction gamma must be >= 0", who);
        return false;
    }
    return true;
}

}  // namespace cb

using namespace cb;

// ======================================================================= ABI
extern "C" {

const char* cb_last_error(void) { return t_err.c_str(); }

size_t cb_workspace_size(int32_t op, int64_t n, int32_t nrun, int32_t nvec, int32_t prec) {
    if (n < 1 || n > kMaxIons || op < 0 || op == CB_OP_MD_ENSEMBLE || op > CB_OP_GRAD || prec < 0 ||
        prec > CB_MIXED_F32D)
        return 0;
    if (op == CB_OP_HVP && (nvec < 1 || nvec > kMaxVec)) return 0;
    return ws_layout(op, n, nrun, nvec, prec).total;
}

cb_status cb_get_config(int32_t op, int64_t n, int32_t prec, int32_t out[5]) {
    if (!out || n < 1 || n > kMaxIons || op < 0 || op > CB_OP_MD_ENSEMBLE || prec < 0 || prec > CB_MIXED_F32D)
        return fail(CB_EINVAL, "cb_get_config: bad argument");
    LaunchCfg c = get_cfg(op, n, prec);
    out[0] = c.algo;
    out[1] = c.p;
    out[2] = c.wg;
    out[3] = c.splits;
    out[4] = c.tuned;
    return ok();
}

cb_status cb_set_config(int32_t op, int64_t n, int32_t prec, int32_t algo, int32_t p, int32_t wg, int32_t splits) {
    if (n < 1 || n > kMaxIons || op < 0 || op > CB_OP_MD_ENSEMBLE || prec < 0 || prec > CB_MIXED_F32D)
        return fail(CB_EINVAL, "cb_set_config: bad argument");
    if (algo == 0 && p == 0 && wg == 0 && splits == 0) {
        drop_cfg(op, n, prec);
        return ok();
    }
    LaunchCfg c{p, wg, splits, 1, algo};
    const bool hv_op = (op == CB_OP_HVP || op == CB_OP_ADJOINT);
    if (!valid_cfg(op, c) || (is_sym(algo) && op != CB_OP_MD_ENSEMBLE && !hv_op && n > kSymMaxN) ||
        (is_sym(algo) && hv_op && n > hvp_sym_max_n(p)) || (algo == ALGO_SMALL && n > kSmallRunMax))
        return fail(CB_EINVAL, "cb_set_config: unsupported configuration algo=%d p=%d wg=%d splits=%d", algo, p, wg,
                    splits);
    put_cfg(op, n, prec, c);
    return ok();
}

cb_status cb_trap_k(const cb_trap* trap, double t, double k_out[3]) {
    cb_status st;
    if (!k_out) return fail(CB_EINVAL, "cb_trap_k: k_out is NULL");
    if (!trap_ok(trap, "cb_trap_k", &st)) return st;
    if (!std::isfinite(t)) return fail(CB_EINVAL, "cb_trap_k: t must be finite");
    const TrapK k = trap_k(*trap, t);
    k_out[0] = k.kx;
    k_out[1] = k.ky;
    k_out[2] = k.kz;
    return ok();
}

cb_status cb_poll_flags(void* stream, uint32_t* flags_out) {
    if (!flags_out) return fail(CB_EINVAL, "cb_poll_flags: flags_out is NULL");
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (hipStreamSynchronize(st) != hipSuccess) return fail(CB_EHIP, "cb_poll_flags: stream sync failed");
    unsigned* d = flags_ptr();
    if (!d) return fail(CB_EHIP, "cb_poll_flags: flag symbol not found");
    unsigned v = 0;
    if (hipMemcpy(&v, d, sizeof v, hipMemcpyDeviceToHost) != hipSuccess)
        return fail(CB_EHIP, "cb_poll_flags: read failed");
    unsigned z = 0;
    if (hipMemcpy(d, &z, sizeof z, hipMemcpyHostToDevice) != hipSuccess)
        return fail(CB_EHIP, "cb_poll_flags: clear failed");
    *flags_out = v;
    if (v & 1u) return fail(CB_ENONFINITE, "non-finite values were produced");
    return ok();
}

}  // extern "C"
