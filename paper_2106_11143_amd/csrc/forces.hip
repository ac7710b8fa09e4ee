// Entry points coulomb_forces, coulomb_energy, md_step and md_run (single
// run): argument checks, workspace carving and the launch sequence of the
// pair kernel and the element-wise epilogue.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <mutex>

#include "internal.hpp"
#include "step_kernels.hpp"

namespace cb {

static bool overlaps(const void* a, const void* b, int64_t n) {
    if (!a || !b) return false;
    const char* pa = static_cast<const char*>(a);
    const char* pb = static_cast<const char*>(b);
    const int64_t bytes = n * (int64_t)sizeof(double);
    return pa < pb + bytes && pb < pa + bytes;
}

static cb_status check_common(const char* who, int64_t n, int32_t prec, double eps2, void* ws, size_t ws_bytes,
                              size_t need) {
    if (n < 1 || n > kMaxIons) return fail(CB_EINVAL, "%s: n = %lld out of range [1, 2^28]", who, (long long)n);
    if (prec < CB_FP64 || prec > CB_MIXED_F32D) return fail(CB_EINVAL, "%s: unknown precision %d", who, prec);
    if (!(eps2 >= 0.0) || !std::isfinite(eps2)) return fail(CB_EINVAL, "%s: eps2 must be finite and >= 0", who);
    if (!ws) return fail(CB_EINVAL, "%s: workspace is NULL", who);
    if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) return fail(CB_EINVAL, "%s: workspace not 256-byte aligned", who);
    if (ws_bytes < need)
        return fail(CB_ENOWS, "%s: workspace has %zu bytes, needs %zu", who, ws_bytes, need);
    return CB_OK;
}

// [a, a + na) and [b, b + nb) doubles intersect.
static bool overlaps2(const void* a, int64_t na, const void* b, int64_t nb) {
    if (!a || !b) return false;
    const char* pa = static_cast<const char*>(a);
    const char* pb = static_cast<const char*>(b);
    return pa < pb + nb * (int64_t)sizeof(double) && pb < pa + na * (int64_t)sizeof(double);
}

static double* at(void* ws, size_t off) { return reinterpret_cast<double*>(static_cast<char*>(ws) + off); }

// Blocks of k_epilogue over E.n ions with epi_parts(E.n, E.S) threads per ion.
static int epilogue_blocks(const EpiParams& E) {
    const int ipb = kEpiThreads / epi_parts(E.n, E.S);
    return (E.n + ipb - 1) / ipb;
}

// k_epilogue on g blocks (epilogue_blocks(E), plus one for a deferred record).
static cb_status launch_epilogue(const EpiParams& E, unsigned g, hipStream_t st) {
    switch (epi_parts(E.n, E.S)) {
        case 16: k_epilogue<16><<<g, kEpiThreads, 0, st>>>(E); break;
        case 8: k_epilogue<8><<<g, kEpiThreads, 0, st>>>(E); break;
        default: k_epilogue<1><<<g, kEpiThreads, 0, st>>>(E); break;
    }
    return check_launch("k_epilogue");
}

struct PairRun {
    LaunchCfg cfg;
    int jlen, S;
};

static PairRun plan(int op, int64_t n, int prec) {
    PairRun r;
    r.cfg = get_cfg(op, n, prec);
    if (r.cfg.algo != ALGO_DIRECT) r.cfg = direct_cfg(CB_OP_ENERGY, n, prec);  // direct kernel needed
    r.jlen = split_len(n, r.cfg.splits);
    r.S = n_splits(n, r.jlen);
    return r;
}

static size_t al256(size_t b) { return (b + 255) / 256 * 256; }

// The pair stage with the configured algorithm: forces, and the potential
// sums too when pot.  Direct: partial sums [S][3][n] at ws+L.part (to be
// scaled by k_C q_i) and [S][n] at ws+L.ppot.  Symmetric: the finished forces
// [3][n] at ws+L.part (S = 1, prescaled), its tiles and partials after them,
// and the potential sums [n] at ws+L.ppot (S = 1).  tiles_ready: when
// non-NULL and true, the tile table of the symmetric stage is already in ws (an earlier
// call of the same md_run); set to true once it is.
static cb_status force_stage(int op, int prec, int64_t n, const double* x, const double* y, const double* z,
                             const double* q, double eps2, void* ws, const WsLayout& L, hipStream_t st, int* S_out,
                             bool* prescaled, bool pot = false, bool* tiles_ready = nullptr) {
    const LaunchCfg cfg = get_cfg(op, n, prec);
    double* part = at(ws, L.part);
    double* ppot = pot ? at(ws, L.ppot) : nullptr;
    if (is_sym(cfg.algo) && n <= kSymMaxN && prec != CB_MIXED_F32D) {
        *S_out = 1;
        *prescaled = true;
        void* tiles_ws = static_cast<char*>(ws) + L.part + al256(sizeof(double) * 3 * (size_t)n);
        const cb_status rc =
            launch_pair_sym(prec, cfg, (int)n, x, y, z, q, eps2, tiles_ws, part, st, ppot, tiles_ready && *tiles_ready);
        if (tiles_ready && rc == CB_OK) *tiles_ready = true;
        return rc;
    }
    const PairRun pr = plan(op, n, prec);
    *S_out = pr.S;
    *prescaled = false;
    return launch_pair(prec, pr.cfg, true, pot, (int)n, x, y, z, q, eps2, pr.jlen, part, ppot, st);
}

// ------------------------------------------- allocation-free forces
// coulomb_forces_noalloc keeps its partial sums in this array instead of a
// caller's workspace.  Each GPU the library runs on holds its own copy (the
// code object's static device memory) until the process ends.  In host code
// `scratch` names a host-side stand-in: the device address comes from
// scratch_addr() alone.
constexpr size_t kScratchBytes = size_t(64) << 20;
constexpr int64_t kNoallocMaxN = (int64_t)(kScratchBytes / (3 * sizeof(double)));  // one j-split of [3][n]
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// Device address of the current GPU's scratch array: looked up with
// hipGetSymbolAddress on the first call on each device (with that device
// current) and kept in a fixed per-device table.
static void* scratch_addr(cb_status* rc) {
    static std::mutex mu;
    static void* per_dev[kMaxDevices];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        *rc = fail(CB_EHIP, "coulomb_forces_noalloc: no current device");
        return nullptr;
    }
    if (dev < 0 || dev >= kMaxDevices) {
        *rc = fail(CB_EUNSUPPORTED, "coulomb_forces_noalloc: device %d beyond the %d the library tracks", dev,
                   kMaxDevices);
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(mu);
    if (!per_dev[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            *rc = fail(CB_EHIP, "coulomb_forces_noalloc: scratch symbol lookup failed: %s", hipGetErrorString(e));
            return nullptr;
        }
        per_dev[dev] = p;
    }
    return per_dev[dev];
}

// Single-run velocity-Verlet driver shared by md_step and md_run.
static cb_status md_single(int64_t n, const cb_state* s, const double* q, const double* m, const cb_trap* trap,
                           double t0, double dt, int64_t nsteps, double eps2, int32_t prec, uint32_t flags,
                           double* energies, int64_t every, void* ws, int op, hipStream_t st) {
    const WsLayout L = ws_layout(op, n, 1, 1, prec);
    // One launch per step (every pair direct, then trap, kick and drift) when
    // so configured: the default up to kSmallRunMax ions.
    const LaunchCfg sc = get_cfg(op, n, prec);
    if (sc.algo == ALGO_SMALL && n <= kSmallRunMax && md_small_ws_bytes(n, sc.splits) <= L.ppot - L.part)
        return md_run_small(n, s, q, m, trap, t0, dt, nsteps, eps2, prec, flags, energies, every, sc.splits,
                            static_cast<char*>(ws) + L.part, L.ppot - L.part, st);
    const PairRun pr = plan(op, n, prec);
    double* part = at(ws, L.part);
    double* ppot = at(ws, L.ppot);
    double* eblk = at(ws, L.eblk);
    unsigned* fl = flags_ptr();
    if (!fl) return fail(CB_EHIP, "md_run: device flag symbol not found");
    EpiParams E{};
    E.n = (int)n;
    E.S = pr.S;
    E.part = part;
    E.ppot = ppot;
    E.q = q;
    E.m = m;
    E.x = s->x; E.y = s->y; E.z = s->z;
    E.vx = s->vx; E.vy = s->vy; E.vz = s->vz;
    E.ax = s->ax; E.ay = s->ay; E.az = s->az;
    E.trap = *trap;
    E.t0 = t0;
    E.dt = dt;
    E.eblk = eblk;
    E.flags = fl;
    cb_status rc;
    const bool rec0 = energies && every > 0;
    const bool init = (flags & CB_INIT_ACCEL) != 0;
    // Energy records: a recording epilogue leaves its block partials in one
    // of two buffers (alternating), and the next epilogue launch sums them
    // with one extra block (stream order makes them complete); a record on
    // the last launch is summed by k_energy_final.
    const size_t nbuf = 3 * ((size_t)n / kEpiMinIons + 1);
    double* ebuf[2] = {eblk, eblk + nbuf};
    int parity = 0;
    const double* pend = nullptr;
    double* pend_out = nullptr;
    int pend_nb = 0;  // block partials of the pending record
    E.efinal = nullptr;
    E.ecount = nullptr;
    auto epilogue = [&](double* rec_out) -> cb_status {
        const int nb = epilogue_blocks(E);
        E.eblk = ebuf[parity];
        E.eprev = pend;
        E.eprev_out = pend_out;
        E.nprev = pend_nb;
        cb_status r = launch_epilogue(E, (unsigned)(nb + (pend ? 1 : 0)), st);
        if (r) return r;
        pend = rec_out ? ebuf[parity] : nullptr;
        pend_out = rec_out;
        pend_nb = rec_out ? nb : 0;
        if (rec_out) parity ^= 1;
        return CB_OK;
    };

    bool prescaled_now = false;
    // Force (and potential) pair launch with the configured algorithm.  A
    // potential alone (an energy record of step 0 without CB_INIT_ACCEL) takes
    // the symmetric stage too when it is configured (its forces unused), else
    // the direct kernel's potential-only pass.
    const bool sym_stage = is_sym(get_cfg(op, n, prec).algo) && n <= kSymMaxN;
    // the symmetric stage's tile table is the same at every step: built by
    // the first force stage of the run, read by the later ones
    bool plan_ready = false;
    auto pairs = [&](bool force, bool pot) -> cb_status {
        if (force || sym_stage) {
            int S = 0;
            bool pre = false;
            cb_status r = force_stage(op, prec, n, s->x, s->y, s->z, q, eps2, ws, L, st, &S, &pre, pot, &plan_ready);
            E.S = S;
            prescaled_now = pre;
            return r;
        }
        E.S = pr.S;
        prescaled_now = false;
        return launch_pair(prec, pr.cfg, force, pot, (int)n, s->x, s->y, s->z, q, eps2, pr.jlen, part, ppot, st);
    };

    // Step 0: initial acceleration and/or energies, then the first drift.
    if (init || rec0) {
        if ((rc = pairs(init, rec0))) return rc;
    }
    E.step = 0;
    E.mode = (init ? EPI_ACCEL : 0u) | (rec0 ? EPI_ENERGY : 0u) | (nsteps > 0 ? EPI_DRIFT : 0u);
    if (prescaled_now) E.mode |= EPI_PRESCALED | EPI_POT_SHARE;
    if (E.mode && (rc = epilogue(rec0 ? energies : nullptr))) return rc;
    for (int64_t k = 1; k <= nsteps; ++k) {
        const bool rec = rec0 && (k % every == 0);
        if ((rc = pairs(true, rec))) return rc;
        E.step = k;
        E.mode = EPI_KICK | (rec ? EPI_ENERGY : 0u) | (k < nsteps ? EPI_DRIFT : 0u) |
                 (prescaled_now ? EPI_PRESCALED | EPI_POT_SHARE : 0u);
        if ((rc = epilogue(rec ? energies + 4 * (k / every) : nullptr))) return rc;
    }
    if (pend) {
        k_energy_final<<<1, kEpiThreads, 0, st>>>(pend_nb, pend, pend_out, REC_ALL);
        if ((rc = check_launch("k_energy_final"))) return rc;
    }
    return ok();
}

static bool state_ok(const cb_state* s, int64_t n, const double* q, const double* m, const char* who,
                     cb_status* st) {
    if (!s) {
        *st = fail(CB_EINVAL, "%s: state is NULL", who);
        return false;
    }
    double* arr[9] = {s->x, s->y, s->z, s->vx, s->vy, s->vz, s->ax, s->ay, s->az};
    for (int a = 0; a < 9; ++a) {
        if (!arr[a]) {
            *st = fail(CB_EINVAL, "%s: state array %d is NULL", who, a);
            return false;
        }
        for (int b = a + 1; b < 9; ++b)
            if (overlaps(arr[a], arr[b], n)) {
                *st = fail(CB_EINVAL, "%s: state arrays %d and %d overlap", who, a, b);
                return false;
            }
        if (overlaps(arr[a], q, n) || overlaps(arr[a], m, n)) {
            *st = fail(CB_EINVAL, "%s: state array %d overlaps q or m", who, a);
            return false;
        }
    }
    if (!q || !m) {
        *st = fail(CB_EINVAL, "%s: q or m is NULL", who);
        return false;
    }
    return true;
}

}  // namespace cb

using namespace cb;

extern "C" {

cb_status coulomb_forces(int64_t n, const double* x, const double* y, const double* z, const double* q,
                         double eps2, int32_t prec, double* fx, double* fy, double* fz, void* ws, size_t ws_bytes,
                         void* stream) {
    const WsLayout L = ws_layout(CB_OP_FORCES, n > 0 ? n : 1, 1, 1, prec);
    cb_status rc = check_common("coulomb_forces", n, prec, eps2, ws, ws_bytes, L.total);
    if (rc) return rc;
    if (!x || !y || !z || !q || !fx || !fy || !fz) return fail(CB_EINVAL, "coulomb_forces: NULL array");
    const void* in[4] = {x, y, z, q};
    const void* out[3] = {fx, fy, fz};
    for (auto o : out) {
        for (auto i : in)
            if (overlaps(o, i, n)) return fail(CB_EINVAL, "coulomb_forces: output aliases an input");
    }
    if (overlaps(fx, fy, n) || overlaps(fx, fz, n) || overlaps(fy, fz, n))
        return fail(CB_EINVAL, "coulomb_forces: outputs overlap");
    hipStream_t st = static_cast<hipStream_t>(stream);
    int S = 0;
    bool prescaled = false;
    if ((rc = force_stage(CB_OP_FORCES, prec, n, x, y, z, q, eps2, ws, L, st, &S, &prescaled))) return rc;
    EpiParams E{};
    E.n = (int)n;
    E.S = S;
    E.part = at(ws, L.part);
    E.q = q;
    E.fx = fx;
    E.fy = fy;
    E.fz = fz;
    E.mode = EPI_FORCES | (prescaled ? EPI_PRESCALED : 0u);
    E.flags = flags_ptr();
    if (!E.flags) return fail(CB_EHIP, "coulomb_forces: device flag symbol not found");
    if ((rc = launch_epilogue(E, (unsigned)epilogue_blocks(E), st))) return rc;
    return ok();
}

cb_status coulomb_forces_noalloc(int64_t n, const double* x, const double* y, const double* z, const double* q,
                                 double eps2, int32_t prec, double* fx, double* fy, double* fz, void* stream) {
    if (n < 1) return fail(CB_EINVAL, "coulomb_forces_noalloc: n = %lld < 1", (long long)n);
    if (n > kNoallocMaxN)
        return fail(CB_ENOWS, "coulomb_forces_noalloc: n = %lld exceeds the %lld ions its %zu-byte static scratch holds",
                    (long long)n, (long long)kNoallocMaxN, kScratchBytes);
    if (prec < CB_FP64 || prec > CB_MIXED_F32D) return fail(CB_EINVAL, "coulomb_forces_noalloc: unknown precision %d", prec);
    if (!(eps2 >= 0.0) || !std::isfinite(eps2)) return fail(CB_EINVAL, "coulomb_forces_noalloc: eps2 must be finite and >= 0");
    if (!x || !y || !z || !q || !fx || !fy || !fz) return fail(CB_EINVAL, "coulomb_forces_noalloc: NULL array");
    const void* in[4] = {x, y, z, q};
    const void* out[3] = {fx, fy, fz};
    for (auto o : out)
        for (auto i : in)
            if (overlaps(o, i, n)) return fail(CB_EINVAL, "coulomb_forces_noalloc: output aliases an input");
    if (overlaps(fx, fy, n) || overlaps(fx, fz, n) || overlaps(fy, fz, n))
        return fail(CB_EINVAL, "coulomb_forces_noalloc: outputs overlap");
    cb_status rc = CB_OK;
    void* ws = scratch_addr(&rc);
    if (!ws) return rc;
    unsigned* fl = flags_ptr();
    if (!fl) return fail(CB_EHIP, "coulomb_forces_noalloc: device flag symbol not found");
    hipStream_t st = static_cast<hipStream_t>(stream);
    double* part = static_cast<double*>(ws);
    // The configured Newton's-third-law stage when its tiles fit beside the
    // finished forces (bitwise the result of coulomb_forces), else the direct
    // kernel with no more j-splits than the scratch holds.
    const LaunchCfg cfg = get_cfg(CB_OP_FORCES, n, prec);
    const size_t fbytes = al256(sizeof(double) * 3 * (size_t)n);
    const bool sym = is_sym(cfg.algo) && n <= kSymMaxN && prec != CB_MIXED_F32D &&
                     fbytes + sym_ws_bytes(n, cfg.p, cfg.splits, false, sym_rows(cfg.algo)) <= kScratchBytes;
    int S = 1;
    if (sym) {
        if ((rc = launch_pair_sym(prec, cfg, (int)n, x, y, z, q, eps2, static_cast<char*>(ws) + fbytes, part, st)))
            return rc;
    } else {
        LaunchCfg c = cfg.algo == ALGO_DIRECT ? cfg : direct_cfg(CB_OP_ENERGY, n, prec);
        const int64_t smax = (int64_t)(kScratchBytes / (3 * sizeof(double) * (size_t)n));
        c.splits = (int)std::max<int64_t>(1, std::min<int64_t>(c.splits, smax));
        const int jlen = split_len(n, c.splits);
        S = n_splits(n, jlen);  // <= c.splits, so [S][3][n] fits
        if ((rc = launch_pair(prec, c, true, false, (int)n, x, y, z, q, eps2, jlen, part, nullptr, st))) return rc;
    }
    EpiParams E{};
    E.n = (int)n;
    E.S = S;
    E.part = part;
    E.q = q;
    E.fx = fx;
    E.fy = fy;
    E.fz = fz;
    E.mode = EPI_FORCES | (sym ? EPI_PRESCALED : 0u);
    E.flags = fl;
    k_epilogue<1><<<(int)((n + kEpiThreads - 1) / kEpiThreads), kEpiThreads, 0, st>>>(E);
    if ((rc = check_launch("k_epilogue"))) return rc;
    return ok();
}

cb_status coulomb_forces_range(int64_t n, int64_t i0, int64_t i1, const double* x, const double* y, const double* z,
                               const double* q, double eps2, int32_t prec, double* fx, double* fy, double* fz,
                               void* ws, size_t ws_bytes, void* stream) {
    const WsLayout L = ws_layout(CB_OP_FORCES, n > 0 ? n : 1, 1, 1, prec);
    cb_status rc = check_common("coulomb_forces_range", n, prec, eps2, ws, ws_bytes, L.total);
    if (rc) return rc;
    if (i0 < 0 || i1 <= i0 || i1 > n)
        return fail(CB_EINVAL, "coulomb_forces_range: need 0 <= i0 < i1 <= n (i0 = %lld, i1 = %lld, n = %lld)",
                    (long long)i0, (long long)i1, (long long)n);
    if (!x || !y || !z || !q || !fx || !fy || !fz) return fail(CB_EINVAL, "coulomb_forces_range: NULL array");
    const int64_t ni = i1 - i0;
    const void* in[4] = {x, y, z, q};
    const void* out[3] = {fx, fy, fz};
    for (auto o : out)
        for (auto i : in)
            if (overlaps2(o, ni, i, n)) return fail(CB_EINVAL, "coulomb_forces_range: output aliases an input");
    if (overlaps2(fx, ni, fy, ni) || overlaps2(fx, ni, fz, ni) || overlaps2(fy, ni, fz, ni))
        return fail(CB_EINVAL, "coulomb_forces_range: outputs overlap");
    hipStream_t st = static_cast<hipStream_t>(stream);
    // The direct kernel over the i-range.  Unless a direct configuration is
    // set for the forces at this n, the range takes the whole launch's shape
    // with its j-splits multiplied by n / ni, so that one GPU's share of a
    // split evaluation fills the chip as the whole evaluation does; the
    // range's partials [S][3][ni] fit the workspace while S ni <= 64 n.
    LaunchCfg cfg = get_cfg(CB_OP_FORCES, n, prec);
    if (cfg.algo != ALGO_DIRECT) {
        cfg = direct_cfg(CB_OP_ENERGY, n, prec);
        const int64_t s = std::min<int64_t>({(int64_t)cfg.splits * n / ni, (int64_t)kMaxSplits * n / ni,
                                             std::max<int64_t>(1, n / 64)});
        cfg.splits = (int)std::max<int64_t>(1, s);
    }
    const int jlen = split_len(n, cfg.splits);
    const int S = n_splits(n, jlen);
    double* part = at(ws, L.part);
    if ((rc = launch_pair_range(prec, cfg, true, false, (int)n, (int)i0, (int)ni, x, y, z, q, eps2, jlen, part,
                                nullptr, st)))
        return rc;
    EpiParams E{};
    E.n = (int)ni;
    E.S = S;
    E.part = part;
    E.q = q + i0;
    E.fx = fx;
    E.fy = fy;
    E.fz = fz;
    E.mode = EPI_FORCES;
    E.flags = flags_ptr();
    if (!E.flags) return fail(CB_EHIP, "coulomb_forces_range: device flag symbol not found");
    k_epilogue<1><<<(int)((ni + kEpiThreads - 1) / kEpiThreads), kEpiThreads, 0, st>>>(E);
    if ((rc = check_launch("k_epilogue"))) return rc;
    return ok();
}

cb_status coulomb_pair_stage(int64_t n, const double* x, const double* y, const double* z, const double* q,
                             double eps2, int32_t prec, int32_t* splits_out, void* ws, size_t ws_bytes,
                             void* stream) {
    const WsLayout L = ws_layout(CB_OP_FORCES, n > 0 ? n : 1, 1, 1, prec);
    cb_status rc = check_common("coulomb_pair_stage", n, prec, eps2, ws, ws_bytes, L.total);
    if (rc) return rc;
    if (!x || !y || !z || !q || !splits_out) return fail(CB_EINVAL, "coulomb_pair_stage: NULL argument");
    int S = 0;
    bool prescaled = false;
    if ((rc = force_stage(CB_OP_FORCES, prec, n, x, y, z, q, eps2, ws, L, static_cast<hipStream_t>(stream), &S,
                          &prescaled)))
        return rc;
    *splits_out = prescaled ? 0 : S;
    return ok();
}

cb_status coulomb_energy(int64_t n, const double* x, const double* y, const double* z, const double* q,
                         double eps2, int32_t prec, double* u_out, void* ws, size_t ws_bytes, void* stream) {
    const WsLayout L = ws_layout(CB_OP_ENERGY, n > 0 ? n : 1, 1, 1, prec);
    cb_status rc = check_common("coulomb_energy", n, prec, eps2, ws, ws_bytes, L.total);
    if (rc) return rc;
    if (prec == CB_MIXED_F32D) return fail(CB_EUNSUPPORTED, "coulomb_energy: CB_MIXED_F32D is for the forces only");
    if (!x || !y || !z || !q || !u_out) return fail(CB_EINVAL, "coulomb_energy: NULL argument");
    hipStream_t st = static_cast<hipStream_t>(stream);
    double* ppot = at(ws, L.ppot);
    double* eblk = at(ws, L.eblk);
    int S = 0;
    bool share = false;  // the potential partials hold energy shares (the symmetric stage)
    const LaunchCfg ecfg = get_cfg(CB_OP_ENERGY, n, prec);
    if (is_sym(ecfg.algo) && n <= kSymMaxN) {
        // the Newton's-third-law stage with the potential as a fourth
        // component (its forces are a by-product, left in the workspace)
        bool prescaled = false;
        if ((rc = force_stage(CB_OP_ENERGY, prec, n, x, y, z, q, eps2, ws, L, st, &S, &prescaled, true))) return rc;
        share = prescaled;
    } else {
        const PairRun pr = plan(CB_OP_ENERGY, n, prec);
        S = pr.S;
        if ((rc = launch_pair(prec, pr.cfg, false, true, (int)n, x, y, z, q, eps2, pr.jlen, nullptr, ppot, st)))
            return rc;
    }
    EpiParams E{};
    E.n = (int)n;
    E.S = S;
    E.ppot = ppot;
    E.q = q;
    E.mode = EPI_ENERGY | EPI_UC_ONLY | (share ? EPI_POT_SHARE : 0u);
    E.eblk = eblk;
    E.flags = flags_ptr();
    if (!E.flags) return fail(CB_EHIP, "coulomb_energy: device flag symbol not found");
    const int nb = epilogue_blocks(E);
    if ((rc = launch_epilogue(E, (unsigned)nb, st))) return rc;
    k_energy_final<<<1, kEpiThreads, 0, st>>>(nb, eblk, u_out, REC_UC);
    if ((rc = check_launch("k_energy_final"))) return rc;
    return ok();
}

cb_status coulomb_trap_grad(int64_t n, const double* x, const double* y, const double* z, const double* q,
                            const double* m, const cb_trap* trap, double t, double eps2, int32_t prec, double* gx,
                            double* gy, double* gz, double* u_out, void* ws, size_t ws_bytes, void* stream) {
    const WsLayout L = ws_layout(CB_OP_GRAD, n > 0 ? n : 1, 1, 1, prec);
    cb_status rc = check_common("coulomb_trap_grad", n, prec, eps2, ws, ws_bytes, L.total);
    if (rc) return rc;
    if (prec == CB_MIXED_F32D) return fail(CB_EUNSUPPORTED, "coulomb_trap_grad: CB_MIXED_F32D is for the forces only");
    if (!x || !y || !z || !q) return fail(CB_EINVAL, "coulomb_trap_grad: NULL input array");
    const bool want_g = gx || gy || gz;
    if (want_g && !(gx && gy && gz)) return fail(CB_EINVAL, "coulomb_trap_grad: gx, gy, gz must all be set or all NULL");
    if (!want_g && !u_out) return fail(CB_EINVAL, "coulomb_trap_grad: nothing to compute (no gradient, no energy)");
    if (m && !trap_ok(trap, "coulomb_trap_grad", &rc)) return rc;
    if (!std::isfinite(t)) return fail(CB_EINVAL, "coulomb_trap_grad: t must be finite");
    const void* in[5] = {x, y, z, q, m};
    double* outs[3] = {gx, gy, gz};
    for (auto o : outs)
        for (auto i : in)
            if (overlaps(o, i, n)) return fail(CB_EINVAL, "coulomb_trap_grad: output aliases an input");
    if (want_g && (overlaps(gx, gy, n) || overlaps(gx, gz, n) || overlaps(gy, gz, n)))
        return fail(CB_EINVAL, "coulomb_trap_grad: outputs overlap");
    for (auto o : outs)
        if (u_out && overlaps2(o, n, u_out, 1)) return fail(CB_EINVAL, "coulomb_trap_grad: u_out aliases an output");
    hipStream_t st = static_cast<hipStream_t>(stream);
    EpiParams E{};
    E.n = (int)n;
    E.q = q;
    E.m = m;
    E.x = const_cast<double*>(x);  // read only in these modes
    E.y = const_cast<double*>(y);
    E.z = const_cast<double*>(z);
    if (m) E.trap = *trap;
    E.t0 = t;
    E.fx = gx;
    E.fy = gy;
    E.fz = gz;
    E.eblk = at(ws, L.eblk);
    E.flags = flags_ptr();
    if (!E.flags) return fail(CB_EHIP, "coulomb_trap_grad: device flag symbol not found");
    E.mode = (want_g ? EPI_GRAD : 0u) | (u_out ? (EPI_ENERGY | EPI_UPOT) : 0u);
    if (u_out) {
        // forces and potentials in one pass, with the energy's configuration
        int S = 0;
        bool prescaled = false;
        if ((rc = force_stage(CB_OP_ENERGY, prec, n, x, y, z, q, eps2, ws, L, st, &S, &prescaled, true))) return rc;
        E.S = S;
        E.part = at(ws, L.part);
        E.ppot = at(ws, L.ppot);
        if (prescaled) E.mode |= EPI_PRESCALED | EPI_POT_SHARE;
    } else {
        int S = 0;
        bool prescaled = false;
        if ((rc = force_stage(CB_OP_FORCES, prec, n, x, y, z, q, eps2, ws, L, st, &S, &prescaled))) return rc;
        E.S = S;
        E.part = at(ws, L.part);
        if (prescaled) E.mode |= EPI_PRESCALED;
    }
    const int nb = epilogue_blocks(E);
    if ((rc = launch_epilogue(E, (unsigned)nb, st))) return rc;
    if (u_out) {
        k_energy_final<<<1, kEpiThreads, 0, st>>>(nb, E.eblk, u_out, REC_UPOT);
        if ((rc = check_launch("k_energy_final"))) return rc;
    }
    return ok();
}

cb_status md_step(int64_t n, const cb_state* s, const double* q, const double* m, const cb_trap* trap, double t,
                  double dt, double eps2, int32_t prec, void* ws, size_t ws_bytes, void* stream) {
    const WsLayout L = ws_layout(CB_OP_MD_STEP, n > 0 ? n : 1, 1, 1, prec);
    cb_status rc = check_common("md_step", n, prec, eps2, ws, ws_bytes, L.total);
    if (rc) return rc;
    if (prec == CB_MIXED_F32D) return fail(CB_EUNSUPPORTED, "md_step: CB_MIXED_F32D is for the forces only");
    if (!(dt > 0.0) || !std::isfinite(dt) || !std::isfinite(t)) return fail(CB_EINVAL, "md_step: need finite t and dt > 0");
    if (!trap_ok(trap, "md_step", &rc)) return rc;
    if (!state_ok(s, n, q, m, "md_step", &rc)) return rc;
    return md_single(n, s, q, m, trap, t, dt, 1, eps2, prec, 0u, nullptr, 0, ws, CB_OP_MD_STEP,
                     static_cast<hipStream_t>(stream));
}

cb_status md_run(int32_t nrun, const int64_t* offsets, const cb_state* s, const double* q, const double* m,
                 const cb_trap* traps, double t0, double dt, int64_t nsteps, double eps2, int32_t prec,
                 uint32_t flags, double* energies, int64_t every, void* ws, size_t ws_bytes, void* stream) {
    if (nrun < 1 || !offsets) return fail(CB_EINVAL, "md_run: need nrun >= 1 and host offsets");
    if (offsets[0] != 0) return fail(CB_EINVAL, "md_run: offsets[0] must be 0");
    for (int r = 0; r < nrun; ++r)
        if (offsets[r + 1] <= offsets[r]) return fail(CB_EINVAL, "md_run: offsets must increase strictly");
    const int64_t n = offsets[nrun];
    const WsLayout L = ws_layout(CB_OP_MD_RUN, n, nrun, 1, prec);
    cb_status rc = check_common("md_run", n, prec, eps2, ws, ws_bytes, L.total);
    if (rc) return rc;
    if (prec == CB_MIXED_F32D) return fail(CB_EUNSUPPORTED, "md_run: CB_MIXED_F32D is for the forces only");
    if (!(dt > 0.0) || !std::isfinite(dt) || !std::isfinite(t0)) return fail(CB_EINVAL, "md_run: need finite t0 and dt > 0");
    if (nsteps < 0) return fail(CB_EINVAL, "md_run: nsteps < 0");
    if (energies && every < 1) return fail(CB_EINVAL, "md_run: every must be >= 1 when energies are requested");
    if (flags & ~CB_INIT_ACCEL) return fail(CB_EINVAL, "md_run: unknown flags 0x%x", flags);
    if (!traps) return fail(CB_EINVAL, "md_run: traps is NULL");
    for (int r = 0; r < nrun; ++r)
        if (!trap_ok(&traps[r], "md_run", &rc)) return rc;
    if (!state_ok(s, n, q, m, "md_run", &rc)) return rc;
    if (energies) {
        const int64_t nrec = nsteps / every + 1;
        double* arr[9] = {s->x, s->y, s->z, s->vx, s->vy, s->vz, s->ax, s->ay, s->az};
        for (auto a : arr)
            if (overlaps2(a, n, energies, 4 * nrec * nrun))
                return fail(CB_EINVAL, "md_run: energies overlaps the state");
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (nrun > 1)
        return md_run_batched(nrun, offsets, s, q, m, traps, t0, dt, nsteps, eps2, prec, flags, energies, every, ws,
                              ws_bytes, st);
    return md_single(n, s, q, m, &traps[0], t0, dt, nsteps, eps2, prec, flags, energies, every, ws, CB_OP_MD_RUN, st);
}

}  // extern "C"
