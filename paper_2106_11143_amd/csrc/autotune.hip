// Autotuner: times the candidate launch configurations (i-particles per lane,
// workgroup size, j-splits) of the all-pairs kernels on synthetic inputs of
// the requested size, keeps the fastest in the in-process table (keyed by
// operation, precision and power-of-two size bucket) and optionally appends
// it to a JSON-lines cache that cb_load_tuning reads back.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "internal.hpp"

namespace cb {

namespace {

struct DevBuf {
    void* p = nullptr;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
};

std::string arch_name() {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
    std::string a = prop.gcnArchName;
    return a.substr(0, a.find(':'));
}

// Synthetic ions: a Gaussian cloud from a fixed linear congruential stream
// (the values only need to be realistic, not random-quality).
void make_inputs(int64_t n, std::vector<double>& h) {
    h.resize(4 * (size_t)n);
    uint64_t s = 0x2106111430ULL;
    auto u01 = [&]() {
        s = s * 6364136223846793005ULL + 1442695040888963407ULL;
        return ((s >> 11) + 0.5) * (1.0 / 9007199254740992.0);
    };
    for (int64_t i = 0; i < n; ++i) {
        for (int c = 0; c < 3; ++c) {
            const double g = std::sqrt(-2.0 * std::log(u01())) * std::cos(6.283185307179586 * u01());
            h[c * (size_t)n + i] = 20e-6 * g;
        }
        h[3 * (size_t)n + i] = 1.602176634e-19;
    }
}

}  // namespace

}  // namespace cb

using namespace cb;

extern "C" {

cb_status cb_autotune(int32_t op, int64_t n, int32_t prec, const char* cache_path) {
    if (prec == CB_MIXED_F32D) return fail(CB_EUNSUPPORTED, "cb_autotune: CB_MIXED_F32D is an ablation, not tuned");
    if (op < 0 || op > CB_OP_ADJOINT || n < 2 || n > (int64_t(1) << 26) || prec < CB_FP64 || prec > CB_FP32_RSQ)
        return fail(CB_EINVAL, "cb_autotune: bad argument");
    const bool hv = (op == CB_OP_HVP || op == CB_OP_ADJOINT);
    const bool energy_only = (op == CB_OP_ENERGY);
    std::vector<double> h;
    make_inputs(n, h);
    DevBuf in, part, v;
    const size_t part_bytes = sizeof(double) * (size_t)kMaxSplits * 3 * (size_t)n;
    if (hipMalloc(&in.p, sizeof(double) * h.size()) != hipSuccess || hipMalloc(&part.p, part_bytes) != hipSuccess ||
        (hv && hipMalloc(&v.p, sizeof(double) * 3 * (size_t)n) != hipSuccess))
        return fail(CB_EHIP, "cb_autotune: allocation failed");
    if (hipMemcpy(in.p, h.data(), sizeof(double) * h.size(), hipMemcpyHostToDevice) != hipSuccess ||
        (hv && hipMemcpy(v.p, h.data(), sizeof(double) * 3 * (size_t)n, hipMemcpyHostToDevice) != hipSuccess))
        return fail(CB_EHIP, "cb_autotune: upload failed");
    const double* x = static_cast<const double*>(in.p);
    const double *y = x + n, *z = x + 2 * n, *q = x + 3 * n;
    hipStream_t st;
    if (hipStreamCreate(&st) != hipSuccess) return fail(CB_EHIP, "cb_autotune: stream creation failed");
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        (void)hipStreamDestroy(st);
        return fail(CB_EHIP, "cb_autotune: event creation failed");
    }
    const int ps_force[] = {1, 2, 4}, ps_hvp[] = {1, 2};
    const int wgs[] = {64, 128, 256};
    const int splits[] = {1, 2, 4, 8, 16, 24, 32, 48, 64};
    LaunchCfg best{0, 0, 0, 1, ALGO_DIRECT};
    float best_ms = 1e30f;
    cb_status rc = CB_OK;
    const int np = hv ? 2 : 3;
    for (int ip = 0; ip < np && rc == CB_OK; ++ip)
        for (int wg : wgs)
            for (int sp : splits) {
                const int p = hv ? ps_hvp[ip] : ps_force[ip];
                if (sp > 1 && n / sp < 64) continue;
                LaunchCfg c{p, wg, sp, 1, ALGO_DIRECT};
                const int jlen = split_len(n, sp);
                auto launch = [&]() -> cb_status {
                    if (hv)
                        return launch_hvp(prec, c, 1, (int)n, x, y, z, q, static_cast<const double*>(v.p), 0.0,
                                          jlen, static_cast<double*>(part.p), st);
                    return launch_pair(prec, c, !energy_only, energy_only, (int)n, x, y, z, q, 0.0, jlen,
                                       energy_only ? nullptr : static_cast<double*>(part.p),
                                       energy_only ? static_cast<double*>(part.p) : nullptr, st);
                };
                if ((rc = launch())) break;
                const int reps = 3;
                (void)hipEventRecord(e0, st);
                for (int r = 0; r < reps && rc == CB_OK; ++r) rc = launch();
                (void)hipEventRecord(e1, st);
                if (rc || hipEventSynchronize(e1) != hipSuccess) {
                    if (!rc) rc = fail(CB_EHIP, "cb_autotune: timing failed");
                    break;
                }
                float ms = 0.f;
                (void)hipEventElapsedTime(&ms, e0, e1);
                ms /= reps;
                if (ms < best_ms) {
                    best_ms = ms;
                    best = c;
                }
            }
    // the Newton's-third-law kernel (forces only, n <= kSymMaxN)
    const bool force_op = (op == CB_OP_FORCES || op == CB_OP_MD_STEP || op == CB_OP_MD_RUN);
    if (rc == CB_OK && force_op && n <= kSymMaxN) {
        size_t need = 0;
        for (int p : kSymP)
            for (int jl : kSymJL)
                need = std::max({need, sym_ws_bytes(n, p, jl), sym_ws_bytes(n, p, jl, false, kSymRows)});
        DevBuf sws, F;
        if (hipMalloc(&sws.p, need) != hipSuccess || hipMalloc(&F.p, sizeof(double) * 3 * (size_t)n) != hipSuccess)
            rc = fail(CB_EHIP, "cb_autotune: allocation failed");
        for (int algo : {ALGO_SYM, ALGO_SYM_LDS, ALGO_SYM_ROWS})
        for (int p : kSymP)
            for (int jl : kSymJL) {
                if (rc) break;
                if (algo == ALGO_SYM_ROWS && !sym_rows_p_ok(p)) continue;
                LaunchCfg c{p, kSymGroup, jl, 1, algo};
                auto launch = [&]() {
                    return launch_pair_sym(prec, c, (int)n, x, y, z, q, 0.0, sws.p, static_cast<double*>(F.p), st);
                };
                if ((rc = launch())) break;
                const int reps = 3;
                (void)hipEventRecord(e0, st);
                for (int r = 0; r < reps && rc == CB_OK; ++r) rc = launch();
                (void)hipEventRecord(e1, st);
                if (rc || hipEventSynchronize(e1) != hipSuccess) {
                    if (!rc) rc = fail(CB_EHIP, "cb_autotune: timing failed");
                    break;
                }
                float ms = 0.f;
                (void)hipEventElapsedTime(&ms, e0, e1);
                ms /= reps;
                if (ms < best_ms) {
                    best_ms = ms;
                    best = c;
                }
            }
        (void)hipStreamSynchronize(st);
    }
    // md_step / md_run of at most kSmallRunMax ions: whole steps (md_run on
    // the synthetic cloud at rest) of the two-launch step with the best force
    // configuration and of the one-launch step for each j-part count; the
    // faster is kept for the md calls.
    const bool md_op = (op == CB_OP_MD_STEP || op == CB_OP_MD_RUN);
    LaunchCfg md_best = best;
    float md_ms = 1e30f;
    if (rc == CB_OK && md_op && n <= kSmallRunMax) {
        DevBuf state, mass, mws;
        const size_t need = cb_workspace_size(CB_OP_MD_RUN, n, 1, 1, prec);
        if (hipMalloc(&state.p, sizeof(double) * 9 * (size_t)n) != hipSuccess ||
            hipMalloc(&mass.p, sizeof(double) * (size_t)n) != hipSuccess || hipMalloc(&mws.p, need) != hipSuccess)
            rc = fail(CB_EHIP, "cb_autotune: allocation failed");
        std::vector<double> hs(9 * (size_t)n, 0.0), hm((size_t)n, 6.6421562664e-26);  // at rest, 40 u
        std::copy(h.begin(), h.begin() + 3 * (size_t)n, hs.begin());
        if (!rc && (hipMemcpy(state.p, hs.data(), sizeof(double) * hs.size(), hipMemcpyHostToDevice) != hipSuccess ||
                    hipMemcpy(mass.p, hm.data(), sizeof(double) * (size_t)n, hipMemcpyHostToDevice) != hipSuccess))
            rc = fail(CB_EHIP, "cb_autotune: upload failed");
        double* sp = static_cast<double*>(state.p);
        const cb_state s9{sp, sp + n, sp + 2 * n, sp + 3 * n, sp + 4 * n, sp + 5 * n, sp + 6 * n, sp + 7 * n, sp + 8 * n};
        cb_trap tr{};
        tr.wx = tr.wy = 6.283185307179586e6;
        tr.wz = 1.2566370614359172e6;
        const int64_t offs[2] = {0, n};
        std::vector<LaunchCfg> cands{best};
        for (int S = 1; S <= kSmallPartsMax && (S == 1 || n / S >= 16); S *= 2) cands.push_back({1, 64, S, 1, ALGO_SMALL});
        for (const LaunchCfg& c : cands) {
            if (rc) break;
            put_cfg(CB_OP_MD_RUN, n, prec, c);
            auto launch = [&]() {
                return md_run(1, offs, &s9, q, static_cast<const double*>(mass.p), &tr, 0.0, 1e-9, 8, 0.0, prec,
                              CB_INIT_ACCEL, nullptr, 0, mws.p, need, st);
            };
            if ((rc = launch())) break;
            (void)hipEventRecord(e0, st);
            rc = launch();
            (void)hipEventRecord(e1, st);
            if (rc || hipEventSynchronize(e1) != hipSuccess) {
                if (!rc) rc = fail(CB_EHIP, "cb_autotune: timing failed");
                break;
            }
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            if (ms < md_ms) {
                md_ms = ms;
                md_best = c;
            }
        }
        drop_cfg(CB_OP_MD_RUN, n, prec);
        (void)hipStreamSynchronize(st);
    }
    (void)hipStreamSynchronize(st);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipStreamDestroy(st);
    if (rc) return rc;
    if (best.p == 0) return fail(CB_EHIP, "cb_autotune: no candidate ran");
    // forces, md_step and md_run share the force kernel; md_step and md_run
    // of at most kSmallRunMax ions get the faster whole step
    if (op == CB_OP_FORCES || md_op) {
        put_cfg(CB_OP_FORCES, n, prec, best);
        if (md_op || n > kSmallRunMax) {
            put_cfg(CB_OP_MD_STEP, n, prec, md_best);
            put_cfg(CB_OP_MD_RUN, n, prec, md_best);
        }
    } else if (hv) {
        put_cfg(CB_OP_HVP, n, prec, best);
        put_cfg(CB_OP_ADJOINT, n, prec, best);
    } else {
        put_cfg(op, n, prec, best);
    }
    if (cache_path) {
        FILE* f = std::fopen(cache_path, "a");
        if (!f) return fail(CB_EINVAL, "cb_autotune: cannot open %s", cache_path);
        auto line = [&](int o, const LaunchCfg& c, float ms) {
            std::fprintf(f,
                         "{\"arch\": \"%s\", \"op\": %d, \"prec\": %d, \"bucket\": %d, \"n\": %lld, \"p\": %d, "
                         "\"wg\": %d, \"splits\": %d, \"algo\": %d, \"ms\": %.6f}\n",
                         arch_name().c_str(), o, prec, n_bucket(n), (long long)n, c.p, c.wg, c.splits, c.algo, ms);
        };
        line(op, best, best_ms);
        if (md_op && n <= kSmallRunMax) line(CB_OP_MD_RUN, md_best, md_ms);
        std::fclose(f);
    }
    return ok();
}

cb_status cb_load_tuning(const char* cache_path) {
    if (!cache_path) return fail(CB_EINVAL, "cb_load_tuning: path is NULL");
    FILE* f = std::fopen(cache_path, "r");
    if (!f) return ok();
    const std::string arch = arch_name();
    char line[512];

    while (std::fgets(line, sizeof line, f)) {
        char a[64] = {0};
        int op, prec, bucket, p, wg, sp, algo = 0;
        long long n;
        if (std::sscanf(line,
                        "{\"arch\": \"%63[^\"]\", \"op\": %d, \"prec\": %d, \"bucket\": %d, \"n\": %lld, \"p\": %d, "
                        "\"wg\": %d, \"splits\": %d, \"algo\": %d",
                        a, &op, &prec, &bucket, &n, &p, &wg, &sp, &algo) < 8)
            continue;
        if (arch != a || op < 0 || op > CB_OP_ADJOINT || prec < 0 || prec > CB_MIXED_F32D || n < 1 ||
            n > kMaxIons)
            continue;
        LaunchCfg c{p, wg, sp, 1, algo};
        if (!valid_cfg(op, c)) continue;
        if (op == CB_OP_FORCES || op == CB_OP_MD_STEP || op == CB_OP_MD_RUN) {
            // as cb_autotune: a forces line also sets the md calls above
            // kSmallRunMax ions; an md line sets the md calls (and forces,
            // unless it is the one-launch step)
            const bool md_line = op != CB_OP_FORCES;
            if (c.algo == ALGO_SMALL && n > kSmallRunMax) continue;
            if (c.algo != ALGO_SMALL) put_cfg(CB_OP_FORCES, n, prec, c);
            if (md_line || n > kSmallRunMax) {
                put_cfg(CB_OP_MD_STEP, n, prec, c);
                put_cfg(CB_OP_MD_RUN, n, prec, c);
            }
        } else if (op == CB_OP_HVP || op == CB_OP_ADJOINT) {
            put_cfg(CB_OP_HVP, n, prec, c);
            put_cfg(CB_OP_ADJOINT, n, prec, c);
        } else {
            put_cfg(op, n, prec, c);
        }

    }
    std::fclose(f);
    return ok();
}

}  // extern "C"
