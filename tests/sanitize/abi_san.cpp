// Sanitizer driver for the host side of the C ABI (test infrastructure):
// built host-only with AddressSanitizer and UndefinedBehaviorSanitizer
// together with the library's sources, it runs every path that needs no GPU
// (workspace sizing, launch-configuration table and tuning-file parsing,
// trap constants, and each entry point's argument checks) with ordinary,
// extreme and malformed arguments.  Exit status 0 and the line
// "abi_san ok" mean no report and every status as expected.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "coulomb.h"

static int g_bad = 0;

static void expect(bool okk, const char* what) {
    if (!okk) {
        std::printf("FAILED: %s (last error: %s)\n", what, cb_last_error());
        ++g_bad;
    }
}

int main(int argc, char** argv) {
    const char* tmpdir = argc > 1 ? argv[1] : "/tmp";
    const int64_t sizes[] = {-5, 0, 1, 2, 63, 64, 65, 1000, 4096, 16383, 16384, 100000, 131072, 262144, 262145,
                             2796202, 3000000, (int64_t)1 << 40, INT64_MAX};
    // workspace sizes: every op, precision and size, including the rejected ones
    for (int op = -1; op <= 8; ++op)
        for (int prec = -1; prec <= 5; ++prec)
            for (int64_t n : sizes)
                for (int nv : {0, 1, 8, 64})
                    (void)cb_workspace_size(op, n, 2, nv, prec);
    expect(cb_workspace_size(CB_OP_FORCES, 100000, 1, 1, CB_FP64) > 0, "forces workspace at 1e5");
    expect(cb_workspace_size(CB_OP_FORCES, 0, 1, 1, CB_FP64) == 0, "workspace at n = 0");

    // the launch-configuration table
    int32_t cfg[5];
    for (int op = -1; op <= 8; ++op)
        for (int prec = -1; prec <= 5; ++prec)
            for (int64_t n : sizes) {
                (void)cb_get_config(op, n, prec, cfg);
                (void)cb_set_config(op, n, prec, 2, 8, 4, 512);
                (void)cb_set_config(op, n, prec, 0, 2, 128, 7);
                (void)cb_set_config(op, n, prec, 2, 3, 9, 100);
                (void)cb_set_config(op, n, prec, 0, 0, 0, 0);
            }
    expect(cb_get_config(CB_OP_FORCES, 1000, CB_FP64, nullptr) == CB_EINVAL, "get_config NULL out");
    expect(cb_set_config(CB_OP_FORCES, 5000, CB_FP64, 0, 3, 256, 1) == CB_EINVAL, "set_config bad p");
    expect(cb_set_config(CB_OP_FORCES, 5000, CB_FP64, 0, 2, 128, 7) == CB_OK, "set_config good");
    expect(cb_get_config(CB_OP_FORCES, 5000, CB_FP64, cfg) == CB_OK && cfg[1] == 2 && cfg[3] == 7,
           "get_config returns what was set");

    // tuning files: missing, malformed and extreme lines
    expect(cb_load_tuning(nullptr) == CB_EINVAL, "load_tuning NULL");
    expect(cb_load_tuning("/nonexistent/dir/none.jsonl") == CB_OK, "load_tuning missing file");
    char path[512];
    std::snprintf(path, sizeof path, "%s/abi_san_tuning.jsonl", tmpdir);
    if (FILE* f = std::fopen(path, "w")) {
        std::fputs("not json at all\n{\"arch\": \"unknown\"\n", f);
        std::fprintf(f, "{\"arch\": \"%s\", \"op\": %d, \"prec\": %d, \"bucket\": %d, \"n\": %lld, \"p\": 2, "
                        "\"wg\": 128, \"splits\": 7, \"algo\": 0}\n", "unknown", 0, 0, 13, 5000LL);
        std::fprintf(f, "{\"arch\": \"%s\", \"op\": %d, \"prec\": %d, \"bucket\": %d, \"n\": %lld, \"p\": 2, "
                        "\"wg\": 128, \"splits\": 7, \"algo\": 0}\n", "unknown", 1, -7, -1, 9223372036854775807LL);
        std::fprintf(f, "{\"arch\": \"%s\", \"op\": %d, \"prec\": %d, \"bucket\": %d, \"n\": %lld, \"p\": 2, "
                        "\"wg\": 128, \"splits\": 7, \"algo\": 0}\n", "unknown", 99, 99, 99, -3LL);
        std::string longline(2000, 'x');
        std::fputs(longline.c_str(), f);
        std::fputs("\n", f);
        std::fclose(f);
        expect(cb_load_tuning(path) == CB_OK, "load_tuning malformed file");
        std::remove(path);
    }

    // trap constants
    double k[3];
    cb_trap tr{};
    tr.kind = 0; tr.wx = 2e6; tr.wy = 2.1e6; tr.wz = 3e5;
    expect(cb_trap_k(&tr, 0.0, k) == CB_OK && std::fabs(k[0] - 4e12) < 1e-3, "trap_k static");
    tr.wx1 = 1e6; tr.wy1 = 1e6; tr.t_ramp0 = 0.0; tr.t_ramp1 = 1e-6;
    expect(cb_trap_k(&tr, 5e-7, k) == CB_OK, "trap_k ramp");
    cb_trap rf{};
    rf.kind = 1; rf.wz = 3e5; rf.rf_a = -1e-3; rf.rf_q = 0.2; rf.rf_omega = 2e7; rf.rf_phase = 0.3;
    expect(cb_trap_k(&rf, 1e-7, k) == CB_OK, "trap_k rf");
    expect(cb_trap_k(nullptr, 0.0, k) == CB_EINVAL, "trap_k NULL trap");
    expect(cb_trap_k(&tr, 0.0, nullptr) == CB_EINVAL, "trap_k NULL out");
    cb_trap badk{};
    badk.kind = 7;
    expect(cb_trap_k(&badk, 0.0, k) == CB_EINVAL, "trap_k bad kind");
    cb_trap nan_t = tr;
    nan_t.wx = NAN;
    expect(cb_trap_k(&nan_t, 0.0, k) == CB_EINVAL, "trap_k NaN frequency");

    // argument checks of the compute entries (every call returns before any launch)
    std::vector<double> buf(64 * 40, 0.0);
    double* P = buf.data();
    double *A = P, *B = P + 64, *Cc = P + 128, *D = P + 192, *E = P + 256, *F = P + 320, *G = P + 384;
    double *H = P + 448, *I = P + 512, *J = P + 576;
    std::vector<char> wsv(1 << 16);
    void* ws = wsv.data();
    const size_t big = (size_t)1 << 40;
    expect(coulomb_forces(0, A, B, Cc, D, 0.0, 0, E, F, G, ws, big, nullptr) == CB_EINVAL, "forces n = 0");
    expect(coulomb_forces(-3, A, B, Cc, D, 0.0, 0, E, F, G, ws, big, nullptr) == CB_EINVAL, "forces n < 0");
    expect(coulomb_forces(10, A, B, Cc, D, 0.0, 9, E, F, G, ws, big, nullptr) == CB_EINVAL, "forces bad prec");
    expect(coulomb_forces(10, A, B, Cc, D, -1.0, 0, E, F, G, ws, big, nullptr) == CB_EINVAL, "forces eps2 < 0");
    expect(coulomb_forces(10, A, B, Cc, D, NAN, 0, E, F, G, ws, big, nullptr) == CB_EINVAL, "forces eps2 NaN");
    expect(coulomb_forces(10, nullptr, B, Cc, D, 0.0, 0, E, F, G, ws, big, nullptr) == CB_EINVAL, "forces NULL x");
    expect(coulomb_forces(10, A, B, Cc, D, 0.0, 0, E, F, G, ws, 100, nullptr) == CB_ENOWS, "forces small ws");
    expect(coulomb_forces(10, A, B, Cc, D, 0.0, 0, A, F, G, ws, big, nullptr) == CB_EINVAL, "forces alias");
    expect(coulomb_forces(INT64_MAX, A, B, Cc, D, 0.0, 0, E, F, G, ws, big, nullptr) != CB_OK, "forces huge n");
    expect(coulomb_forces_noalloc(0, A, B, Cc, D, 0.0, 0, E, F, G, nullptr) == CB_EINVAL, "noalloc n = 0");
    expect(coulomb_forces_noalloc(3000000, A, B, Cc, D, 0.0, 0, E, F, G, nullptr) != CB_OK, "noalloc beyond scratch");
    expect(coulomb_forces_noalloc(INT64_MAX, A, B, Cc, D, 0.0, 0, E, F, G, nullptr) != CB_OK, "noalloc huge n");
    expect(coulomb_forces_range(10, 5, 3, A, B, Cc, D, 0.0, 0, E, F, G, ws, big, nullptr) == CB_EINVAL,
           "range i0 > i1");
    expect(coulomb_forces_range(10, 0, 11, A, B, Cc, D, 0.0, 0, E, F, G, ws, big, nullptr) == CB_EINVAL,
           "range i1 > n");
    expect(coulomb_forces_range(10, -1, 4, A, B, Cc, D, 0.0, 0, E, F, G, ws, big, nullptr) == CB_EINVAL,
           "range i0 < 0");
    int32_t splits = 0;
    expect(coulomb_pair_stage(0, A, B, Cc, D, 0.0, 0, &splits, ws, big, nullptr) == CB_EINVAL, "pair_stage n = 0");
    double u = 0.0;
    expect(coulomb_energy(10, A, B, Cc, D, 0.0, 0, nullptr, ws, big, nullptr) == CB_EINVAL, "energy NULL out");
    expect(coulomb_energy(0, A, B, Cc, D, 0.0, 0, &u, ws, big, nullptr) == CB_EINVAL, "energy n = 0");
    expect(coulomb_trap_grad(10, A, B, Cc, D, E, nullptr, 0.0, 0.0, 0, F, G, H, &u, ws, big, nullptr) == CB_EINVAL,
           "trap_grad NULL trap");
    expect(coulomb_trap_grad(10, A, B, Cc, D, E, &badk, 0.0, 0.0, 0, F, G, H, &u, ws, big, nullptr) == CB_EINVAL,
           "trap_grad bad kind");
    cb_state s{A, B, Cc, E, F, G, H, I, J};
    expect(md_step(10, &s, D, D, &tr, 0.0, 0.0, 0.0, 0, ws, big, nullptr) == CB_EINVAL, "md_step dt = 0");
    expect(md_step(10, nullptr, D, D, &tr, 0.0, 1e-9, 0.0, 0, ws, big, nullptr) == CB_EINVAL, "md_step NULL state");
    cb_state s2{A, A, A, A, A, A, A, A, A};
    expect(md_step(10, &s2, D, D, &tr, 0.0, 1e-9, 0.0, 0, ws, big, nullptr) == CB_EINVAL, "md_step aliased state");
    int64_t offs[3] = {0, 5, 4};
    cb_trap trs[2] = {tr, tr};
    expect(md_run(2, offs, &s, D, D, trs, 0.0, 1e-9, 10, 0.0, 0, 1, nullptr, 0, ws, big, nullptr) == CB_EINVAL,
           "md_run decreasing offsets");
    expect(md_run(0, offs, &s, D, D, trs, 0.0, 1e-9, 10, 0.0, 0, 1, nullptr, 0, ws, big, nullptr) == CB_EINVAL,
           "md_run no runs");
    expect(md_run(1, nullptr, &s, D, D, trs, 0.0, 1e-9, 10, 0.0, 0, 1, nullptr, 0, ws, big, nullptr) == CB_EINVAL,
           "md_run NULL offsets");
    expect(md_run(1, offs, &s, D, D, trs, 0.0, 1e-9, -1, 0.0, 0, 1, nullptr, 0, ws, big, nullptr) == CB_EINVAL,
           "md_run negative steps");
    expect(coulomb_hvp(10, A, B, Cc, D, 0, E, F, nullptr, nullptr, 0.0, 0.0, 0, ws, big, nullptr) == CB_EINVAL,
           "hvp nvec = 0");
    expect(coulomb_hvp(10, A, B, Cc, D, 1000, E, F, nullptr, nullptr, 0.0, 0.0, 0, ws, big, nullptr) == CB_EINVAL,
           "hvp nvec too large");
    expect(coulomb_hvp(10, A, B, Cc, D, 1, E, E, nullptr, nullptr, 0.0, 0.0, 0, ws, big, nullptr) == CB_EINVAL,
           "hvp alias");
    expect(md_adjoint_step(10, A, B, Cc, D, E, &tr, 1e-9, 0.0, 0, 0, nullptr, F, ws, big, nullptr) == CB_EINVAL,
           "adjoint NULL lambda");
    expect(cb_poll_flags(nullptr, nullptr) == CB_EINVAL, "poll_flags NULL");
    expect(cb_autotune(-1, 1000, 0, nullptr) != CB_OK, "autotune bad op");
    expect(std::strlen(cb_last_error()) > 0, "last error text");

    if (g_bad) {
        std::printf("abi_san: %d check(s) failed\n", g_bad);
        return 1;
    }
    std::printf("abi_san ok\n");
    return 0;
}
