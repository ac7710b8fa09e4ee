/*
 * Sanitizer driver for the CPU oracle (test infrastructure): built with
 * AddressSanitizer and UndefinedBehaviorSanitizer together with the oracle's
 * own sources, it calls every entry point on small ragged inputs (the empty
 * cloud, one ion, a handful) so that an out-of-bounds index, an
 * uninitialised read or an undefined operation in the oracle stops the run
 * with a report.  Exit status 0 and the line "oracle_san ok" mean clean.
 */
#include "../../oracle/coulomb_oracle.c"
#include "../../oracle/coulomb_oracle_plain.c"

#include <stdio.h>

static double urand(uint64_t* s) {
    *s = *s * 6364136223846793005ULL + 1442695040888963407ULL;
    return (double)(*s >> 11) * (1.0 / 9007199254740992.0);
}

static void run(int64_t n, int nthreads, uint64_t seed) {
    const int64_t nn = n > 0 ? n : 1;
    double* st = calloc((size_t)(9 * nn), sizeof(double));
    double* q = calloc((size_t)nn, sizeof(double));
    double* m = calloc((size_t)nn, sizeof(double));
    double* f = calloc((size_t)(3 * nn), sizeof(double));
    double* kap = calloc((size_t)nn, sizeof(double));
    double* phi = calloc((size_t)nn, sizeof(double));
    const int nvec = 3, nsteps = 5, every = 2;
    double* v = calloc((size_t)(3 * nvec * nn), sizeof(double));
    double* hv = calloc((size_t)(3 * nvec * nn), sizeof(double));
    double* en = calloc((size_t)(4 * (nsteps / every + 1)), sizeof(double));
    double* traj = calloc((size_t)(9 * nn * nsteps), sizeof(double));
    int64_t idx[3] = {0, n > 1 ? n - 1 : 0, n > 2 ? n / 2 : 0};
    double out[4];
    for (int64_t i = 0; i < 3 * nn; ++i) st[i] = (urand(&seed) - 0.5) * 2e-5;
    for (int64_t i = 0; i < nn; ++i) {
        q[i] = 1.602176634e-19 * (i % 3 == 0 ? 2.0 : 1.0);
        m[i] = 40.0 * 1.66053906660e-27;
    }
    for (int64_t i = 0; i < 3 * nvec * nn; ++i) v[i] = urand(&seed) - 0.5;
    or_trap tr = {0, 2e6, 2.1e6, 3e5, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    or_trap rf = {1, 0, 0, 3e5, -0.001, 0.2, 2.0e7, 0.3, 0, 0, 0, 0, 0};
    or_forces(n, st, st + nn, st + 2 * nn, q, 0.0, 0, NULL, f, f + nn, f + 2 * nn, kap, nthreads);
    if (n > 0) {
        double fs[9];
        or_forces(n, st, st + nn, st + 2 * nn, q, 1e-16, 3, idx, fs, fs + 3, fs + 6, NULL, nthreads);
    }
    (void)or_coulomb_energy(n, st, st + nn, st + 2 * nn, q, 0.0, phi, nthreads);
    (void)or_trap_energy(n, st, st + nn, st + 2 * nn, m, &rf, 1e-7);
    (void)or_kinetic_energy(n, st + 3 * nn, st + 4 * nn, st + 5 * nn, m);
    or_accel(n, st, st + nn, st + 2 * nn, q, m, &rf, 1e-7, 0.0, f, f + nn, f + 2 * nn, nthreads);
    or_hvp(n, st, st + nn, st + 2 * nn, q, nvec, v, hv, m, &tr, 0.0, 0.0, nthreads);
    (void)orp_forces_range(n, st, st + nn, st + 2 * nn, q, 0.0, 0, n, f, f + nn, f + 2 * nn, nthreads);
    if (n > 0) {
        or_md_run(n, st, q, m, &rf, 0.0, 1e-9, nsteps, 0.0, 1, en, every, traj, nthreads);
        or_md_run(n, st, q, m, &tr, 0.0, 1e-9, nsteps, 0.0, 0, NULL, 0, NULL, nthreads);
        or_msd_grad(n, st, q, m, &tr, 1e-9, nsteps, 0.0, out, nthreads);
    }
    free(st); free(q); free(m); free(f); free(kap); free(phi); free(v); free(hv); free(en); free(traj);
}

int main(void) {
    const int64_t sizes[] = {0, 1, 2, 7, 33};
    for (size_t k = 0; k < sizeof sizes / sizeof sizes[0]; ++k) {
        run(sizes[k], 1, 11 + k);
        run(sizes[k], 3, 17 + k);
    }
    double kk[3];
    or_trap ramp = {0, 2e6, 2e6, 3e5, 0, 0, 0, 0, 0, 1e6, 1e6, 0.0, 1e-6};
    or_trap_k(&ramp, 5e-7, kk);
    printf("oracle_san ok\n");
    return 0;
}
