/*
 * The oracle's timed variant: the paper's classical all-pairs double loop
 * (section 3), in FP64 with SQRT+DIV, the self pair skipped, no compensation,
 * OpenMP static partition of the i loop inside one parallel region
 * (section 6.3), built -O3 -march=native so the compiler vectorises it as it
 * sees fit (the paper's "compiler-optimised" baseline).
 *
 * TEST INFRASTRUCTURE ONLY: used as the CPU baseline that the GPU throughput
 * is reported beside, never by the product path.  The accuracy reference is
 * or_forces in coulomb_oracle.c, not this function.
 */
#include <math.h>
#include <stdint.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORP_PI 3.14159265358979323846
static const double ORP_EPS0 = 8.8541878128e-12; /* F/m, CODATA 2018 */

/* Sum over j of q_j (r_i - r_j) / (|r_i - r_j|^2 + eps2)^{3/2} for j in
 * [j0, j1), added to acc[3]: one square root and one division per pair. */
static inline void orp_row(const double* x, const double* y, const double* z, const double* q, double eps2,
                           double xi, double yi, double zi, int64_t j0, int64_t j1, double acc[3]) {
    double sx = 0.0, sy = 0.0, sz = 0.0;
    for (int64_t j = j0; j < j1; ++j) {
        const double dx = xi - x[j], dy = yi - y[j], dz = zi - z[j];
        const double r2 = dx * dx + dy * dy + dz * dz + eps2;
        const double inv_r = 1.0 / sqrt(r2);
        const double s = q[j] * (inv_r * inv_r * inv_r);
        sx += dx * s;
        sy += dy * s;
        sz += dz * s;
    }
    acc[0] += sx;
    acc[1] += sy;
    acc[2] += sz;
}

/* Forces on ions i0 .. i1-1 against all n ions, written to f?[i - i0].
 * Returns the number of threads used. */
int orp_forces_range(int64_t n, const double* x, const double* y, const double* z, const double* q,
                     double eps2, int64_t i0, int64_t i1, double* fx, double* fy, double* fz,
                     int nthreads) {
    const double kc = 1.0 / (4.0 * ORP_PI * ORP_EPS0);
    int used = 1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel
    {
#ifdef _OPENMP
#pragma omp single
        used = omp_get_num_threads();
#endif
#pragma omp for schedule(static)
        for (int64_t i = i0; i < i1; ++i) {
            double acc[3] = {0.0, 0.0, 0.0};
            orp_row(x, y, z, q, eps2, x[i], y[i], z[i], 0, i, acc);      /* j < i */
            orp_row(x, y, z, q, eps2, x[i], y[i], z[i], i + 1, n, acc);  /* j > i: the self pair skipped */
            const double c = kc * q[i];
            fx[i - i0] = c * acc[0];
            fy[i - i0] = c * acc[1];
            fz[i - i0] = c * acc[2];
        }
    }
    return used;
}
