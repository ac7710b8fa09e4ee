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
            const double xi = x[i], yi = y[i], zi = z[i];
            double ax = 0.0, ay = 0.0, az = 0.0;
            for (int64_t j = 0; j < i; ++j) {
                double dx = xi - x[j], dy = yi - y[j], dz = zi - z[j];
                double r2inv = dx * dx + dy * dy + dz * dz + eps2;
                r2inv = 1.0 / sqrt(r2inv);
                r2inv = r2inv * r2inv * r2inv * q[j];
                ax += dx * r2inv;
                ay += dy * r2inv;
                az += dz * r2inv;
            }
            for (int64_t j = i + 1; j < n; ++j) {
                double dx = xi - x[j], dy = yi - y[j], dz = zi - z[j];
                double r2inv = dx * dx + dy * dy + dz * dz + eps2;
                r2inv = 1.0 / sqrt(r2inv);
                r2inv = r2inv * r2inv * r2inv * q[j];
                ax += dx * r2inv;
                ay += dy * r2inv;
                az += dz * r2inv;
            }
            const double c = kc * q[i];
            fx[i - i0] = c * ax;
            fy[i - i0] = c * ay;
            fz[i - i0] = c * az;
        }
    }
    return used;
}
