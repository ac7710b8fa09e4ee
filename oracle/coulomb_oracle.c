/*
 * Slow, plain FP64 CPU oracle for the all-pairs Coulomb force and the
 * velocity-Verlet motion of ions in a linear Paul trap.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product (the HIP library and its
 * Python binding) may include, link or call this file.  It shares no code,
 * header or constant with the GPU path; the only thing both sides share is the
 * seeded input generator, which holds none of this arithmetic.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -fPIC -shared (no fast-math, no
 * FMA contraction), so every operation below is one IEEE binary64 operation,
 * rounded to nearest-even, in the order written.
 *
 * What is computed (paper section 2, eq. (1); section 3, the classical double
 * loop):
 *   F_i = k_C q_i sum_{j != i} q_j (r_i - r_j) / (|r_i - r_j|^2 + eps2)^{3/2}
 * with 1/sqrt taken as one IEEE square root followed by one IEEE division
 * (the "SQRT+DIV" method of section 2), j ascending, the self pair skipped
 * (the double loop runs over every j; with zero softening its j = i term is
 * 0 * inf, so the equation's sum is read as excluding it), and every force
 * component accumulated with Neumaier compensation so the oracle's own
 * summation error is about one rounding of the result.
 *
 * Readings of the paper taken here:
 *  - softening is added to r^2 (as the double loop does), not inside the norm;
 *  - the trap term acts on ion i (eq. (1) prints x_j, y_j);
 *  - the RF drive is cos(Omega t + phi) with Omega in rad/s, and its amplitude
 *    2 Q V_RF / (m r0^2) is written in Mathieu form as q Omega^2 / 2, with the
 *    paper's sign: a_x = -(a Omega^2/4 + q Omega^2/2 cos(Omega t+phi)) x and
 *    a_y = -a_x-coefficient * y;
 *  - charges and masses are per ion (the paper uses one species);
 *  - velocity-Verlet as the paper's three-step list in section 2.
 *
 * Constants: CODATA 2018 vacuum permittivity; k_C = 1/(4 pi eps0).
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_PI 3.14159265358979323846
static const double OR_EPS0 = 8.8541878128e-12; /* F/m, CODATA 2018 */

double or_coulomb_constant(void) { return 1.0 / (4.0 * OR_PI * OR_EPS0); }

/* ---------------------------------------------------------------- sums -- */
/* Neumaier's improved Kahan summation: s carries the sum, c the lost low
 * order part; the value is s + c. */
typedef struct { double s, c; } or_sum;

static inline void or_add(or_sum* a, double v) {
    double t = a->s + v;
    if (fabs(a->s) >= fabs(v)) a->c += (a->s - t) + v;
    else a->c += (v - t) + a->s;
    a->s = t;
}
static inline double or_val(const or_sum* a) { return a->s + a->c; }

static void or_set_threads(int nthreads) {
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

/* --------------------------------------------------------------- trap -- */
/* Trap parameters, mirrored field by field in oracle.py.  kind 0: static
 * pseudo-potential (wx, wy, wz in rad/s), with an optional linear ramp of
 * wx, wy from (wx, wy) at t_ramp0 to (wx1, wy1) at t_ramp1 (off when
 * t_ramp1 <= t_ramp0).  kind 1: explicit RF drive in Mathieu form plus a
 * static axial well wz. */
typedef struct {
    int32_t kind;
    double wx, wy, wz;
    double rf_a, rf_q, rf_omega, rf_phase;
    double gamma;
    double wx1, wy1, t_ramp0, t_ramp1;
} or_trap;

/* Spring constants per unit mass k = (kx, ky, kz) at time t, so the trap
 * acceleration is a = -(kx x, ky y, kz z) and the trap energy of an ion is
 * m (kx x^2 + ky y^2 + kz z^2) / 2. */
void or_trap_k(const or_trap* tr, double t, double k[3]) {
    if (tr->kind == 1) {
        double w2 = tr->rf_omega * tr->rf_omega;
        double kx = tr->rf_a * w2 / 4.0 + tr->rf_q * w2 / 2.0 * cos(tr->rf_omega * t + tr->rf_phase);
        k[0] = kx;
        k[1] = -kx;
        k[2] = tr->wz * tr->wz;
        return;
    }
    double wx = tr->wx, wy = tr->wy;
    if (tr->t_ramp1 > tr->t_ramp0) {
        double s = (t - tr->t_ramp0) / (tr->t_ramp1 - tr->t_ramp0);
        if (s < 0.0) s = 0.0;
        if (s > 1.0) s = 1.0;
        wx = tr->wx + s * (tr->wx1 - tr->wx);
        wy = tr->wy + s * (tr->wy1 - tr->wy);
    }
    k[0] = wx * wx;
    k[1] = wy * wy;
    k[2] = tr->wz * tr->wz;
}

/* ------------------------------------------------------------- forces -- */
/* Forces on the ions listed in idx (all ions when idx is NULL; ni entries
 * otherwise), written to fx/fy/fz[k] for the k-th listed ion.  kappa (may be
 * NULL) receives sum_j |f_ij| / |sum_j f_ij|, the condition number of the
 * ion's force sum (vector 2-norms), which bounds how far any other summation
 * order may land from the exact sum. */
void or_forces(int64_t n, const double* x, const double* y, const double* z, const double* q,
               double eps2, int64_t ni, const int64_t* idx, double* fx, double* fy, double* fz,
               double* kappa, int nthreads) {
    const double kc = or_coulomb_constant();
    if (idx == NULL) ni = n;
    or_set_threads(nthreads);
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < ni; ++k) {
        int64_t i = idx ? idx[k] : k;
        or_sum sx = {0, 0}, sy = {0, 0}, sz = {0, 0};
        or_sum mag = {0, 0};
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double dx = x[i] - x[j];
            double dy = y[i] - y[j];
            double dz = z[i] - z[j];
            double r2 = dx * dx + dy * dy + dz * dz + eps2;
            double rinv = 1.0 / sqrt(r2);
            double s = rinv * rinv * rinv * q[j];
            double tx = dx * s, ty = dy * s, tz = dz * s;
            or_add(&sx, tx);
            or_add(&sy, ty);
            or_add(&sz, tz);
            if (kappa) or_add(&mag, sqrt(tx * tx + ty * ty + tz * tz));
        }
        double ax = or_val(&sx), ay = or_val(&sy), az = or_val(&sz);
        double c = kc * q[i];
        fx[k] = c * ax;
        fy[k] = c * ay;
        fz[k] = c * az;
        if (kappa) {
            double nrm = sqrt(ax * ax + ay * ay + az * az);
            kappa[k] = or_val(&mag) / nrm;
        }
    }
}

/* Potential phi_i = sum_{j != i} q_j (r_ij^2 + eps2)^{-1/2} (compensated) and
 * the Coulomb energy U_C = k_C/2 sum_i q_i phi_i = k_C sum_{i<j} q_i q_j / r_ij
 * (compensated over i).  phi may be NULL. */
double or_coulomb_energy(int64_t n, const double* x, const double* y, const double* z, const double* q,
                         double eps2, double* phi, int nthreads) {
    const double kc = or_coulomb_constant();
    double* p = phi ? phi : (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    or_set_threads(nthreads);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        or_sum s = {0, 0};
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double dx = x[i] - x[j];
            double dy = y[i] - y[j];
            double dz = z[i] - z[j];
            double r2 = dx * dx + dy * dy + dz * dz + eps2;
            or_add(&s, q[j] * (1.0 / sqrt(r2)));
        }
        p[i] = or_val(&s);
    }
    or_sum u = {0, 0};
    for (int64_t i = 0; i < n; ++i) or_add(&u, q[i] * p[i]);
    double out = 0.5 * kc * or_val(&u);
    if (!phi) free(p);
    return out;
}

/* Trap energy sum_i m_i (kx x^2 + ky y^2 + kz z^2) / 2 at time t. */
double or_trap_energy(int64_t n, const double* x, const double* y, const double* z, const double* m,
                      const or_trap* tr, double t) {
    double k[3];
    or_trap_k(tr, t, k);
    or_sum u = {0, 0};
    for (int64_t i = 0; i < n; ++i)
        or_add(&u, 0.5 * m[i] * (k[0] * x[i] * x[i] + k[1] * y[i] * y[i] + k[2] * z[i] * z[i]));
    return or_val(&u);
}

double or_kinetic_energy(int64_t n, const double* vx, const double* vy, const double* vz, const double* m) {
    or_sum u = {0, 0};
    for (int64_t i = 0; i < n; ++i)
        or_add(&u, 0.5 * m[i] * (vx[i] * vx[i] + vy[i] * vy[i] + vz[i] * vz[i]));
    return or_val(&u);
}

/* Total acceleration a_i = F_i / m_i - k(t) * r_i (eq. (1) without friction). */
void or_accel(int64_t n, const double* x, const double* y, const double* z, const double* q, const double* m,
              const or_trap* tr, double t, double eps2, double* ax, double* ay, double* az, int nthreads) {
    double k[3];
    or_forces(n, x, y, z, q, eps2, 0, NULL, ax, ay, az, NULL, nthreads);
    or_trap_k(tr, t, k);
    for (int64_t i = 0; i < n; ++i) {
        ax[i] = ax[i] / m[i] - k[0] * x[i];
        ay[i] = ay[i] / m[i] - k[1] * y[i];
        az[i] = az[i] / m[i] - k[2] * z[i];
    }
}

/* ----------------------------------------------------- velocity-Verlet -- */
/* Energies of one state: out[0] = kinetic, out[1] = Coulomb, out[2] = trap,
 * out[3] = their sum. */
static void or_energies(int64_t n, const double* s, const double* q, const double* m, const or_trap* tr,
                        double t, double eps2, double* out, int nthreads) {
    const double *x = s, *y = s + n, *z = s + 2 * n, *vx = s + 3 * n, *vy = s + 4 * n, *vz = s + 5 * n;
    out[0] = or_kinetic_energy(n, vx, vy, vz, m);
    out[1] = or_coulomb_energy(n, x, y, z, q, eps2, NULL, nthreads);
    out[2] = or_trap_energy(n, x, y, z, m, tr, t);
    out[3] = out[0] + out[1] + out[2];
}

/* Runs nsteps velocity-Verlet steps of constant dt from time t0 (section 2's
 * three-step list):
 *   r_{n+1} = r_n + v_n dt + dt^2/2 a_n
 *   a_{n+1} = a(r_{n+1}, t0 + (n+1) dt)
 *   v_{n+1} = v_n + dt/2 (a_n + a_{n+1})
 * With the friction term of eq. (1), -Gamma v / m (tr->gamma = Gamma > 0),
 * the velocity-dependent part is taken by the trapezoidal rule, with
 * g_i = Gamma / m_i and a the conservative (Coulomb + trap) acceleration:
 *   r_{n+1} = r_n + v_n dt + dt^2/2 (a_n - g_i v_n)
 *   v_{n+1} = (v_n (1 - g_i dt/2) + dt/2 (a_n + a_{n+1})) / (1 + g_i dt/2)
 * (the paper states the friction term but not how the integrator treats it;
 * this is the reading taken).  state's a is the conservative acceleration.
 * state holds 9 arrays of n doubles: x y z vx vy vz ax ay az, updated in
 * place.  When init_accel is set, a_0 = a(r_0, t0) is computed first;
 * otherwise the given a is a_0.  When energies is non-NULL, energies[4*k ..]
 * receives (K, U_C, U_trap, E) of step k*every for k = 0 .. nsteps/every.
 * When traj is non-NULL it receives the 9n-double state after every step
 * (nsteps blocks; block s is the state of step s+1). */
void or_md_run(int64_t n, double* state, const double* q, const double* m, const or_trap* tr, double t0,
               double dt, int64_t nsteps, double eps2, int init_accel, double* energies, int64_t every,
               double* traj, int nthreads) {
    double *x = state, *y = state + n, *z = state + 2 * n;
    double *vx = state + 3 * n, *vy = state + 4 * n, *vz = state + 5 * n;
    double *ax = state + 6 * n, *ay = state + 7 * n, *az = state + 8 * n;
    double* an = (double*)malloc(sizeof(double) * 3 * (size_t)n);
    double *anx = an, *any = an + n, *anz = an + 2 * n;
    if (init_accel) or_accel(n, x, y, z, q, m, tr, t0, eps2, ax, ay, az, nthreads);
    int64_t rec = 0;
    if (energies && every > 0) or_energies(n, state, q, m, tr, t0, eps2, energies + 4 * rec++, nthreads);
    const double hdt2 = 0.5 * dt * dt, hdt = 0.5 * dt;
    const double Gam = tr->gamma;
    for (int64_t s = 0; s < nsteps; ++s) {
        if (Gam == 0.0) {
            for (int64_t i = 0; i < n; ++i) {
                x[i] = x[i] + vx[i] * dt + hdt2 * ax[i];
                y[i] = y[i] + vy[i] * dt + hdt2 * ay[i];
                z[i] = z[i] + vz[i] * dt + hdt2 * az[i];
            }
        } else {
            for (int64_t i = 0; i < n; ++i) {
                double g = Gam / m[i];
                x[i] = x[i] + vx[i] * dt + hdt2 * (ax[i] - g * vx[i]);
                y[i] = y[i] + vy[i] * dt + hdt2 * (ay[i] - g * vy[i]);
                z[i] = z[i] + vz[i] * dt + hdt2 * (az[i] - g * vz[i]);
            }
        }
        double t1 = t0 + (double)(s + 1) * dt;
        or_accel(n, x, y, z, q, m, tr, t1, eps2, anx, any, anz, nthreads);
        if (Gam == 0.0) {
            for (int64_t i = 0; i < n; ++i) {
                vx[i] = vx[i] + hdt * (ax[i] + anx[i]);
                vy[i] = vy[i] + hdt * (ay[i] + any[i]);
                vz[i] = vz[i] + hdt * (az[i] + anz[i]);
            }
        } else {
            for (int64_t i = 0; i < n; ++i) {
                double g = Gam / m[i];
                double lo = 1.0 - g * hdt, hi = 1.0 + g * hdt;
                vx[i] = (vx[i] * lo + hdt * (ax[i] + anx[i])) / hi;
                vy[i] = (vy[i] * lo + hdt * (ay[i] + any[i])) / hi;
                vz[i] = (vz[i] * lo + hdt * (az[i] + anz[i])) / hi;
            }
        }
        for (int64_t i = 0; i < n; ++i) {
            ax[i] = anx[i];
            ay[i] = any[i];
            az[i] = anz[i];
        }
        if (traj) memcpy(traj + (size_t)s * 9 * (size_t)n, state, sizeof(double) * 9 * (size_t)n);
        if (energies && every > 0 && (s + 1) % every == 0)
            or_energies(n, state, q, m, tr, t1, eps2, energies + 4 * rec++, nthreads);
    }
    free(an);
}

/* ---------------------------------------------------- Hessian products -- */
/* Products of the Hessian of U = U_C + U_trap(t) with nvec vectors.  The
 * Coulomb pair term k_C q_i q_j (|d|^2 + eps2)^{-1/2}, d = r_i - r_j, has the
 * 3x3 Hessian block k_C q_i q_j (3 d d^T s^5 - I s^3) (s = (|d|^2+eps2)^{-1/2})
 * on the diagonal (i,i) and its negative off the diagonal (i,j), so
 *   (H v)_i = k_C q_i sum_{j != i} q_j [3 d (d . (v_i - v_j)) s^5 - (v_i - v_j) s^3]
 * plus, when m is non-NULL, the trap's diagonal m_i k(t) v_i.
 * v and hv are [nvec][3][n] (x block, y block, z block per vector). */
void or_hvp(int64_t n, const double* x, const double* y, const double* z, const double* q, int32_t nvec,
            const double* v, double* hv, const double* m, const or_trap* tr, double t, double eps2,
            int nthreads) {
    const double kc = or_coulomb_constant();
    double k[3] = {0, 0, 0};
    if (m) or_trap_k(tr, t, k);
    or_set_threads(nthreads);
    for (int32_t b = 0; b < nvec; ++b) {
        const double *vx = v + (size_t)b * 3 * n, *vy = vx + n, *vz = vy + n;
        double *hx = hv + (size_t)b * 3 * n, *hy = hx + n, *hz = hy + n;
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            or_sum sx = {0, 0}, sy = {0, 0}, sz = {0, 0};
            for (int64_t j = 0; j < n; ++j) {
                if (j == i) continue;
                double dx = x[i] - x[j], dy = y[i] - y[j], dz = z[i] - z[j];
                double r2 = dx * dx + dy * dy + dz * dz + eps2;
                double s = 1.0 / sqrt(r2);
                double s3 = s * s * s;
                double s5 = s3 * s * s;
                double ux = vx[i] - vx[j], uy = vy[i] - vy[j], uz = vz[i] - vz[j];
                double dot = dx * ux + dy * uy + dz * uz;
                double c = 3.0 * dot * s5;
                or_add(&sx, q[j] * (dx * c - ux * s3));
                or_add(&sy, q[j] * (dy * c - uy * s3));
                or_add(&sz, q[j] * (dz * c - uz * s3));
            }
            double ci = kc * q[i];
            hx[i] = ci * or_val(&sx);
            hy[i] = ci * or_val(&sy);
            hz[i] = ci * or_val(&sz);
            if (m) {
                hx[i] += m[i] * k[0] * vx[i];
                hy[i] += m[i] * k[1] * vy[i];
                hz[i] += m[i] * k[2] * vz[i];
            }
        }
    }
}

/* ------------------------------------------------- trajectory gradient -- */
/* Loss L = (1/n) sum_i |r_i(T) - r_i(0)|^2 after nsteps velocity-Verlet
 * steps from (r0, v0) with a_0 = a(r_0, t0), in a static pseudo-potential
 * trap (kind 0, no ramp), and its gradient with respect to (wx, wy, wz),
 * obtained by the discrete adjoint of the same steps (reverse-mode
 * differentiation of the recurrence as written; the whole trajectory is kept
 * in memory).  For one step (r, v, a) -> (r', v', a') with adjoints
 * (lr', lv', la'):
 *   la* = la' + dt/2 lv'                 (a' enters v' and is the new a)
 *   lr* = lr' + J^T la*,  J = da/dr = -(H_C/m) - diag(k)  at r'
 *   dL/dw_c += sum_i (-2 w_c r'_ic) la*_ic
 *   lr = lr*,  lv = lv' + dt lr*,  la = dt/2 lv' + dt^2/2 lr*
 * and finally a_0 = a(r_0) adds dL/dw_c += sum_i (-2 w_c r_0ic) la_0ic.
 * state0 holds x y z vx vy vz (6n doubles).  out[0] = L, out[1..3] = dL/dw.
 * Without friction only (tr->gamma != 0 gives NaN in every output). */
void or_msd_grad(int64_t n, const double* state0, const double* q, const double* m, const or_trap* tr,
                 double dt, int64_t nsteps, double eps2, double* out, int nthreads) {
    if (tr->gamma != 0.0) {
        out[0] = out[1] = out[2] = out[3] = NAN;
        return;
    }
    const size_t N9 = 9 * (size_t)n;
    double* tr_all = (double*)malloc(sizeof(double) * N9 * (size_t)(nsteps + 1));
    memcpy(tr_all, state0, sizeof(double) * 6 * (size_t)n);
    or_md_run(n, tr_all, q, m, tr, 0.0, dt, 0, eps2, 1, NULL, 0, NULL, nthreads); /* a_0 */
    double* st = (double*)malloc(sizeof(double) * N9);
    memcpy(st, tr_all, sizeof(double) * N9);
    or_md_run(n, st, q, m, tr, 0.0, dt, nsteps, eps2, 0, NULL, 0, tr_all + N9, nthreads);
    free(st);
    const double w[3] = {tr->wx, tr->wy, tr->wz};
    double k[3];
    or_trap_k(tr, 0.0, k);
    const double* rT = tr_all + N9 * (size_t)nsteps;
    or_sum L = {0, 0};
    double* lr = (double*)calloc(3 * (size_t)n, sizeof(double));
    double* lv = (double*)calloc(3 * (size_t)n, sizeof(double));
    double* la = (double*)calloc(3 * (size_t)n, sizeof(double));
    double* las = (double*)malloc(sizeof(double) * 3 * (size_t)n);
    double* u = (double*)malloc(sizeof(double) * 3 * (size_t)n);
    double* hu = (double*)malloc(sizeof(double) * 3 * (size_t)n);
    for (int c = 0; c < 3; ++c)
        for (int64_t i = 0; i < n; ++i) {
            double d = rT[c * n + i] - tr_all[c * n + i];
            or_add(&L, d * d);
            lr[c * n + i] = 2.0 * d / (double)n;
        }
    or_sum g[3] = {{0, 0}, {0, 0}, {0, 0}};
    for (int64_t s = nsteps; s >= 1; --s) {
        const double* rp = tr_all + N9 * (size_t)s; /* r' of the step s-1 -> s */
        for (size_t e = 0; e < 3 * (size_t)n; ++e) las[e] = la[e] + 0.5 * dt * lv[e];
        for (int c = 0; c < 3; ++c)
            for (int64_t i = 0; i < n; ++i) u[c * n + i] = las[c * n + i] / m[i];
        or_hvp(n, rp, rp + n, rp + 2 * n, q, 1, u, hu, m, tr, 0.0, eps2, nthreads);
        for (int c = 0; c < 3; ++c)
            for (int64_t i = 0; i < n; ++i) {
                size_t e = c * n + i;
                double lrs = lr[e] - hu[e];
                or_add(&g[c], -2.0 * w[c] * rp[e] * las[e]);
                double lvp = lv[e];
                lr[e] = lrs;
                lv[e] = lvp + dt * lrs;
                la[e] = 0.5 * dt * lvp + 0.5 * dt * dt * lrs;
            }
    }
    for (int c = 0; c < 3; ++c)
        for (int64_t i = 0; i < n; ++i) or_add(&g[c], -2.0 * w[c] * tr_all[c * n + i] * la[c * n + i]);
    out[0] = or_val(&L) / (double)n;
    out[1] = or_val(&g[0]);
    out[2] = or_val(&g[1]);
    out[3] = or_val(&g[2]);
    (void)k;
    free(tr_all);
    free(lr);
    free(lv);
    free(la);
    free(las);
    free(u);
    free(hu);
}
