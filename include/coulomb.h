/*
 * coulomb.h -- C ABI of libcoulomb_mi355x.so: direct all-pairs Coulomb forces
 * and velocity-Verlet motion of ions in a linear Paul trap, on one MI355X
 * (gfx950) GPU.
 *
 * Physics (paper, section 2, eq. (1), with the readings below):
 *   F_i   = k_C q_i sum_{j != i} q_j (r_i - r_j) / (|r_i - r_j|^2 + eps2)^{3/2}
 *   a_i   = F_i / m_i - (kx(t) x_i, ky(t) y_i, kz(t) z_i)
 *   U_C   = k_C sum_{i<j} q_i q_j (|r_i - r_j|^2 + eps2)^{-1/2}
 *   U_trap= sum_i m_i (kx x_i^2 + ky y_i^2 + kz z_i^2) / 2,  K = sum_i m_i |v_i|^2 / 2
 * with k_C = 1/(4 pi eps0) (CODATA 2018 eps0), the self pair excluded, eps2
 * (softening) added to r^2 as in the paper's section 3 double loop, and the
 * trap spring constants per unit mass k(t) given by cb_trap below.
 * Velocity-Verlet is the paper's three-step list (section 2):
 *   r' = r + v dt + a dt^2/2;  a' = a(r', t + dt);  v' = v + (a + a') dt/2.
 *
 * Conventions shared by every call:
 *  - Units are SI (m, s, kg, C, N, J).  Every array argument is a DEVICE
 *    pointer to contiguous float64 data of length n (structure of arrays)
 *    unless stated otherwise; host pointers are marked "host".
 *  - The caller owns all buffers.  The library never allocates or frees
 *    device memory in these calls and keeps no pointer after it returns.
 *    Scratch space is the caller's workspace `ws` of `ws_bytes` bytes (device
 *    memory, any alignment of 256 bytes or more), sized by
 *    cb_workspace_size(); too small a workspace returns CB_ENOWS.
 *  - All work is enqueued on `stream` (a hipStream_t; NULL is the default
 *    stream) and the call returns after enqueueing.  Host arrays passed in
 *    (offsets, traps) may be reused as soon as the call returns.
 *  - Argument errors are detected before anything is enqueued and returned as
 *    CB_EINVAL / CB_ENOWS / CB_EUNSUPPORTED; a failed launch returns CB_EHIP.
 *    cb_last_error() then describes the failure (thread-local string).
 *  - Outputs must not alias inputs except for the documented in-place state.
 *  - Results are deterministic: the same inputs, precision and launch
 *    configuration (see cb_autotune) give bitwise identical outputs; no
 *    floating-point atomics are used.
 *  - Non-finite outputs (e.g. two coincident ions with eps2 = 0) are not an
 *    error; they set a device flag that cb_poll_flags() reports.
 *
 * Readings of the paper (it is silent or inconsistent on these points):
 *  - the sum of eq. (1) excludes j = i;
 *  - the trap term of eq. (1) acts on ion i (it prints x_j, y_j);
 *  - the RF drive 2 Q V_RF cos(.) / (m r0^2) is written in Mathieu form
 *    q Omega^2/2 cos(Omega t + phi) with Omega in rad/s;
 *  - charges and masses are per ion.
 */
#ifndef COULOMB_MI355X_H
#define COULOMB_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes returned by every call. */
typedef enum {
    CB_OK = 0,
    CB_EINVAL = 1,        /* bad argument (NULL, n < 1, dt <= 0, aliasing, ...) */
    CB_EHIP = 2,          /* a HIP runtime call or kernel launch failed */
    CB_ENOWS = 3,         /* workspace too small */
    CB_ENONFINITE = 4,    /* reported by cb_poll_flags when the flag is set */
    CB_EUNSUPPORTED = 5   /* valid request the library does not handle */
} cb_status;

/* How 1/sqrt(r^2 + eps2) is evaluated (paper, sections 2 and 4: the cost and
 * accuracy of the inverse square root decide the speed of the pair loop).
 *  CB_FP64      FP32 hardware estimate of the FP32-rounded r^2, refined to
 *               full double precision by a second-order correction of
 *               q r^-3 (one order beyond the Newton-Raphson step of
 *               section 4); all arithmetic but the estimate is FP64.  The
 *               default.  Like CB_MIXED it requires r^2 + eps2 inside the
 *               FP32 normal range (1.2e-38 .. 3.4e38 m^2; ion spacings from
 *               1.1e-19 m to 1.8e19 m), which every trapped-ion geometry
 *               meets; CB_FP64_IEEE has no such limit.
 *  CB_MIXED     FP32 hardware estimate of the FP32-rounded r^2 followed by ONE
 *               FP64 Newton-Raphson step on the FP64 r^2 (the analogue of the
 *               paper's "RSQRT14 + 1 N-W"); displacements, r^2, the force
 *               numerator and all accumulation stay FP64.  Relative force
 *               error well below 1e-7.  Requires r^2 + eps2 inside the FP32
 *               normal range (1.2e-38 .. 3.4e38 m^2).
 *  CB_FP64_IEEE one correctly rounded square root and one correctly rounded
 *               division (the paper's "SQRT+DIV"); the slow reference.
 *  CB_FP32_RSQ  the FP32 hardware estimate alone, no refinement (the
 *               analogue of the paper's lowest-accuracy "RSQRT14").
 *  CB_MIXED_F32D  ablation of CB_MIXED: as CB_MIXED, but each displacement
 *               is rounded to FP32 and used so in r^2 and in the force
 *               numerator (the literal "FP32 displacement" reading of the
 *               mixed path; relative force error about 2^-24 per pair).
 *               coulomb_forces and coulomb_forces_range only (the direct
 *               kernel); other entry points return CB_EUNSUPPORTED. */
typedef enum {
    CB_FP64 = 0,
    CB_MIXED = 1,
    CB_FP64_IEEE = 2,
    CB_FP32_RSQ = 3,
    CB_MIXED_F32D = 4
} cb_precision;

/* Operation codes for cb_workspace_size / cb_autotune.  CB_OP_MD_ENSEMBLE
 * only keys the launch configuration of md_run with nrun > 1
 * (cb_get_config / cb_set_config); its workspace is that of CB_OP_MD_RUN.
 * CB_OP_GRAD only sizes the workspace of coulomb_trap_grad (whose launches
 * follow the CB_OP_FORCES and CB_OP_ENERGY configurations). */
typedef enum { CB_OP_FORCES = 0, CB_OP_ENERGY = 1, CB_OP_MD_STEP = 2, CB_OP_MD_RUN = 3,
               CB_OP_HVP = 4, CB_OP_ADJOINT = 5, CB_OP_MD_ENSEMBLE = 6, CB_OP_GRAD = 7 } cb_op;

/* md_run flags. */
#define CB_INIT_ACCEL 1u /* compute a(r_0, t0) before the first step instead of using s->a* */

/* md_adjoint_step flags. */
#define CB_ADJ_FINAL 1u  /* only add the trap-frequency term of (r, la); no HVP, no update */

/* Trap (host struct, passed by pointer, read during the call only).
 *  kind 0: static pseudo-potential, k = (wx^2, wy^2, wz^2), with an optional
 *          linear ramp of wx, wy from (wx, wy) at t_ramp0 to (wx1, wy1) at
 *          t_ramp1, constant outside; the ramp is off when t_ramp1 <= t_ramp0.
 *  kind 1: explicit RF drive in Mathieu form plus a static axial well:
 *          kx = rf_a rf_omega^2/4 + rf_q rf_omega^2/2 cos(rf_omega t + rf_phase),
 *          ky = -kx, kz = wz^2.
 *  gamma: the friction coefficient Gamma >= 0 (kg/s) of eq. (1)'s -Gamma v / m
 *          term (0 = none).  md_step / md_run integrate it by the trapezoidal
 *          rule inside velocity-Verlet (g = Gamma / m_i): the drift uses
 *          a - g v, and v_{n+1} = (v_n (1 - g dt/2) + dt/2 (a_n + a_{n+1})) /
 *          (1 + g dt/2); the state's a stays the conservative acceleration.
 *          md_adjoint_step needs gamma = 0; coulomb_hvp ignores it.
 *  All frequencies in rad/s. */
typedef struct {
    int32_t kind;
    double wx, wy, wz;
    double rf_a, rf_q, rf_omega, rf_phase;
    double gamma;
    double wx1, wy1, t_ramp0, t_ramp1;
} cb_trap;

/* Velocity-Verlet state: nine device arrays (positions, velocities,
 * accelerations), in/out.  For md_run with several runs they hold the runs
 * packed one after the other (see offsets). */
typedef struct {
    double *x, *y, *z, *vx, *vy, *vz, *ax, *ay, *az;
} cb_state;

/* Size in bytes of the workspace the call `op` needs for n ions (n_total for
 * md_run), nrun runs, nvec HVP vectors and precision prec.  0 on bad input
 * (including n outside [1, 2^28], the range every entry point accepts).
 * For md_run with nrun > 1 it covers both ensemble paths for any split of
 * n_total into nrun runs of at most 4096 ions (about 0.5 KB per ion). */
size_t cb_workspace_size(int32_t op, int64_t n, int32_t nrun, int32_t nvec, int32_t prec);

/* Forces F_i (N) on all n ions (eq. (1), Coulomb term times m; section 3
 * double loop).  x, y, z, q: inputs (m, C).  fx, fy, fz: outputs, must not
 * alias the inputs.  n = 1 gives zero force.  eps2 >= 0 (m^2). */
cb_status coulomb_forces(int64_t n, const double* x, const double* y, const double* z, const double* q,
                         double eps2, int32_t prec, double* fx, double* fy, double* fz,
                         void* ws, size_t ws_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * coulomb_forces without a workspace argument.  Same inputs, outputs,
 * precisions and errors as coulomb_forces; the partial sums live in a static
 * 64 MiB device array that the library holds on each GPU it runs on until the
 * process ends, so this call allocates nothing (no hipMalloc, no hipFree, no
 * allocating library routine).  n at most 2796202 (64 MiB over 24 bytes per
 * ion); larger n returns CB_ENOWS.  The configured Newton's-third-law stage
 * runs when its tiles fit in the array (up to about 32768 ions: the result
 * is then bitwise that of coulomb_forces), otherwise the all-pairs kernel
 * with as many j-splits as fit (the same forces up to summation order).
 * Every call on one GPU shares that GPU's array: calls that overlap in time
 * on one GPU (other streams, other threads) race and give undefined results;
 * calls ordered on one stream are safe.  Nothing in the array needs to start
 * at zero: each call overwrites what it reads. */
cb_status coulomb_forces_noalloc(int64_t n, const double* x, const double* y, const double* z, const double* q,
                                 double eps2, int32_t prec, double* fx, double* fy, double* fz, void* stream);

/* Forces (N) on the ions i0 .. i1-1 only, from all n ions (the same sum as
 * coulomb_forces, eq. (1) and the section 3 double loop, restricted to a
 * contiguous range of i): the share of one GPU when a force evaluation is
 * split across GPUs by ion index, each GPU holding every position.  x, y, z,
 * q: n doubles each.  fx, fy, fz: outputs of i1 - i0 doubles, indexed by
 * i - i0; they must not alias the inputs.  0 <= i0 < i1 <= n, else
 * CB_EINVAL.  Every ordered pair with i in the range is evaluated (no
 * Newton's third law); the sums are deterministic.  Workspace:
 * cb_workspace_size(CB_OP_FORCES, n, 1, 1, prec) suffices. */
cb_status coulomb_forces_range(int64_t n, int64_t i0, int64_t i1, const double* x, const double* y, const double* z,
                               const double* q, double eps2, int32_t prec, double* fx, double* fy, double* fz,
                               void* ws, size_t ws_bytes, void* stream);

/* The first stage of coulomb_forces on its own (everything but the final
 * element-wise pass), for timing the pair loop and for callers that finish
 * the sums themselves.  With algorithm 0 (see cb_get_config) the all-pairs
 * kernel leaves its j-split partial force sums, before the fixed-order sum
 * over splits and the k_C q_i factor, at the start of ws as [splits][3][n]
 * doubles and *splits_out (host) is the number of splits; with algorithms 1,
 * 2 and 4 (the Newton's-third-law stages) the start of ws holds the finished
 * forces [3][n] and *splits_out is 0. */
cb_status coulomb_pair_stage(int64_t n, const double* x, const double* y, const double* z, const double* q,
                             double eps2, int32_t prec, int32_t* splits_out, void* ws, size_t ws_bytes,
                             void* stream);

/* Coulomb energy U_C = k_C sum_{i<j} q_i q_j / (r_ij^2 + eps2)^{1/2} (J), the
 * Coulomb part of the potential whose negative gradient is eq. (1)'s
 * Coulomb force (section 2), into u_out[0] (device, one double).  x, y, z,
 * q as for coulomb_forces.  Summed in a fixed order (deterministic). */
cb_status coulomb_energy(int64_t n, const double* x, const double* y, const double* z, const double* q,
                         double eps2, int32_t prec, double* u_out, void* ws, size_t ws_bytes, void* stream);

/* Gradient and value of the potential energy of eq. (1) at time t,
 *   U = U_C + U_trap(t),   g_i = dU/dr_i = -F_i + m_i k(t) r_i,
 * with F the Coulomb forces of coulomb_forces and k(t) the trap's spring
 * constants per unit mass (cb_trap_k).  m NULL: the Coulomb part alone
 * (trap ignored).  gx, gy, gz: outputs (device, n doubles each), all three
 * or none; u_out: output (device, one double: U in J) or NULL; at least one
 * of the two is requested.  Outputs must not alias inputs or each other.
 * The gradient alone takes the configured force stage (CB_OP_FORCES); with
 * the energy, the all-pairs kernel evaluates forces and potentials in one
 * pass (CB_OP_ENERGY's configuration).  The trap terms are added in the same
 * element-wise pass that finishes the Coulomb sums.  Workspace:
 * cb_workspace_size(CB_OP_GRAD, n, 1, 1, prec).  (Used by the autograd
 * functions and the minimiser, so that no trap arithmetic runs outside the
 * library.) */
cb_status coulomb_trap_grad(int64_t n, const double* x, const double* y, const double* z, const double* q,
                            const double* m, const cb_trap* trap, double t, double eps2, int32_t prec, double* gx,
                            double* gy, double* gz, double* u_out, void* ws, size_t ws_bytes, void* stream);

/* The trap's spring constants per unit mass at time t into k_out[3] (host),
 * so that the trap acceleration is -(kx x, ky y, kz z) (eq. (1); see
 * cb_trap for the pseudo-potential, its ramp and the RF drive in Mathieu
 * form).  The same function the kernels evaluate.  Host only; no GPU work. */
cb_status cb_trap_k(const cb_trap* trap, double t, double k_out[3]);

/* One velocity-Verlet step from time t (section 2): s holds (r_n, v_n, a_n)
 * on entry and (r_{n+1}, v_{n+1}, a_{n+1}) on return, with a_{n+1} taken at
 * t + dt.  q (C), m (kg): per-ion charges and masses.  dt > 0. */
cb_status md_step(int64_t n, const cb_state* s, const double* q, const double* m, const cb_trap* trap,
                  double t, double dt, double eps2, int32_t prec, void* ws, size_t ws_bytes, void* stream);

/* nsteps velocity-Verlet steps (section 2, as md_step) of nrun independent
 * runs packed in s, q, m:
 * run r owns ions offsets[r] .. offsets[r+1]-1 (offsets: host, nrun+1
 * entries, offsets[0] = 0, strictly increasing) and follows traps[r] (host,
 * nrun entries).  Step k of every run is at time t0 + k dt.  With flags &
 * CB_INIT_ACCEL, a_0 = a(r_0, t0) is computed first; otherwise s->a* must
 * hold a_0.  When energies is non-NULL (device, [nrun][nsteps/every + 1][4])
 * it receives (K, U_C, U_trap, K + U_C + U_trap) of steps 0, every, 2 every,
 * ..., for each run; every >= 1 then.
 * nrun = 1 runs the multi-workgroup step kernels (any n).  nrun > 1 needs
 * every run to hold at most 4096 ions (CB_EUNSUPPORTED otherwise) and takes
 * one of two ensemble paths (configuration key CB_OP_MD_ENSEMBLE):
 *  - algorithm 0: one persistent launch, one workgroup per run at a time,
 *    positions in LDS, runs taken largest first;
 *  - algorithm 2: per step, one launch of the Newton's-third-law pair tiles
 *    of every run and one launch that finishes the forces and applies the
 *    kick and drift (p i-particles per lane, j-segment length JL).
 * Without a forced or tuned entry the path with the smaller estimated step
 * time is taken (algorithm 0 wins only for ensembles of small runs whose
 * step is shorter than the stepped path's launch latency), with p = 4 and
 * JL = 256, or JL = 512 for ensembles of at least 2^30 ordered pairs.  Both paths give the same trajectories up to rounding
 * (different summation orders); each is deterministic.
 * Graph capture: md_run may be called on a stream that is being captured.
 * With nrun = 1 it enqueues kernels and device copies only.  With nrun > 1
 * it also copies run tables (built from offsets and traps at the call) from
 * host memory; under capture those tables are first copied into a host
 * block that the captured graph owns (released after the graph is
 * destroyed), so offsets and traps may be freed on return and every replay
 * repeats the captured call: same runs, traps, t0, nsteps, energy slots and
 * workspace, continuing from whatever state s holds. */
cb_status md_run(int32_t nrun, const int64_t* offsets, const cb_state* s, const double* q, const double* m,
                 const cb_trap* traps, double t0, double dt, int64_t nsteps, double eps2, int32_t prec,
                 uint32_t flags, double* energies, int64_t every, void* ws, size_t ws_bytes, void* stream);

/* Hessian-vector products of U = U_C (+ U_trap(t) when m is non-NULL) with
 * nvec vectors v (device, [nvec][3][n]: x block, y block, z block per vector)
 * into hv (same layout, must not alias v):
 *   (H v)_i = k_C q_i sum_{j != i} q_j [3 d (d . (v_i - v_j)) s^5 - (v_i - v_j) s^3]
 *             + m_i k(t) v_i,     d = r_i - r_j, s = (|d|^2 + eps2)^{-1/2}.
 * (Not in the paper: the second derivative of its eq. (1) energy, used for
 * normal modes and trajectory gradients.)  1 <= nvec <= 8. */
cb_status coulomb_hvp(int64_t n, const double* x, const double* y, const double* z, const double* q,
                      int32_t nvec, const double* v, double* hv, const double* m, const cb_trap* trap,
                      double t, double eps2, int32_t prec, void* ws, size_t ws_bytes, void* stream);

/* One step of the discrete adjoint (reverse mode) of md_step, for a static
 * pseudo-potential trap (kind 0, no ramp).  x, y, z hold r_{n+1}; lam
 * (device, [9][n]) holds the adjoints (l_r, l_v, l_a) of (r_{n+1}, v_{n+1},
 * a_{n+1}) on entry and those of (r_n, v_n, a_n) on return:
 *   la* = la + dt/2 lv;  lr* = lr + J^T la*,  J = da/dr at r_{n+1};
 *   dldw[c] += sum_i (-2 w_c r_ic) la*_ic   (c = x, y, z; dldw device, 3 doubles);
 *   lr <- lr*;  lv <- lv + dt lr*;  la <- dt/2 lv + dt^2/2 lr*  (old lv).
 * With flags & CB_ADJ_FINAL it only adds sum_i (-2 w_c r_ic) la_ic (the a_0
 * term) and leaves lam unchanged. */
cb_status md_adjoint_step(int64_t n, const double* x, const double* y, const double* z, const double* q,
                          const double* m, const cb_trap* trap, double dt, double eps2, int32_t prec,
                          uint32_t flags, double* lam, double* dldw, void* ws, size_t ws_bytes, void* stream);

/* Synchronises `stream`, writes the device flag word to *flags_out (bit 0:
 * a non-finite value was produced since the last poll), clears it, and
 * returns CB_ENONFINITE when bit 0 was set, CB_OK otherwise. */
cb_status cb_poll_flags(void* stream, uint32_t* flags_out);

/* Thread-local description of the last error ("" if none). */
const char* cb_last_error(void);

/* Times the candidate launch configurations (i-particles per lane, workgroup
 * size, j-split count) of `op` at n ions and precision prec on the current
 * device, keeps the fastest for all later calls with n in the same
 * power-of-two bucket, and, when cache_path is non-NULL, merges it into that
 * JSON-lines file.  For md_step / md_run at n <= 8192 the force kernel is
 * tuned for coulomb_forces, and the j-parts of the one-launch step
 * (algorithm 3) for the md calls.  Uses synthetic inputs it allocates itself (this call, and
 * cb_load_tuning, are the only ones that allocate).  Synchronous. */
cb_status cb_autotune(int32_t op, int64_t n, int32_t prec, const char* cache_path);

/* Loads tuned configurations written by cb_autotune (missing file: CB_OK). */
cb_status cb_load_tuning(const char* cache_path);

/* The launch configuration the next call of `op` at (n, prec) will use:
 * out[0] = algorithm (0: every ordered pair evaluated, j-split partial sums;
 *          1: each unordered pair evaluated once and applied to both ions by
 *          Newton's third law, forces only, n <= 2^18, the reactions summed
 *          over the wave by cross-lane permutes; 2: as 1, summed through LDS;
 *          4: as 2, with four i-blocks to a workgroup that share one
 *          j-segment and sum their reactions in LDS before one write, which
 *          cuts the partial sums written and read back by four;
 *          3: md_step / md_run of one run of at most 8192 ions in one launch
 *          per step, every ordered pair evaluated by one wave per 64 ions and
 *          j-part, the parts added in a fixed order by the last to finish,
 *          then trap, kick and drift -- the default up to 256 ions),
 * out[1] = i-particles per lane, out[2] = workgroup size (algorithm 0) or
 *          j's per reduction group (algorithms 1, 2, 4),
 * out[3] = j-splits (algorithm 0), j-segment length (algorithms 1, 2, 4) or
 *          j-parts per 64 ions (algorithm 3),
 * out[4] = 1 if it came from tuning or cb_set_config.
 * CB_EINVAL for a NULL out, n outside [1, 2^28], or an op or prec outside
 * its enum. */
cb_status cb_get_config(int32_t op, int64_t n, int32_t prec, int32_t out[5]);

/* Forces the launch configuration for (op, n power-of-two bucket, prec), with
 * the fields of cb_get_config.  Algorithm 0: p in {1,2,4} ({1,2} for the HVP
 * and adjoint), wg in {64,128,256}, splits in 1..64.  Algorithms 1 and 2 (forces,
 * energy, md_step, md_run; n <= 2^18): p in {2,3,4,5,6,8}, wg = j's per reduction
 * group = 4, splits = segment length in {256,512,1024,2048}.  Algorithm 4
 * (the same ops and sizes): p in {4, 6, 8},
 * wg = 4, the same segment lengths.  Algorithm 3
 * (md_step, md_run; n <= 8192): p = 1, wg = 64, splits = j-parts in 1..32.
 * For CB_OP_HVP and CB_OP_ADJOINT, algorithm 2 is the Newton's-third-law
 * product: p in {1, 2, 4}, wg = the most vectors per pass in {1, 2, 4},
 * splits = segment length in {64, 128, 256, 512}; n <= 131072 p.
 * For CB_OP_MD_ENSEMBLE (n = total ions): algorithm 0 with p = 4, wg = 512,
 * splits = 1 (the persistent kernel's fixed shape), or algorithm 2 with p in
 * {4, 8}, wg = 4, splits = JL in {256, 512}.
 * algo = p = wg = splits = 0 removes a forced or tuned entry (back to the
 * built-in heuristic).  CB_EINVAL if unsupported, or for n outside [1, 2^28]
 * or an op or prec outside its enum. */
cb_status cb_set_config(int32_t op, int64_t n, int32_t prec, int32_t algo, int32_t p, int32_t wg, int32_t splits);

#ifdef __cplusplus
}
#endif
#endif /* COULOMB_MI355X_H */
