// Entry points coulomb_hvp and md_adjoint_step: Hessian-vector products of
// the Coulomb + trap energy and one reverse step of the discrete adjoint of
// velocity-Verlet.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "hvp_kernels.hpp"
#include "hvp_sym.hpp"
#include "internal.hpp"
#include "split_sum.hpp"
#include "step_common.hpp"

namespace cb {

// ------------------------------------------------------------ dispatch
template <int PREC, int P, int NV>
static void go_hvp(dim3 g, dim3 b, hipStream_t st, int n, const double* x, const double* y, const double* z,
                   const double* q, const double* v, double eps2, int jlen, double* part) {
    k_hvp<PREC, P, NV><<<g, b, 0, st>>>(n, x, y, z, q, v, eps2, jlen, part);
}

template <int PREC, int P>
static bool go_hvp_nv(int nv, dim3 g, dim3 b, hipStream_t st, int n, const double* x, const double* y,
                      const double* z, const double* q, const double* v, double eps2, int jlen, double* part) {
    switch (nv) {
        case 1: go_hvp<PREC, P, 1>(g, b, st, n, x, y, z, q, v, eps2, jlen, part); return true;
        case 2: go_hvp<PREC, P, 2>(g, b, st, n, x, y, z, q, v, eps2, jlen, part); return true;
        case 4: go_hvp<PREC, P, 4>(g, b, st, n, x, y, z, q, v, eps2, jlen, part); return true;
        default: return false;
    }
}

template <int PREC>
static bool go_hvp_p(int p, int nv, dim3 g, dim3 b, hipStream_t st, int n, const double* x, const double* y,
                     const double* z, const double* q, const double* v, double eps2, int jlen, double* part) {
    if (p == 1) return go_hvp_nv<PREC, 1>(nv, g, b, st, n, x, y, z, q, v, eps2, jlen, part);
    if (p == 2) return go_hvp_nv<PREC, 2>(nv, g, b, st, n, x, y, z, q, v, eps2, jlen, part);
    return false;
}

cb_status launch_hvp(int prec, const LaunchCfg& c, int nvec, int n, const double* x, const double* y,
                     const double* z, const double* q, const double* v, double eps2, int jlen, double* part,
                     hipStream_t st) {
    const int S = n_splits(n, jlen);
    const int ipb = 64 * c.p * (c.wg / 64);
    dim3 grid((n + ipb - 1) / ipb, S), block(c.wg);
    bool okk = false;
    switch (prec) {
        case PREC_FP64: okk = go_hvp_p<PREC_FP64>(c.p, nvec, grid, block, st, n, x, y, z, q, v, eps2, jlen, part); break;
        case PREC_MIXED: okk = go_hvp_p<PREC_MIXED>(c.p, nvec, grid, block, st, n, x, y, z, q, v, eps2, jlen, part); break;
        case PREC_IEEE: okk = go_hvp_p<PREC_IEEE>(c.p, nvec, grid, block, st, n, x, y, z, q, v, eps2, jlen, part); break;
        case PREC_FP32: okk = go_hvp_p<PREC_FP32>(c.p, nvec, grid, block, st, n, x, y, z, q, v, eps2, jlen, part); break;
        default: break;
    }
    if (!okk) return fail(CB_EINVAL, "launch_hvp: unsupported precision %d / p %d / nvec %d", prec, c.p, nvec);
    return check_launch("k_hvp");
}

// ------------------------------------------- Newton's third law (hvp_sym.hpp)
static size_t al256h(size_t b) { return (b + 255) / 256 * 256; }

// tile table | Pi[npass T][4][3][IB] | R[npass T][4][3][JL] | packed j
// records [npass][n][16] (npass passes of at most 4 vectors in one launch)
size_t hvp_sym_ws_bytes(int64_t n, int p, int jl, int npass) {
    const int IB = 64 * p;
    const int64_t T = sym_tiles(n, IB, jl);
    const size_t np = (size_t)npass;
    return sym_plan_bytes(n, IB, jl) + al256h(sizeof(double) * 12 * (size_t)IB * (np * T + 1)) +
           al256h(sizeof(double) * 12 * (size_t)jl * (np * T + 1)) +
           al256h(sizeof(double) * kHvpRec * np * (size_t)n);
}

template <int PREC, int P, int NV>
static void go_hvp_sym(int npass, int n, const SymPlan& pl, int JL, const double* x, const double* y,
                       const double* z, const double* q, const double* v, const double* J, double eps2, double* Pi,
                       double* R, hipStream_t st) {
    const dim3 g((unsigned)pl.T, (unsigned)npass);
    k_hvp_sym<PREC, P, NV><<<g, 64, 0, st>>>(n, x, y, z, q, v, J, eps2, JL, pl.tiles, Pi, R);
}

template <int PREC, int NV>
static bool go_hvp_sym_p(int P, int npass, int n, const SymPlan& pl, int JL, const double* x, const double* y,
                         const double* z, const double* q, const double* v, const double* J, double eps2, double* Pi,
                         double* R, hipStream_t st) {
    switch (P) {
        case 1: go_hvp_sym<PREC, 1, NV>(npass, n, pl, JL, x, y, z, q, v, J, eps2, Pi, R, st); return true;
        case 2: go_hvp_sym<PREC, 2, NV>(npass, n, pl, JL, x, y, z, q, v, J, eps2, Pi, R, st); return true;
        case 4: go_hvp_sym<PREC, 4, NV>(npass, n, pl, JL, x, y, z, q, v, J, eps2, Pi, R, st); return true;
        default: return false;
    }
}

template <int PREC>
static bool go_hvp_sym_nv(int nv, int P, int npass, int n, const SymPlan& pl, int JL, const double* x,
                          const double* y, const double* z, const double* q, const double* v, const double* J,
                          double eps2, double* Pi, double* R, hipStream_t st) {
    switch (nv) {
        case 1: return go_hvp_sym_p<PREC, 1>(P, npass, n, pl, JL, x, y, z, q, v, J, eps2, Pi, R, st);
        case 2: return go_hvp_sym_p<PREC, 2>(P, npass, n, pl, JL, x, y, z, q, v, J, eps2, Pi, R, st);
        case 4: return go_hvp_sym_p<PREC, 4>(P, npass, n, pl, JL, x, y, z, q, v, J, eps2, Pi, R, st);
        default: return false;
    }
}

template <int PREC>
static bool go_hvp_fin(int nv, int npass, unsigned nb, int n, int IB, int JL, int lgJL, int T, const double* x,
                       const double* y, const double* z, const double* q, const double* v, double eps2,
                       const int* rowstart, const double* Pi, const double* R, const double* m, TrapK k, double* hv,
                       unsigned* fl, hipStream_t st) {
    const dim3 g(nb, (unsigned)(npass * nv)), b(64 * kFinishParts);
    switch (nv) {
        case 1: k_hvp_sym_finish<PREC, 1><<<g, b, 0, st>>>(n, IB, JL, lgJL, T, x, y, z, q, v, eps2, rowstart, Pi, R, m, k, hv, fl); return true;
        case 2: k_hvp_sym_finish<PREC, 2><<<g, b, 0, st>>>(n, IB, JL, lgJL, T, x, y, z, q, v, eps2, rowstart, Pi, R, m, k, hv, fl); return true;
        case 4: k_hvp_sym_finish<PREC, 4><<<g, b, 0, st>>>(n, IB, JL, lgJL, T, x, y, z, q, v, eps2, rowstart, Pi, R, m, k, hv, fl); return true;
        default: return false;
    }
}

// nvec products in passes of 4, 2, 1 vectors (at most c.wg per pass), up to
// kHvpSymPasses passes of one size in one launch: per launch the j records
// are packed, the tiles evaluated and each ion finished (trap term included).
static cb_status launch_hvp_sym(int prec, const LaunchCfg& c, int nvec, int n, const double* x, const double* y,
                                const double* z, const double* q, const double* v, const double* m, TrapK k,
                                double eps2, void* ws, double* hv, unsigned* fl, hipStream_t st) {
    const int P = c.p, JL = c.splits, IB = 64 * P;
    if (!hvp_sym_cfg_ok(P, JL) || n > hvp_sym_max_n(P))
        return fail(CB_EINVAL, "coulomb_hvp: bad Newton's-third-law configuration p %d / JL %d at n = %d", P, JL, n);
    const int nvmax = c.wg;  // the most vectors per pass: 1, 2 or 4
    const int wsp = hvp_sym_passes(nvec, nvmax);  // the passes the workspace holds
    SymPlan pl;  // its table is filled by the first pack launch below
    cb_status rc = sym_plan(n, IB, JL, ws, &pl, st, 1, true);
    if (rc) return rc;
    const int nG = (n + IB - 1) / IB;
    const size_t np = (size_t)wsp;
    char* base = static_cast<char*>(ws) + pl.bytes;
    double* Pi = reinterpret_cast<double*>(base);
    base += al256h(sizeof(double) * 12 * (size_t)IB * (np * pl.T + 1));
    double* R = reinterpret_cast<double*>(base);
    base += al256h(sizeof(double) * 12 * (size_t)JL * (np * pl.T + 1));
    double* J = reinterpret_cast<double*>(base);
    int lgJL = 0;
    while ((1 << lgJL) < JL) ++lgJL;
    const unsigned nb = (unsigned)((n + 63) / 64);
    for (int b0 = 0; b0 < nvec;) {
        const int left = std::min(nvec - b0, nvmax);
        const int nv = left >= 4 ? 4 : left >= 2 ? 2 : 1;
        const int npass = std::max(1, std::min(wsp, (nvec - b0) / nv));
        const double* vb = v + (size_t)b0 * 3 * n;
        double* hb = hv + (size_t)b0 * 3 * n;
        const int plan_groups = b0 == 0 ? nG : 0;
        k_hvp_pack<<<dim3((n + 255) / 256 + (plan_groups > 0 ? 1 : 0), npass), 256, 0, st>>>(
            n, nv, x, y, z, q, vb, J, IB, JL, plan_groups, pl.rowstart, pl.tiles);
        if ((rc = check_launch("k_hvp_pack"))) return rc;
        bool okk = false;
        if (pl.T > 0) {
            switch (prec) {
                case PREC_FP64: okk = go_hvp_sym_nv<PREC_FP64>(nv, P, npass, n, pl, JL, x, y, z, q, vb, J, eps2, Pi, R, st); break;
                case PREC_MIXED: okk = go_hvp_sym_nv<PREC_MIXED>(nv, P, npass, n, pl, JL, x, y, z, q, vb, J, eps2, Pi, R, st); break;
                case PREC_IEEE: okk = go_hvp_sym_nv<PREC_IEEE>(nv, P, npass, n, pl, JL, x, y, z, q, vb, J, eps2, Pi, R, st); break;
                case PREC_FP32: okk = go_hvp_sym_nv<PREC_FP32>(nv, P, npass, n, pl, JL, x, y, z, q, vb, J, eps2, Pi, R, st); break;
                default: break;
            }
            if (!okk) return fail(CB_EINVAL, "coulomb_hvp: unsupported precision %d / p %d", prec, P);
            if ((rc = check_launch("k_hvp_sym"))) return rc;
        }
        const int T = (int)pl.T;
        switch (prec) {
            case PREC_FP64: okk = go_hvp_fin<PREC_FP64>(nv, npass, nb, n, IB, JL, lgJL, T, x, y, z, q, vb, eps2, pl.rowstart, Pi, R, m, k, hb, fl, st); break;
            case PREC_MIXED: okk = go_hvp_fin<PREC_MIXED>(nv, npass, nb, n, IB, JL, lgJL, T, x, y, z, q, vb, eps2, pl.rowstart, Pi, R, m, k, hb, fl, st); break;
            case PREC_IEEE: okk = go_hvp_fin<PREC_IEEE>(nv, npass, nb, n, IB, JL, lgJL, T, x, y, z, q, vb, eps2, pl.rowstart, Pi, R, m, k, hb, fl, st); break;
            default: okk = go_hvp_fin<PREC_FP32>(nv, npass, nb, n, IB, JL, lgJL, T, x, y, z, q, vb, eps2, pl.rowstart, Pi, R, m, k, hb, fl, st); break;
        }
        if (!okk) return fail(CB_EINVAL, "coulomb_hvp: unsupported vector count %d", nv);
        if ((rc = check_launch("k_hvp_sym_finish"))) return rc;
        b0 += npass * nv;
    }
    return CB_OK;
}

// --------------------------------------------------------- element-wise
// hv[b][c][i] = k_C q_i sum_s part[s][b][c][i] + m_i k_c v[b][c][i].
__global__ void __launch_bounds__(kEpiThreads) k_hvp_epi(int n, int S, int nv, const double* __restrict__ part,
                                                        const double* __restrict__ q, const double* __restrict__ m,
                                                        TrapK k, const double* __restrict__ v,
                                                        double* __restrict__ hv, unsigned* flags) {
    const int i = blockIdx.x * kEpiThreads + threadIdx.x;
    if (i >= n) return;
    const double c = kCoulomb * q[i];
    const double kk[3] = {k.kx, k.ky, k.kz};
    bool ok = true;
    const size_t stride = (size_t)nv * 3 * n;
    for (int b = 0; b < nv; ++b) {
        double s[3];
        const double* ps[3] = {part + ((size_t)b * 3) * n + i, part + ((size_t)b * 3 + 1) * n + i,
                               part + ((size_t)b * 3 + 2) * n + i};
        const size_t st[3] = {stride, stride, stride};
        split_sums<3>(ps, st, S, s);  // the vector's three components' loads together
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            double h = c * s[d];
            const size_t e = ((size_t)b * 3 + d) * n + i;
            if (m) h += m[i] * kk[d] * v[e];
            hv[e] = h;
            ok = ok && __builtin_isfinite(h);
        }
    }
    if (!ok) atomicOr(flags, 1u);
}

// u = (la + dt/2 lv) / m  (input of the adjoint step's HVP).
__global__ void __launch_bounds__(kEpiThreads) k_adj_pre(int n, const double* __restrict__ lam,
                                                        const double* __restrict__ m, double dt,
                                                        double* __restrict__ u) {
    const int i = blockIdx.x * kEpiThreads + threadIdx.x;
    if (i >= n) return;
    const double inv_m = 1.0 / m[i];
    for (int c = 0; c < 3; ++c) {
        const double las = lam[(6 + c) * (size_t)n + i] + 0.5 * dt * lam[(3 + c) * (size_t)n + i];
        u[c * (size_t)n + i] = las * inv_m;
    }
}

// The adjoint update after the HVP, plus per-block partial sums of the
// trap-frequency gradient terms -2 w_c r_c la*_c.  final_only: only the
// gradient term of (r, la), lam unchanged.  part: the Coulomb product's
// j-split partials [S][3][n] (to be scaled by k_C q_i), or with prescaled
// the finished Coulomb product [3][n] (S = 1).
__global__ void __launch_bounds__(kEpiThreads) k_adj_post(int n, int S, const double* __restrict__ part,
                                                         const double* __restrict__ x, const double* __restrict__ y,
                                                         const double* __restrict__ z, const double* __restrict__ q,
                                                         const double* __restrict__ m, const double* __restrict__ u,
                                                         TrapK k, double wx, double wy, double wz, double dt,
                                                         int final_only, int prescaled, double* __restrict__ lam,
                                                         double* __restrict__ eblk, unsigned* flags) {
    const int i = blockIdx.x * kEpiThreads + threadIdx.x;
    double g[3] = {0.0, 0.0, 0.0};
    if (i < n) {
        const double r[3] = {x[i], y[i], z[i]};
        const double w[3] = {wx, wy, wz};
        bool ok = true;
        if (final_only) {
            for (int c = 0; c < 3; ++c) g[c] = -2.0 * w[c] * r[c] * lam[(6 + c) * (size_t)n + i];
        } else {
            const double kk[3] = {k.kx, k.ky, k.kz};
            const double cq = prescaled ? 1.0 : kCoulomb * q[i];
            double ss[3];
            const double* ps[3] = {part + i, part + (size_t)n + i, part + 2 * (size_t)n + i};
            const size_t st[3] = {3 * (size_t)n, 3 * (size_t)n, 3 * (size_t)n};
            split_sums<3>(ps, st, S, ss);  // the three components' loads together
            for (int c = 0; c < 3; ++c) {
                const double s = ss[c];
                const size_t e = (size_t)c * n + i;
                const double hu = cq * s + m[i] * kk[c] * u[e];
                const double lr = lam[e], lv = lam[3 * (size_t)n + e], la = lam[6 * (size_t)n + e];
                const double las = la + 0.5 * dt * lv;
                const double lrs = lr - hu;
                g[c] = -2.0 * w[c] * r[c] * las;
                lam[e] = lrs;
                lam[3 * (size_t)n + e] = lv + dt * lrs;
                lam[6 * (size_t)n + e] = 0.5 * dt * lv + 0.5 * dt * dt * lrs;
                ok = ok && __builtin_isfinite(lrs) && __builtin_isfinite(hu);
            }
        }
        if (!ok) atomicOr(flags, 1u);
    }
    block_sum3(g[0], g[1], g[2]);
    if (threadIdx.x == 0) {
        eblk[blockIdx.x * 3 + 0] = g[0];
        eblk[blockIdx.x * 3 + 1] = g[1];
        eblk[blockIdx.x * 3 + 2] = g[2];
    }
}

// dldw[c] += fixed-order sum of the block partials.
__global__ void __launch_bounds__(kEpiThreads) k_adj_final(int nb, const double* __restrict__ eblk,
                                                          double* __restrict__ dldw) {
    double a = 0.0, b = 0.0, c = 0.0;
    for (int t = threadIdx.x; t < nb; t += kEpiThreads) {
        a += eblk[t * 3 + 0];
        b += eblk[t * 3 + 1];
        c += eblk[t * 3 + 2];
    }
    block_sum3(a, b, c);
    if (threadIdx.x == 0) {
        dldw[0] += a;
        dldw[1] += b;
        dldw[2] += c;
    }
}

static bool overl(const void* a, const void* b, size_t bytes_a, size_t bytes_b) {
    if (!a || !b) return false;
    const char* pa = static_cast<const char*>(a);
    const char* pb = static_cast<const char*>(b);
    return pa < pb + bytes_b && pb < pa + bytes_a;
}

static cb_status hvp_common(const char* who, int64_t n, int32_t prec, double eps2, void* ws, size_t ws_bytes,
                            size_t need) {
    if (n < 1 || n > kMaxIons) return fail(CB_EINVAL, "%s: n = %lld out of range [1, 2^28]", who, (long long)n);
    if (prec == CB_MIXED_F32D) return fail(CB_EUNSUPPORTED, "%s: CB_MIXED_F32D is for the forces only", who);
    if (prec < CB_FP64 || prec > CB_FP32_RSQ) return fail(CB_EINVAL, "%s: unknown precision %d", who, prec);
    if (!(eps2 >= 0.0) || !std::isfinite(eps2)) return fail(CB_EINVAL, "%s: eps2 must be finite and >= 0", who);
    if (!ws) return fail(CB_EINVAL, "%s: workspace is NULL", who);
    if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) return fail(CB_EINVAL, "%s: workspace not 256-byte aligned", who);
    if (ws_bytes < need) return fail(CB_ENOWS, "%s: workspace has %zu bytes, needs %zu", who, ws_bytes, need);
    return CB_OK;
}

static double* at(void* ws, size_t off) { return reinterpret_cast<double*>(static_cast<char*>(ws) + off); }

}  // namespace cb

using namespace cb;

extern "C" {

cb_status coulomb_hvp(int64_t n, const double* x, const double* y, const double* z, const double* q, int32_t nvec,
                      const double* v, double* hv, const double* m, const cb_trap* trap, double t, double eps2,
                      int32_t prec, void* ws, size_t ws_bytes, void* stream) {
    if (nvec < 1 || nvec > kMaxVec) return fail(CB_EINVAL, "coulomb_hvp: nvec = %d out of range [1, %d]", nvec, kMaxVec);
    const WsLayout L = ws_layout(CB_OP_HVP, n > 0 ? n : 1, 1, nvec, prec);
    cb_status rc = hvp_common("coulomb_hvp", n, prec, eps2, ws, ws_bytes, L.total);
    if (rc) return rc;
    if (!x || !y || !z || !q || !v || !hv) return fail(CB_EINVAL, "coulomb_hvp: NULL array");
    if (m && !trap_ok(trap, "coulomb_hvp", &rc)) return rc;
    if (!std::isfinite(t)) return fail(CB_EINVAL, "coulomb_hvp: t must be finite");
    const size_t vb = sizeof(double) * 3 * (size_t)nvec * (size_t)n, ab = sizeof(double) * (size_t)n;
    const void* ins[] = {x, y, z, q, m};
    for (auto p : ins)
        if (overl(hv, p, vb, ab)) return fail(CB_EINVAL, "coulomb_hvp: hv aliases an input");
    if (overl(hv, v, vb, vb)) return fail(CB_EINVAL, "coulomb_hvp: hv aliases v");
    unsigned* fl = flags_ptr();
    if (!fl) return fail(CB_EHIP, "coulomb_hvp: device flag symbol not found");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const LaunchCfg cfg = get_cfg(CB_OP_HVP, n, prec);
    const TrapK k = m ? trap_k(*trap, t) : TrapK{0.0, 0.0, 0.0};
    double* part = at(ws, L.part);
    if (is_sym(cfg.algo)) {
        if ((rc = launch_hvp_sym(prec, cfg, nvec, (int)n, x, y, z, q, v, m, k, eps2, part, hv, fl, st))) return rc;
        return ok();
    }
    const int jlen = split_len(n, cfg.splits);
    const int S = n_splits(n, jlen);
    // vectors in passes of 4, 2, 1 (eight per pass need too many registers)
    for (int b0 = 0; b0 < nvec;) {
        const int left = nvec - b0;
        const int nv = left >= 4 ? 4 : left >= 2 ? 2 : 1;
        const double* vb0 = v + (size_t)b0 * 3 * n;
        if ((rc = launch_hvp(prec, cfg, nv, (int)n, x, y, z, q, vb0, eps2, jlen, part, st))) return rc;
        k_hvp_epi<<<(int)((n + kEpiThreads - 1) / kEpiThreads), kEpiThreads, 0, st>>>(
            (int)n, S, nv, part, q, m, k, vb0, hv + (size_t)b0 * 3 * n, fl);
        if ((rc = check_launch("k_hvp_epi"))) return rc;
        b0 += nv;
    }
    return ok();
}

cb_status md_adjoint_step(int64_t n, const double* x, const double* y, const double* z, const double* q,
                          const double* m, const cb_trap* trap, double dt, double eps2, int32_t prec, uint32_t flags,
                          double* lam, double* dldw, void* ws, size_t ws_bytes, void* stream) {
    const WsLayout L = ws_layout(CB_OP_ADJOINT, n > 0 ? n : 1, 1, 1, prec);
    cb_status rc = hvp_common("md_adjoint_step", n, prec, eps2, ws, ws_bytes, L.total);
    if (rc) return rc;
    if (!x || !y || !z || !q || !m || !lam || !dldw) return fail(CB_EINVAL, "md_adjoint_step: NULL argument");
    if (!trap_ok(trap, "md_adjoint_step", &rc)) return rc;
    if (trap->kind != 0 || trap->t_ramp1 > trap->t_ramp0 || trap->gamma != 0.0)
        return fail(CB_EUNSUPPORTED,
                    "md_adjoint_step: needs a static pseudo-potential trap (kind 0, no ramp, no friction)");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(CB_EINVAL, "md_adjoint_step: dt must be > 0");
    if (flags & ~CB_ADJ_FINAL) return fail(CB_EINVAL, "md_adjoint_step: unknown flags 0x%x", flags);
    const size_t lb = sizeof(double) * 9 * (size_t)n, ab = sizeof(double) * (size_t)n;
    const void* ins[] = {x, y, z, q, m};
    for (auto p : ins)
        if (overl(lam, p, lb, ab)) return fail(CB_EINVAL, "md_adjoint_step: lam aliases an input");
    if (overl(dldw, lam, 3 * sizeof(double), lb)) return fail(CB_EINVAL, "md_adjoint_step: dldw aliases lam");
    unsigned* fl = flags_ptr();
    if (!fl) return fail(CB_EHIP, "md_adjoint_step: device flag symbol not found");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int nb = (int)((n + kEpiThreads - 1) / kEpiThreads);
    const TrapK k = trap_k(*trap, 0.0);
    double* part = at(ws, L.part);
    double* eblk = at(ws, L.eblk);
    double* u = at(ws, L.aux);
    int S = 0;
    bool prescaled = false;
    const bool final_only = (flags & CB_ADJ_FINAL) != 0;
    if (!final_only) {
        k_adj_pre<<<nb, kEpiThreads, 0, st>>>((int)n, lam, m, dt, u);
        if ((rc = check_launch("k_adj_pre"))) return rc;
        const LaunchCfg cfg = get_cfg(CB_OP_ADJOINT, n, prec);
        if (is_sym(cfg.algo)) {
            // the Coulomb product H_C u by Newton's third law, finished into
            // part[3][n] (no trap term: k_adj_post adds it), scratch after it
            S = 1;
            prescaled = true;
            void* hws = static_cast<char*>(ws) + L.part + al256h(sizeof(double) * 3 * (size_t)n);
            if ((rc = launch_hvp_sym(prec, cfg, 1, (int)n, x, y, z, q, u, nullptr, TrapK{0.0, 0.0, 0.0}, eps2, hws,
                                     part, fl, st)))
                return rc;
        } else {
            const int jlen = split_len(n, cfg.splits);
            S = n_splits(n, jlen);
            if ((rc = launch_hvp(prec, cfg, 1, (int)n, x, y, z, q, u, eps2, jlen, part, st))) return rc;
        }
    }
    k_adj_post<<<nb, kEpiThreads, 0, st>>>((int)n, S, part, x, y, z, q, m, u, k, trap->wx, trap->wy, trap->wz, dt,
                                            final_only ? 1 : 0, prescaled ? 1 : 0, lam, eblk, fl);
    if ((rc = check_launch("k_adj_post"))) return rc;
    k_adj_final<<<1, kEpiThreads, 0, st>>>(nb, eblk, dldw);
    if ((rc = check_launch("k_adj_final"))) return rc;
    return ok();
}

}  // extern "C"
