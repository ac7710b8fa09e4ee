// Stepped ensemble path of md_run with many runs (the Kibble-Zurek statistics
// use case of the paper's introduction).  Instead of one workgroup per run
// (batched.hip), every velocity-Verlet step is two launches over all runs at
// once, so that no run's size bounds the makespan:
//   1. k_pair_sym_ens: the Newton's-third-law tiles (pair_sym.hpp) of every
//      run, one wave per tile, longest tiles first.  A tile entry holds its
//      run's first ion and size, the slot of its partials, and its row and
//      segment.
//   2. k_ens_step: per 64 ions of one run, the finish of the force (pairs
//      inside the ion's own i-block, the i sums of its row and the reactions
//      from the rows above, each summed in a fixed order) fused with the trap,
//      the kick and the next drift.  The drift writes the other of two
//      position buffers: other workgroups of the launch still read the
//      current positions of the same i-block.
// Energy records add each ion's Coulomb potential (a direct pass over its
// run) on the recording step, and k_ens_energy sums the 64-ion partials of
// each run in chunk order.  Results do not depend on timing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "internal.hpp"
#include "pair_sym.hpp"
#include "step_common.hpp"

namespace cb {

template <int PREC, int P>
__global__ void __launch_bounds__(64, (sym_waves<PREC, P>())) k_pair_sym_ens(const double* __restrict__ x,
                                                                     const double* __restrict__ y,
                                                                     const double* __restrict__ z,
                                                                     const double* __restrict__ q, double eps2,
                                                                     int JL, const int4* __restrict__ tiles,
                                                                     double* __restrict__ Pi,
                                                                     double* __restrict__ R) {
    __shared__ __align__(16) double red_buf[12 * kRedStride];
    const int4 tl = tiles[blockIdx.x];  // first ion, ions, slot, row << 16 | segment
    const int o = tl.x;
    sym_tile<PREC, P, 1>(tl.y, x + o, y + o, z + o, q + o, eps2, JL, tl.w >> 16, tl.w & 0xffff, tl.z, red_buf, Pi,
                         R);
}

struct EnsParams {
    const int2* chunks;    // [nchunk] (run, first ion of the chunk within the run)
    const int4* runs;      // [nrun] (first ion, ions, first row-start entry, first chunk)
    const int* rowstart;   // per run, rows 0..nI: partial slot of (row, segment 0); concatenated
    const cb_trap* traps;  // [nrun]
    const double* Pi;      // [slots][3][IB]
    const double* R;       // [slots][3][JL]
    const double *x, *y, *z;  // positions at this step (read)
    double *xn, *yn, *zn;     // positions after the drift (written)
    const double* q;
    const double* m;
    double *vx, *vy, *vz, *ax, *ay, *az;
    int IB, JL, lgJL;
    double eps2, t0, dt;
    long long step;     // the trap is taken at step_time(t0, dt, step)
    unsigned mode;      // EPI_ACCEL, EPI_KICK, EPI_DRIFT, EPI_ENERGY
    double* echunk;     // [nchunk][3]: K, U_C, U_trap of each chunk (EPI_ENERGY)
    unsigned* flags;
};

constexpr int kEnsVals = 10;  // 3 direct, 3 row i sums, 3 reactions, potential

template <int PREC>
__global__ void __launch_bounds__(64 * kFinishParts) k_ens_step(EnsParams P) {
    __shared__ double red[kFinishParts][kEnsVals][64];
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int2 ch = P.chunks[blockIdx.x];
    const int4 ru = P.runs[ch.x];
    const int o = ru.x, n = ru.y;
    const double *X = P.x + o, *Y = P.y + o, *Z = P.z + o, *Q = P.q + o;
    const int* rowstart = P.rowstart + ru.z;
    const int k0 = ch.y, k = k0 + lane, kc = min(k, n - 1);
    const unsigned mode = P.mode;
    const double xk = X[kc], yk = Y[kc], zk = Z[kc];
    const SeriesK K;
    double v[kEnsVals];
#pragma unroll
    for (int c = 0; c < kEnsVals; ++c) v[c] = 0.0;
    if (mode & (EPI_ACCEL | EPI_KICK)) {
        const int IB = P.IB, JL = P.JL, lgJL = P.lgJL;
        const int Ik = k0 / IB;
        const int b0 = Ik * IB, b1 = min(n, b0 + IB);
        int lo, hi;
        share(b0, b1, w, lo, hi);
        for (int j = lo; j < hi; ++j) {
            const double dx = xk - X[j], dy = yk - Y[j], dz = zk - Z[j];
            const double r2 = __builtin_fma(dx, dx, __builtin_fma(dy, dy, __builtin_fma(dz, dz, P.eps2)));
            double s = sym_s<PREC>(r2, Q[j], K);
            if (j == kc) s = 0.0;
            v[0] = __builtin_fma(dx, s, v[0]);
            v[1] = __builtin_fma(dy, s, v[1]);
            v[2] = __builtin_fma(dz, s, v[2]);
        }
        const int off = kc - b0;
        share(rowstart[Ik], rowstart[Ik + 1], w, lo, hi);
        for (int t = lo; t < hi; ++t) {
            const double* Pt = P.Pi + (size_t)t * 3 * IB + off;
            v[3] += Pt[0];
            v[4] += Pt[IB];
            v[5] += Pt[2 * IB];
        }
        share(0, Ik, w, lo, hi);
        for (int I = lo; I < hi; ++I) {
            const int rel = kc - (I + 1) * IB;
            const int sI = rel >> lgJL;
            const double* Rt = P.R + (size_t)(rowstart[I] + sI) * 3 * JL + (rel - (sI << lgJL));
            v[6] += Rt[0];
            v[7] += Rt[JL];
            v[8] += Rt[2 * JL];
        }
    }
    if (mode & EPI_ENERGY) {  // potential sum_j q_j / r_kj over the whole run
        int lo, hi;
        share(0, n, w, lo, hi);
        for (int j = lo; j < hi; ++j) {
            const double dx = xk - X[j], dy = yk - Y[j], dz = zk - Z[j];
            const double r2 = __builtin_fma(dx, dx, __builtin_fma(dy, dy, __builtin_fma(dz, dz, P.eps2)));
            double s, y;
            inv_r<PREC, false, true>(r2, Q[j], K, s, y);
            if (j == kc) y = 0.0;
            v[9] = __builtin_fma(Q[j], y, v[9]);
        }
    }
#pragma unroll
    for (int c = 0; c < kEnsVals; ++c) red[w][c][lane] = v[c];
    __syncthreads();
    if (w != 0) return;
    double tot[kEnsVals];
#pragma unroll
    for (int c = 0; c < kEnsVals; ++c) {
        double a = red[0][c][lane];
#pragma unroll
        for (int u = 1; u < kFinishParts; ++u) a += red[u][c][lane];
        tot[c] = a;
    }
    double eK = 0.0, eC = 0.0, eT = 0.0;
    if (k < n) {
        const int i = o + k;
        const double qk = Q[k];
        const double Fx = kCoulomb * (tot[3] + qk * (tot[0] - tot[6]));
        const double Fy = kCoulomb * (tot[4] + qk * (tot[1] - tot[7]));
        const double Fz = kCoulomb * (tot[5] + qk * (tot[2] - tot[8]));
        const cb_trap& tr = P.traps[ch.x];
        const TrapK kk = trap_k(tr, step_time(P.t0, P.dt, P.step));
        double x = xk, y = yk, z = zk;
        double vx = P.vx[i], vy = P.vy[i], vz = P.vz[i];
        double ax = P.ax[i], ay = P.ay[i], az = P.az[i];
        const double mi = P.m[i];
        bool ok = true;
        if (mode & (EPI_ACCEL | EPI_KICK)) {
            const double anx = Fx / mi - kk.kx * x;
            const double any = Fy / mi - kk.ky * y;
            const double anz = Fz / mi - kk.kz * z;
            if (mode & EPI_KICK) {
                const double h = 0.5 * P.dt;
                if (tr.gamma == 0.0) {
                    vx = vx + h * (ax + anx);
                    vy = vy + h * (ay + any);
                    vz = vz + h * (az + anz);
                } else {  // friction -g v by the trapezoidal rule, g = Gamma / m_i
                    const double g = tr.gamma / mi, lo = 1.0 - g * h, hi = 1.0 + g * h;
                    vx = (vx * lo + h * (ax + anx)) / hi;
                    vy = (vy * lo + h * (ay + any)) / hi;
                    vz = (vz * lo + h * (az + anz)) / hi;
                }
                P.vx[i] = vx;
                P.vy[i] = vy;
                P.vz[i] = vz;
            }
            ax = anx;
            ay = any;
            az = anz;
            P.ax[i] = ax;
            P.ay[i] = ay;
            P.az[i] = az;
            ok = finite3(ax, ay, az) && finite3(vx, vy, vz);
        }
        if (mode & EPI_ENERGY) {
            eK = 0.5 * mi * (vx * vx + vy * vy + vz * vz);
            eC = 0.5 * kCoulomb * qk * tot[9];
            eT = 0.5 * mi * (kk.kx * x * x + kk.ky * y * y + kk.kz * z * z);
            ok = ok && finite3(eK, eC, eT);
        }
        if (mode & EPI_DRIFT) {
            const double dt = P.dt, h2 = 0.5 * dt * dt;
            if (tr.gamma == 0.0) {
                x = x + vx * dt + h2 * ax;
                y = y + vy * dt + h2 * ay;
                z = z + vz * dt + h2 * az;
            } else {  // the drift sees the friction acceleration -g v too
                const double g = tr.gamma / mi;
                x = x + vx * dt + h2 * (ax - g * vx);
                y = y + vy * dt + h2 * (ay - g * vy);
                z = z + vz * dt + h2 * (az - g * vz);
            }
            P.xn[i] = x;
            P.yn[i] = y;
            P.zn[i] = z;
            ok = ok && finite3(x, y, z);
        }
        if (!ok) atomicOr(P.flags, 1u);
    }
    if (mode & EPI_ENERGY) {
        // fixed butterfly over the wave: every lane ends with the same sums
#pragma unroll
        for (int d = 32; d > 0; d >>= 1) {
            eK += __shfl_xor(eK, d);
            eC += __shfl_xor(eC, d);
            eT += __shfl_xor(eT, d);
        }
        if (lane == 0) {
            P.echunk[(size_t)blockIdx.x * 3 + 0] = eK;
            P.echunk[(size_t)blockIdx.x * 3 + 1] = eC;
            P.echunk[(size_t)blockIdx.x * 3 + 2] = eT;
        }
    }
}

// Record `rec` of every run: the chunk partials of run r summed in chunk
// order into energies[r][rec][0..3] = K, U_C, U_trap, E.
__global__ void __launch_bounds__(64) k_ens_energy(const int4* __restrict__ runs, int nrun, int nchunk,
                                                   const double* __restrict__ echunk, double* __restrict__ energies,
                                                   long long nrec, long long rec) {
    const int r = blockIdx.x;
    const int c0 = runs[r].w, c1 = r + 1 < nrun ? runs[r + 1].w : nchunk;
    double a = 0.0, b = 0.0, c = 0.0;
    for (int k = c0 + (int)threadIdx.x; k < c1; k += 64) {
        a += echunk[(size_t)k * 3 + 0];
        b += echunk[(size_t)k * 3 + 1];
        c += echunk[(size_t)k * 3 + 2];
    }
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) {
        a += __shfl_xor(a, d);
        b += __shfl_xor(b, d);
        c += __shfl_xor(c, d);
    }
    if (threadIdx.x == 0) {
        double* e = energies + ((size_t)r * nrec + rec) * 4;
        e[0] = a;
        e[1] = b;
        e[2] = c;
        e[3] = a + b + c;
    }
}

// ----------------------------------------------------------------- host

static size_t al(size_t b) { return (b + 255) / 256 * 256; }

bool ens_cfg_ok(int p, int jl) { return (p == 4 || p == 8) && (jl == 256 || jl == 512); }

// Tables of one ensemble at (P, JL): what the workspace must hold.
struct EnsTables {
    std::vector<int4> tiles, runs;
    std::vector<int> rowstart;
    std::vector<int2> chunks;
    size_t bytes = 0;
};

static EnsTables ens_tables(int nrun, const int64_t* offsets, int P, int JL) {
    EnsTables E;
    const int IB = 64 * P;
    struct Tile {
        int4 t;
        int len;
    };
    std::vector<Tile> tl;
    int slot = 0;
    E.runs.resize(nrun);
    for (int r = 0; r < nrun; ++r) {
        const int o = (int)offsets[r], n = (int)(offsets[r + 1] - offsets[r]);
        const int nI = (n + IB - 1) / IB;
        E.runs[r] = make_int4(o, n, (int)E.rowstart.size(), (int)E.chunks.size());
        for (int I = 0; I < nI; ++I) {
            E.rowstart.push_back(slot);
            const int ns = sym_nseg(n, IB, JL, I);
            for (int sg = 0; sg < ns; ++sg) {
                const int j0 = (I + 1) * IB + sg * JL;
                tl.push_back({make_int4(o, n, slot, (I << 16) | sg), std::min(JL, n - j0)});
                ++slot;
            }
        }
        E.rowstart.push_back(slot);
        for (int k0 = 0; k0 < n; k0 += 64) E.chunks.push_back(make_int2(r, k0));
    }
    // longest tiles first, so that the short ones fill the end of the launch
    std::stable_sort(tl.begin(), tl.end(), [](const Tile& a, const Tile& b) { return a.len > b.len; });
    E.tiles.reserve(tl.size());
    for (const Tile& t : tl) E.tiles.push_back(t.t);
    const size_t T = E.tiles.size(), nch = E.chunks.size(), ntot = (size_t)offsets[nrun];
    E.bytes = al(sizeof(int4) * (T + 1)) + al(sizeof(int4) * nrun) + al(sizeof(int) * E.rowstart.size()) +
              al(sizeof(int2) * nch) + al(sizeof(cb_trap) * nrun) + al(sizeof(double) * 3 * IB * (T + 1)) +
              al(sizeof(double) * 3 * (size_t)JL * (T + 1)) + al(sizeof(double) * 3 * ntot) +
              al(sizeof(double) * 3 * nch);
    return E;
}

// Upper bound of ens_tables(...).bytes over every ensemble of ntot ions in
// nrun runs of at most kMaxBatchIons, for every allowed (P, JL).  A run of n
// ions has at most n^2 / (2 IB JL) + n / IB tiles.
size_t ens_ws_bound(int64_t ntot, int32_t nrun) {
    size_t best = 0;
    const double N = (double)ntot;
    for (int P : {4, 8})
        for (int JL : {256, 512}) {
            const int IB = 64 * P;
            const size_t T = (size_t)std::ceil(N * (0.5 * kMaxBatchIons / ((double)IB * JL) + 1.0 / IB)) + nrun;
            const size_t rows = (size_t)std::ceil(N / IB) + 2 * (size_t)nrun;
            const size_t nch = (size_t)std::ceil(N / 64) + nrun;
            const size_t b = al(sizeof(int4) * (T + 1)) + al(sizeof(int4) * nrun) + al(sizeof(int) * rows) +
                             al(sizeof(int2) * nch) + al(sizeof(cb_trap) * nrun) +
                             al(sizeof(double) * 3 * IB * (T + 1)) + al(sizeof(double) * 3 * (size_t)JL * (T + 1)) +
                             al(sizeof(double) * 3 * (size_t)ntot) + al(sizeof(double) * 3 * nch);
            best = std::max(best, b);
        }
    return best;
}

template <int PREC, int P>
static void go_ens_pair(unsigned T, const double* x, const double* y, const double* z, const double* q, double eps2,
                        int JL, const int4* tiles, double* Pi, double* R, hipStream_t st) {
    k_pair_sym_ens<PREC, P><<<T, 64, 0, st>>>(x, y, z, q, eps2, JL, tiles, Pi, R);
}

template <int PREC>
static void go_ens_pair_p(int P, unsigned T, const double* x, const double* y, const double* z, const double* q,
                          double eps2, int JL, const int4* tiles, double* Pi, double* R, hipStream_t st) {
    if (P == 8) go_ens_pair<PREC, 8>(T, x, y, z, q, eps2, JL, tiles, Pi, R, st);
    else go_ens_pair<PREC, 4>(T, x, y, z, q, eps2, JL, tiles, Pi, R, st);
}

cb_status md_run_ensemble(int32_t nrun, const int64_t* offsets, const cb_state* s, const double* q,
                          const double* m, const cb_trap* traps, double t0, double dt, int64_t nsteps, double eps2,
                          int32_t prec, uint32_t flags, double* energies, int64_t every, int P, int JL, void* ws,
                          size_t ws_bytes, hipStream_t st) {
    if (!ens_cfg_ok(P, JL)) return fail(CB_EINVAL, "md_run: ensemble configuration p=%d JL=%d not supported", P, JL);
    const int IB = 64 * P;
    const EnsTables E = ens_tables(nrun, offsets, P, JL);
    if (ws_bytes < E.bytes)
        return fail(CB_ENOWS, "md_run: the ensemble path needs %zu workspace bytes, has %zu", E.bytes, ws_bytes);
    unsigned* fl = flags_ptr();
    if (!fl) return fail(CB_EHIP, "md_run: device flag symbol not found");
    const size_t T = E.tiles.size(), nch = E.chunks.size(), ntot = (size_t)offsets[nrun];

    char* base = static_cast<char*>(ws);
    auto carve = [&](size_t bytes) {
        char* p = base;
        base += al(bytes);
        return p;
    };
    int4* d_tiles = reinterpret_cast<int4*>(carve(sizeof(int4) * (T + 1)));
    int4* d_runs = reinterpret_cast<int4*>(carve(sizeof(int4) * nrun));
    int* d_rows = reinterpret_cast<int*>(carve(sizeof(int) * E.rowstart.size()));
    int2* d_chunks = reinterpret_cast<int2*>(carve(sizeof(int2) * nch));
    cb_trap* d_traps = reinterpret_cast<cb_trap*>(carve(sizeof(cb_trap) * nrun));
    double* Pi = reinterpret_cast<double*>(carve(sizeof(double) * 3 * IB * (T + 1)));
    double* R = reinterpret_cast<double*>(carve(sizeof(double) * 3 * (size_t)JL * (T + 1)));
    double* pos2 = reinterpret_cast<double*>(carve(sizeof(double) * 3 * ntot));
    double* echunk = reinterpret_cast<double*>(carve(sizeof(double) * 3 * nch));

    // Host buffers are pageable: HIP consumes them before hipMemcpyAsync returns.
    auto up = [&](void* dst, const void* src, size_t bytes) {
        return bytes == 0 || hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st) == hipSuccess;
    };
    if (!up(d_tiles, E.tiles.data(), sizeof(int4) * T) || !up(d_runs, E.runs.data(), sizeof(int4) * nrun) ||
        !up(d_rows, E.rowstart.data(), sizeof(int) * E.rowstart.size()) ||
        !up(d_chunks, E.chunks.data(), sizeof(int2) * nch) || !up(d_traps, traps, sizeof(cb_trap) * nrun))
        return fail(CB_EHIP, "md_run: ensemble table upload failed");

    double* bufA[3] = {s->x, s->y, s->z};
    double* bufB[3] = {pos2, pos2 + ntot, pos2 + 2 * ntot};
    double** cur = bufA;
    double** nxt = bufB;

    EnsParams EP{};
    EP.chunks = d_chunks;
    EP.runs = d_runs;
    EP.rowstart = d_rows;
    EP.traps = d_traps;
    EP.Pi = Pi;
    EP.R = R;
    EP.q = q;
    EP.m = m;
    EP.vx = s->vx; EP.vy = s->vy; EP.vz = s->vz;
    EP.ax = s->ax; EP.ay = s->ay; EP.az = s->az;
    EP.IB = IB;
    EP.JL = JL;
    int lgJL = 0;
    while ((1 << lgJL) < JL) ++lgJL;
    EP.lgJL = lgJL;
    EP.eps2 = eps2;
    EP.t0 = t0;
    EP.dt = dt;
    EP.echunk = echunk;
    EP.flags = fl;
    const long long nrec = energies ? nsteps / every + 1 : 0;

    auto pair_stage = [&]() -> cb_status {
        if (T == 0) return CB_OK;
        switch (prec) {
            case CB_FP64: go_ens_pair_p<PREC_FP64>(P, (unsigned)T, cur[0], cur[1], cur[2], q, eps2, JL, d_tiles, Pi, R, st); break;
            case CB_MIXED: go_ens_pair_p<PREC_MIXED>(P, (unsigned)T, cur[0], cur[1], cur[2], q, eps2, JL, d_tiles, Pi, R, st); break;
            case CB_FP64_IEEE: go_ens_pair_p<PREC_IEEE>(P, (unsigned)T, cur[0], cur[1], cur[2], q, eps2, JL, d_tiles, Pi, R, st); break;
            default: go_ens_pair_p<PREC_FP32>(P, (unsigned)T, cur[0], cur[1], cur[2], q, eps2, JL, d_tiles, Pi, R, st); break;
        }
        return check_launch("k_pair_sym_ens");
    };
    // finish + trap + kick / drift of step `step`; the drift swaps the buffers
    auto step_launch = [&](long long step, unsigned mode) -> cb_status {
        EP.x = cur[0]; EP.y = cur[1]; EP.z = cur[2];
        EP.xn = nxt[0]; EP.yn = nxt[1]; EP.zn = nxt[2];
        EP.step = step;
        EP.mode = mode;
        switch (prec) {
            case CB_FP64: k_ens_step<PREC_FP64><<<(unsigned)nch, 64 * kFinishParts, 0, st>>>(EP); break;
            case CB_MIXED: k_ens_step<PREC_MIXED><<<(unsigned)nch, 64 * kFinishParts, 0, st>>>(EP); break;
            case CB_FP64_IEEE: k_ens_step<PREC_IEEE><<<(unsigned)nch, 64 * kFinishParts, 0, st>>>(EP); break;
            default: k_ens_step<PREC_FP32><<<(unsigned)nch, 64 * kFinishParts, 0, st>>>(EP); break;
        }
        cb_status rc = check_launch("k_ens_step");
        if (rc) return rc;
        if (mode & EPI_DRIFT) std::swap(cur, nxt);
        return CB_OK;
    };
    auto record = [&](long long rec) -> cb_status {
        k_ens_energy<<<(unsigned)nrun, 64, 0, st>>>(d_runs, nrun, (int)nch, echunk, energies, nrec, rec);
        return check_launch("k_ens_energy");
    };

    cb_status rc;
    const bool rec0 = energies != nullptr;
    const bool init = (flags & CB_INIT_ACCEL) != 0;
    const unsigned mode0 = (init ? EPI_ACCEL : 0u) | (rec0 ? EPI_ENERGY : 0u) | (nsteps > 0 ? EPI_DRIFT : 0u);
    if (init && (rc = pair_stage())) return rc;
    if (mode0) {
        if ((rc = step_launch(0, mode0))) return rc;
        if (rec0 && (rc = record(0))) return rc;
    }
    for (long long k = 1; k <= nsteps; ++k) {
        const bool rec = rec0 && (k % every == 0);
        if ((rc = pair_stage())) return rc;
        if ((rc = step_launch(k, EPI_KICK | (rec ? EPI_ENERGY : 0u) | (k < nsteps ? EPI_DRIFT : 0u)))) return rc;
        if (rec && (rc = record(k / every))) return rc;
    }
    if (cur != bufA)
        for (int c = 0; c < 3; ++c)
            if (hipMemcpyAsync(bufA[c], cur[c], sizeof(double) * ntot, hipMemcpyDeviceToDevice, st) != hipSuccess)
                return fail(CB_EHIP, "md_run: copy of the final positions failed");
    return ok();
}

}  // namespace cb
