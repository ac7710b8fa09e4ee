"""Seeded synthetic inputs for the five workloads (shared by tests, bench and
smoke; holds none of the force, trap or integrator arithmetic).

Every array is float64 numpy, SI units (m, m/s, C, kg).  Each generator uses
``numpy.random.Generator(PCG64(seed))`` with the default seed
``BASE_SEED + workload number``, so the GPU path and the CPU oracle consume the
same bytes.  The recipes (all synthetic; the paper names no dataset):

1. ``cloud1024``: N=1024 singly charged 40 u ions, positions N(0, (20 um)^2) per
   axis, Maxwell velocities at 10 mK, static pseudo-potential trap
   wx = wy = 2 pi 1 MHz, wz = 2 pi 0.2 MHz, dt = 1 ns, 100 steps.
2. ``rf32768``: N=32768, uniform in the ellipsoid with semi-axes
   (150, 150, 1000) um, at rest, explicit RF drive a = 0, q = 0.3,
   Omega = 2 pi 10 MHz, phase 0, wz = 2 pi 0.1 MHz, dt = one twentieth of
   the RF period (5 ns), 1000 steps.
3. ``cloud100k``: N=100000, positions N(0, diag(150, 150, 800)^2 um^2), at rest,
   charge +e with exactly round(0.01 N) ions at +2e chosen by a seeded
   permutation, workload 1's trap, dt = 1 ns, 200 steps.
4. ``kz512``: 512 independent runs, N_r uniform in [64, 4096]; each starts as a
   Gaussian cloud sized like the cold crystal of its trap (density estimate
   below) with 10 mK Maxwell velocities; wx, wy ramp linearly from
   2 pi 1.5 MHz to 2 pi 0.6 MHz over 0 .. 20 us, wz = 2 pi 0.15 MHz, dt = 2 ns,
   10^4 steps.
5. ``crystal8192``: N=8192, static trap wx = wy = 2 pi 1 MHz, wz = 2 pi 0.05 MHz,
   a Gaussian start (to be relaxed to the crystal by the minimiser) and 10 mK
   Maxwell velocities for the gradient run; dt = 1 ns, 2000 steps,
   checkpoints every 50 steps.

Cloud sizes for 4 and 5 use the cold-plasma density n0 = eps0 m (wx^2+wy^2+wz^2)/e^2
and a spheroid whose axis ratio is the inverse trap-frequency ratio, with
Gaussian sigma = semi-axis / sqrt(5) (equal second moment); this is only a
starting guess, not part of the method.
"""
from __future__ import annotations

import math

import numpy as np

BASE_SEED = 2106_11143

E_CHARGE = 1.602176634e-19  # C (CODATA 2018, exact)
AMU = 1.66053906660e-27  # kg (CODATA 2018)
K_B = 1.380649e-23  # J/K (CODATA 2018, exact)
EPS0_INPUT = 8.8541878128e-12  # F/m, only for the cloud-size guess
MASS_40U = 40.0 * AMU
TWO_PI = 2.0 * math.pi

TRAP_FIELDS = ("kind", "wx", "wy", "wz", "rf_a", "rf_q", "rf_omega", "rf_phase", "gamma",
               "wx1", "wy1", "t_ramp0", "t_ramp1")


def trap_dict(**kw) -> dict:
    d = {f: 0.0 for f in TRAP_FIELDS}
    d["kind"] = 0
    d.update(kw)
    return d


def pseudo_trap(fx_hz, fy_hz, fz_hz) -> dict:
    return trap_dict(kind=0, wx=TWO_PI * fx_hz, wy=TWO_PI * fy_hz, wz=TWO_PI * fz_hz)


def rf_trap(a, q, omega_hz, fz_hz, phase=0.0) -> dict:
    return trap_dict(kind=1, rf_a=a, rf_q=q, rf_omega=TWO_PI * omega_hz, rf_phase=phase, wz=TWO_PI * fz_hz)


def ramp_trap(f0_hz, f1_hz, fz_hz, t0, t1) -> dict:
    return trap_dict(kind=0, wx=TWO_PI * f0_hz, wy=TWO_PI * f0_hz, wz=TWO_PI * fz_hz,
                     wx1=TWO_PI * f1_hz, wy1=TWO_PI * f1_hz, t_ramp0=t0, t_ramp1=t1)


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def maxwell(g: np.random.Generator, n: int, T: float, m: float) -> np.ndarray:
    """(3, n) velocities, each component N(0, k_B T / m)."""
    return g.normal(0.0, math.sqrt(K_B * T / m), size=(3, n))


def uniform_ellipsoid(g: np.random.Generator, n: int, semi) -> np.ndarray:
    """(3, n) points uniform in the ellipsoid with the given semi-axes
    (direction uniform on the sphere times u^(1/3), then scaled)."""
    d = g.normal(size=(3, n))
    d /= np.linalg.norm(d, axis=0)
    r = g.random(n) ** (1.0 / 3.0)
    return d * r * np.asarray(semi, dtype=np.float64)[:, None]


def crystal_sigma(n: int, wx: float, wy: float, wz: float, m: float = MASS_40U) -> np.ndarray:
    """Gaussian sigma (3,) of a starting cloud sized like the cold crystal."""
    n0 = EPS0_INPUT * m * (wx * wx + wy * wy + wz * wz) / E_CHARGE ** 2
    R = (3.0 * n / (4.0 * math.pi * n0)) ** (1.0 / 3.0)
    wr = math.sqrt(0.5 * (wx * wx + wy * wy))
    aspect = max(wr / wz, 1e-3)  # semi_z / semi_r
    rr = R / aspect ** (1.0 / 3.0)
    return np.array([rr, rr, rr * aspect]) / math.sqrt(5.0)


def _pack(pos, vel, q, m, **extra) -> dict:
    d = dict(x=np.ascontiguousarray(pos[0]), y=np.ascontiguousarray(pos[1]), z=np.ascontiguousarray(pos[2]),
             vx=np.ascontiguousarray(vel[0]), vy=np.ascontiguousarray(vel[1]), vz=np.ascontiguousarray(vel[2]),
             q=np.ascontiguousarray(q), m=np.ascontiguousarray(m), n=int(pos.shape[1]))
    d.update(extra)
    return d


def cloud1024(n: int = 1024, seed: int | None = None) -> dict:
    g = rng(BASE_SEED + 1 if seed is None else seed)
    pos = g.normal(0.0, 20e-6, size=(3, n))
    vel = maxwell(g, n, 10e-3, MASS_40U)
    return _pack(pos, vel, np.full(n, E_CHARGE), np.full(n, MASS_40U), name="cloud1024",
                 trap=pseudo_trap(1.0e6, 1.0e6, 0.2e6), dt=1e-9, nsteps=100, t0=0.0, eps2=0.0)


def rf32768(n: int = 32768, seed: int | None = None) -> dict:
    g = rng(BASE_SEED + 2 if seed is None else seed)
    pos = uniform_ellipsoid(g, n, (150e-6, 150e-6, 1000e-6))
    vel = np.zeros((3, n))
    omega_hz = 10.0e6
    dt = 1.0 / omega_hz / 20.0
    return _pack(pos, vel, np.full(n, E_CHARGE), np.full(n, MASS_40U), name="rf32768",
                 trap=rf_trap(0.0, 0.3, omega_hz, 0.1e6), dt=dt, nsteps=1000, t0=0.0, eps2=0.0)


def cloud100k(n: int = 100000, seed: int | None = None) -> dict:
    g = rng(BASE_SEED + 3 if seed is None else seed)
    pos = g.normal(size=(3, n)) * np.array([150e-6, 150e-6, 800e-6])[:, None]
    q = np.full(n, E_CHARGE)
    q[g.permutation(n)[: int(round(0.01 * n))]] = 2.0 * E_CHARGE
    vel = np.zeros((3, n))
    return _pack(pos, vel, q, np.full(n, MASS_40U), name="cloud100k",
                 trap=pseudo_trap(1.0e6, 1.0e6, 0.2e6), dt=1e-9, nsteps=200, t0=0.0, eps2=0.0)


def kz512(nrun: int = 512, nmin: int = 64, nmax: int = 4096, nsteps: int = 10000,
          seed: int | None = None) -> dict:
    """Packed ensemble: arrays are the runs' SoA arrays concatenated, with
    offsets (nrun+1,) int64 (CSR) and one trap dict per run."""
    g = rng(BASE_SEED + 4 if seed is None else seed)
    ns = g.integers(nmin, nmax + 1, size=nrun)
    trap = ramp_trap(1.5e6, 0.6e6, 0.15e6, 0.0, 20e-6)
    pos, vel = [], []
    for nr in ns:
        sig = crystal_sigma(int(nr), trap["wx"], trap["wy"], trap["wz"])
        pos.append(g.normal(size=(3, nr)) * sig[:, None])
        vel.append(maxwell(g, int(nr), 10e-3, MASS_40U))
    pos = np.concatenate(pos, axis=1)
    vel = np.concatenate(vel, axis=1)
    ntot = pos.shape[1]
    offsets = np.zeros(nrun + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(ns)
    return _pack(pos, vel, np.full(ntot, E_CHARGE), np.full(ntot, MASS_40U), name="kz512",
                 offsets=offsets, nrun=int(nrun), traps=[dict(trap) for _ in range(nrun)], trap=trap,
                 dt=2e-9, nsteps=int(nsteps), t0=0.0, eps2=0.0)


def crystal8192(n: int = 8192, seed: int | None = None) -> dict:
    g = rng(BASE_SEED + 5 if seed is None else seed)
    trap = pseudo_trap(1.0e6, 1.0e6, 0.05e6)
    sig = crystal_sigma(n, trap["wx"], trap["wy"], trap["wz"])
    pos = g.normal(size=(3, n)) * sig[:, None]
    vel = maxwell(g, n, 10e-3, MASS_40U)
    return _pack(pos, vel, np.full(n, E_CHARGE), np.full(n, MASS_40U), name="crystal8192",
                 trap=trap, dt=1e-9, nsteps=2000, checkpoint_every=50, t0=0.0, eps2=0.0)


def group_by_charge(d: dict) -> dict:
    """The same ions relabelled so that equal charges are contiguous (a
    stable sort by charge; for cloud100k the +2e ions come last): the same
    physical system, ordered as the paper's split of species into separate
    N-body sub-problems (section 2).  perm: grouped ion k is ion perm[k] of d."""
    perm = np.argsort(d["q"], kind="stable")
    out = dict(d)
    for k in ("x", "y", "z", "vx", "vy", "vz", "q", "m"):
        out[k] = np.ascontiguousarray(d[k][perm])
    out["perm"] = perm
    out["name"] = d.get("name", "") + "_grouped"
    return out


WORKLOADS = {1: cloud1024, 2: rf32768, 3: cloud100k, 4: kz512, 5: crystal8192}


def make(k: int, **kw) -> dict:
    """Workload k (1..5) with optional overrides (n=..., seed=...)."""
    return WORKLOADS[k](**kw)


def state9(d: dict) -> np.ndarray:
    """(9, n) state array x y z vx vy vz ax ay az (accelerations zero)."""
    n = d["n"]
    s = np.zeros((9, n))
    s[0], s[1], s[2] = d["x"], d["y"], d["z"]
    s[3], s[4], s[5] = d["vx"], d["vy"], d["vz"]
    return s
