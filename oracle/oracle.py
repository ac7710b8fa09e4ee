"""Python face of the FP64 CPU oracle (``coulomb_oracle.c``).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import this module.  The product
path (the HIP library and ``paper_2106_11143_amd``) never imports, links or
runs anything under ``oracle/``, and this module imports nothing from it.

Every function here is a thin ctypes call into the C oracle, which follows the
paper's equations of motion (section 2, eq. (1)), its velocity-Verlet list
(section 2) and its classical double loop (section 3); see the header of
``coulomb_oracle.c`` for the readings taken.  Arrays are float64 numpy arrays.

``two_ion_error_model`` restates the paper's section 4 error estimate (used to
pin the constants against Table 1); it is analysis, not part of the hot path.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import tempfile

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_BUILD = os.path.join(_HERE, "_build")
_LIB_PATH = os.path.join(_BUILD, "liboracle.so")
_SOURCES = {
    "coulomb_oracle.c": ["-O2", "-ffp-contract=off", "-fno-fast-math"],
    "coulomb_oracle_plain.c": ["-O3", "-march=native"],
}

# Boltzmann constant (CODATA 2018, exact), used only by the section 4 error model.
K_B = 1.380649e-23


class Trap(C.Structure):
    """Mirror of the oracle's trap record (field order and types must match)."""

    _fields_ = [
        ("kind", C.c_int32),
        ("wx", C.c_double), ("wy", C.c_double), ("wz", C.c_double),
        ("rf_a", C.c_double), ("rf_q", C.c_double), ("rf_omega", C.c_double), ("rf_phase", C.c_double),
        ("gamma", C.c_double),
        ("wx1", C.c_double), ("wy1", C.c_double), ("t_ramp0", C.c_double), ("t_ramp1", C.c_double),
    ]


def make_trap(d: dict | None) -> Trap:
    t = Trap()
    for name, _ in Trap._fields_:
        setattr(t, name, (d or {}).get(name, 0))
    return t


def build(force: bool = False) -> str:
    """Compile the oracle with gcc into oracle/_build/liboracle.so."""
    srcs = [os.path.join(_HERE, s) for s in _SOURCES]
    if not force and os.path.exists(_LIB_PATH):
        newest = max(os.path.getmtime(s) for s in srcs)
        if os.path.getmtime(_LIB_PATH) >= newest:
            return _LIB_PATH
    os.makedirs(_BUILD, exist_ok=True)
    with tempfile.TemporaryDirectory(dir=_BUILD) as tmp:
        objs = []
        for src, flags in _SOURCES.items():
            obj = os.path.join(tmp, src.replace(".c", ".o"))
            subprocess.run(["gcc", "-std=c11", "-fPIC", "-fopenmp", "-Wall", "-c", *flags,
                            os.path.join(_HERE, src), "-o", obj], check=True)
            objs.append(obj)
        out = os.path.join(tmp, "liboracle.so")
        subprocess.run(["gcc", "-shared", "-fopenmp", *objs, "-o", out, "-lm"], check=True)
        os.replace(out, _LIB_PATH)
    return _LIB_PATH


_lib = None
_P = C.POINTER(C.c_double)
_PI64 = C.POINTER(C.c_int64)


def lib():
    global _lib
    if _lib is None:
        L = C.CDLL(build())
        L.or_coulomb_constant.restype = C.c_double
        L.or_forces.argtypes = [C.c_int64, _P, _P, _P, _P, C.c_double, C.c_int64, _PI64, _P, _P, _P, _P, C.c_int]
        L.or_coulomb_energy.argtypes = [C.c_int64, _P, _P, _P, _P, C.c_double, _P, C.c_int]
        L.or_coulomb_energy.restype = C.c_double
        L.or_trap_k.argtypes = [C.POINTER(Trap), C.c_double, _P]
        L.or_trap_energy.argtypes = [C.c_int64, _P, _P, _P, _P, C.POINTER(Trap), C.c_double]
        L.or_trap_energy.restype = C.c_double
        L.or_kinetic_energy.argtypes = [C.c_int64, _P, _P, _P, _P]
        L.or_kinetic_energy.restype = C.c_double
        L.or_accel.argtypes = [C.c_int64, _P, _P, _P, _P, _P, C.POINTER(Trap), C.c_double, C.c_double,
                               _P, _P, _P, C.c_int]
        L.or_md_run.argtypes = [C.c_int64, _P, _P, _P, C.POINTER(Trap), C.c_double, C.c_double, C.c_int64,
                                C.c_double, C.c_int, _P, C.c_int64, _P, C.c_int]
        L.or_hvp.argtypes = [C.c_int64, _P, _P, _P, _P, C.c_int32, _P, _P, _P, C.POINTER(Trap), C.c_double,
                             C.c_double, C.c_int]
        L.or_msd_grad.argtypes = [C.c_int64, _P, _P, _P, C.POINTER(Trap), C.c_double, C.c_int64, C.c_double,
                                  _P, C.c_int]
        L.orp_forces_range.argtypes = [C.c_int64, _P, _P, _P, _P, C.c_double, C.c_int64, C.c_int64,
                                       _P, _P, _P, C.c_int]
        L.orp_forces_range.restype = C.c_int
        _lib = L
    return _lib


def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_P)


def _threads(nthreads):
    if nthreads:
        return int(nthreads)
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        return os.cpu_count() or 1


def coulomb_constant() -> float:
    return lib().or_coulomb_constant()


def forces(x, y, z, q, eps2=0.0, idx=None, kappa=False, nthreads=None):
    """Forces (N) on the ions in idx (all when None); optionally their kappa."""
    n = len(x)
    (x, px), (y, py), (z, pz), (q, pq) = _d(x), _d(y), _d(z), _d(q)
    if idx is None:
        ni, pidx = n, None
    else:
        idx = np.ascontiguousarray(idx, dtype=np.int64)
        if idx.size and (idx.min() < 0 or idx.max() >= n):
            raise IndexError("oracle.forces: idx out of range")
        ni, pidx = len(idx), idx.ctypes.data_as(_PI64)
    fx, fy, fz, kp = (np.empty(ni) for _ in range(4))
    lib().or_forces(n, px, py, pz, pq, float(eps2), ni, pidx, fx.ctypes.data_as(_P), fy.ctypes.data_as(_P),
                    fz.ctypes.data_as(_P), kp.ctypes.data_as(_P) if kappa else None, _threads(nthreads))
    return (fx, fy, fz, kp) if kappa else (fx, fy, fz)


def coulomb_energy(x, y, z, q, eps2=0.0, nthreads=None):
    """(U_C in J, per-ion potential sums phi_i = sum_j q_j / r_ij in C/m)."""
    n = len(x)
    (x, px), (y, py), (z, pz), (q, pq) = _d(x), _d(y), _d(z), _d(q)
    phi = np.empty(n)
    u = lib().or_coulomb_energy(n, px, py, pz, pq, float(eps2), phi.ctypes.data_as(_P), _threads(nthreads))
    return u, phi


def trap_k(trap: dict, t: float) -> np.ndarray:
    k = np.empty(3)
    tr = make_trap(trap)
    lib().or_trap_k(C.byref(tr), float(t), k.ctypes.data_as(_P))
    return k


def trap_energy(x, y, z, m, trap, t):
    (x, px), (y, py), (z, pz), (m, pm) = _d(x), _d(y), _d(z), _d(m)
    tr = make_trap(trap)
    return lib().or_trap_energy(len(x), px, py, pz, pm, C.byref(tr), float(t))


def kinetic_energy(vx, vy, vz, m):
    (vx, a), (vy, b), (vz, c), (m, d) = _d(vx), _d(vy), _d(vz), _d(m)
    return lib().or_kinetic_energy(len(vx), a, b, c, d)


def accel(x, y, z, q, m, trap, t, eps2=0.0, nthreads=None):
    n = len(x)
    (x, px), (y, py), (z, pz), (q, pq), (m, pm) = _d(x), _d(y), _d(z), _d(q), _d(m)
    out = np.empty((3, n))
    tr = make_trap(trap)
    lib().or_accel(n, px, py, pz, pq, pm, C.byref(tr), float(t), float(eps2), out[0].ctypes.data_as(_P),
                   out[1].ctypes.data_as(_P), out[2].ctypes.data_as(_P), _threads(nthreads))
    return out


def md_run(state, q, m, trap, t0, dt, nsteps, eps2=0.0, init_accel=True, every=0, keep_traj=False,
           nthreads=None):
    """Velocity-Verlet run.  state is a (9, n) array x y z vx vy vz ax ay az
    (ax.. ignored when init_accel).  Returns (new_state, energies or None,
    traj or None); energies has shape (nsteps//every + 1, 4) = K, U_C, U_trap, E;
    traj has shape (nsteps, 9, n)."""
    st = np.array(state, dtype=np.float64, order="C", copy=True).reshape(9, -1)
    n = st.shape[1]
    q, pq = _d(q)
    m, pm = _d(m)
    en = np.empty((nsteps // every + 1, 4)) if every else None
    tj = np.empty((nsteps, 9, n)) if keep_traj else None
    tr = make_trap(trap)
    lib().or_md_run(n, st.ctypes.data_as(_P), pq, pm, C.byref(tr), float(t0), float(dt), int(nsteps),
                    float(eps2), int(bool(init_accel)), en.ctypes.data_as(_P) if en is not None else None,
                    int(every), tj.ctypes.data_as(_P) if tj is not None else None, _threads(nthreads))
    return st, en, tj


def hvp(x, y, z, q, v, m=None, trap=None, t=0.0, eps2=0.0, nthreads=None):
    """Hessian-vector products; v has shape (nvec, 3, n) (or (3, n))."""
    n = len(x)
    v = np.ascontiguousarray(v, dtype=np.float64)
    single = v.ndim == 2
    v = v.reshape(-1, 3, n)
    (x, px), (y, py), (z, pz), (q, pq) = _d(x), _d(y), _d(z), _d(q)
    hv = np.empty_like(v)
    if m is not None:
        m, pm = _d(m)
    else:
        pm = None
    tr = make_trap(trap)
    lib().or_hvp(n, px, py, pz, pq, v.shape[0], v.ctypes.data_as(_P), hv.ctypes.data_as(_P), pm, C.byref(tr),
                 float(t), float(eps2), _threads(nthreads))
    return hv[0] if single else hv


def msd_grad(state0, q, m, trap, dt, nsteps, eps2=0.0, nthreads=None):
    """(L, dL/d(wx, wy, wz)) for the mean-square displacement after nsteps."""
    st = np.ascontiguousarray(np.asarray(state0, dtype=np.float64).reshape(-1)[: 6 * len(q)])
    q, pq = _d(q)
    m, pm = _d(m)
    out = np.empty(4)
    tr = make_trap(trap)
    lib().or_msd_grad(len(q), st.ctypes.data_as(_P), pq, pm, C.byref(tr), float(dt), int(nsteps), float(eps2),
                      out.ctypes.data_as(_P), _threads(nthreads))
    return out[0], out[1:].copy()


def forces_plain_range(x, y, z, q, i0, i1, eps2=0.0, nthreads=None):
    """Timed variant (plain double loop): forces on ions i0..i1-1; returns
    (fx, fy, fz, threads_used)."""
    n = len(x)
    (x, px), (y, py), (z, pz), (q, pq) = _d(x), _d(y), _d(z), _d(q)
    if not 0 <= i0 <= i1 <= n:
        raise IndexError("oracle.forces_plain_range: bad range")
    f = np.empty((3, i1 - i0))
    used = lib().orp_forces_range(n, px, py, pz, pq, float(eps2), int(i0), int(i1), f[0].ctypes.data_as(_P),
                                  f[1].ctypes.data_as(_P), f[2].ctypes.data_as(_P), _threads(nthreads))
    return f[0], f[1], f[2], used


def two_ion_error_model(eps: float, T: float, dt: float, Q: float, m: float):
    """Section 4's estimate of the one-step errors caused by a relative error
    eps in 1/|x2 - x1|, at the closest approach d_min = 4 Q^2 k_C / (k_B T) of
    two ions with thermal speed v = sqrt(k_B T / m).  Returns (dx/d, dv/v):
      dx = 3/2 dt^2 (Q^2 k_C / m) d^-2 eps,   taken relative to d;
      dv = 3 dt (Q^2 k_C / m) d^-2 eps,       taken relative to v.
    The first is the position error of section 4 divided by d_min (the
    printed closed form for dx/d is dimensionally inconsistent, so the
    ratio is formed directly)."""
    kc = coulomb_constant()
    alpha = Q * Q * kc / m
    dmin = 4.0 * Q * Q * kc / (K_B * T)
    dx = 1.5 * dt * dt * alpha * dmin ** -2 * eps
    dv = 3.0 * dt * alpha * dmin ** -2 * eps
    v = np.sqrt(K_B * T / m)
    return dx / dmin, dv / v
