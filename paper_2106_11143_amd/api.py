"""Thin Python binding of libcoulomb_mi355x.so over torch device tensors.

Argument marshalling only: every step of the computation runs in the HIP
library (see include/coulomb.h for the contract of each call).  Tensors are
float64, contiguous, on one ROCm device; work is enqueued on
``torch.cuda.current_stream()``.  Scratch memory is a per-(device, stream)
torch buffer sized with ``cb_workspace_size``.

Loading fails loudly when the library has not been built (there is no CPU
fallback): build it with ``python -m paper_2106_11143_amd.build``.
"""
from __future__ import annotations

import ctypes as C
import os
import threading

import torch  # imported first so the library binds to torch's HIP runtime

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcoulomb_mi355x.so")

CB_OK, CB_EINVAL, CB_EHIP, CB_ENOWS, CB_ENONFINITE, CB_EUNSUPPORTED = range(6)
STATUS_NAMES = {0: "CB_OK", 1: "CB_EINVAL", 2: "CB_EHIP", 3: "CB_ENOWS", 4: "CB_ENONFINITE", 5: "CB_EUNSUPPORTED"}
PRECISIONS = {"fp64": 0, "mixed": 1, "ieee": 2, "fp32": 3, "mixed_f32d": 4}
OPS = {"forces": 0, "energy": 1, "md_step": 2, "md_run": 3, "hvp": 4, "adjoint": 5, "md_ensemble": 6, "grad": 7}
CB_INIT_ACCEL = 1
CB_ADJ_FINAL = 1

EXPORTS = ("cb_workspace_size", "coulomb_forces", "coulomb_forces_range", "coulomb_pair_stage", "coulomb_energy",
           "coulomb_trap_grad", "cb_trap_k", "coulomb_forces_noalloc", "md_step", "md_run", "coulomb_hvp", "md_adjoint_step", "cb_poll_flags",
           "cb_last_error", "cb_autotune", "cb_load_tuning", "cb_get_config", "cb_set_config")


class CoulombError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class Trap(C.Structure):
    """ctypes mirror of cb_trap."""

    _fields_ = [
        ("kind", C.c_int32),
        ("wx", C.c_double), ("wy", C.c_double), ("wz", C.c_double),
        ("rf_a", C.c_double), ("rf_q", C.c_double), ("rf_omega", C.c_double), ("rf_phase", C.c_double),
        ("gamma", C.c_double),
        ("wx1", C.c_double), ("wy1", C.c_double), ("t_ramp0", C.c_double), ("t_ramp1", C.c_double),
    ]


class State(C.Structure):
    """ctypes mirror of cb_state (nine device pointers)."""

    _fields_ = [(k, C.c_void_p) for k in ("x", "y", "z", "vx", "vy", "vz", "ax", "ay", "az")]


STATE_KEYS = ("x", "y", "z", "vx", "vy", "vz", "ax", "ay", "az")

_lib = None
_lock = threading.Lock()
_P = C.c_void_p


def lib() -> C.CDLL:
    """The loaded native library (raises if it is missing)."""
    global _lib
    if _lib is None:
        with _lock:
            if _lib is None:
                if not os.path.exists(LIB_PATH):
                    raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_2106_11143_amd.build`")
                L = C.CDLL(LIB_PATH)
                i32, i64, u32, d, sz = C.c_int32, C.c_int64, C.c_uint32, C.c_double, C.c_size_t
                L.cb_workspace_size.argtypes = [i32, i64, i32, i32, i32]
                L.cb_workspace_size.restype = sz
                L.coulomb_forces.argtypes = [i64, _P, _P, _P, _P, d, i32, _P, _P, _P, _P, sz, _P]
                L.coulomb_forces_noalloc.argtypes = [i64, _P, _P, _P, _P, d, i32, _P, _P, _P, _P]
                L.coulomb_forces_range.argtypes = [i64, i64, i64, _P, _P, _P, _P, d, i32, _P, _P, _P, _P, sz, _P]
                L.coulomb_energy.argtypes = [i64, _P, _P, _P, _P, d, i32, _P, _P, sz, _P]
                L.coulomb_trap_grad.argtypes = [i64, _P, _P, _P, _P, _P, C.POINTER(Trap), d, d, i32, _P, _P, _P, _P,
                                                _P, sz, _P]
                L.cb_trap_k.argtypes = [C.POINTER(Trap), d, C.POINTER(C.c_double)]
                L.coulomb_pair_stage.argtypes = [i64, _P, _P, _P, _P, d, i32, C.POINTER(C.c_int32), _P, sz, _P]
                L.md_step.argtypes = [i64, C.POINTER(State), _P, _P, C.POINTER(Trap), d, d, d, i32, _P, sz, _P]
                L.md_run.argtypes = [i32, C.POINTER(C.c_int64), C.POINTER(State), _P, _P, C.POINTER(Trap), d, d,
                                     i64, d, i32, u32, _P, i64, _P, sz, _P]
                L.coulomb_hvp.argtypes = [i64, _P, _P, _P, _P, i32, _P, _P, _P, C.POINTER(Trap), d, d, i32, _P, sz,
                                          _P]
                L.md_adjoint_step.argtypes = [i64, _P, _P, _P, _P, _P, C.POINTER(Trap), d, d, i32, u32, _P, _P, _P,
                                              sz, _P]
                L.cb_poll_flags.argtypes = [_P, C.POINTER(C.c_uint32)]
                L.cb_last_error.restype = C.c_char_p
                L.cb_autotune.argtypes = [i32, i64, i32, C.c_char_p]
                L.cb_load_tuning.argtypes = [C.c_char_p]
                L.cb_get_config.argtypes = [i32, i64, i32, C.POINTER(C.c_int32)]
                L.cb_set_config.argtypes = [i32, i64, i32, i32, i32, i32, i32]
                for name in EXPORTS:
                    if name not in ("cb_workspace_size", "cb_last_error"):
                        getattr(L, name).restype = C.c_int
                _lib = L
    return _lib


def last_error() -> str:
    return lib().cb_last_error().decode()


def _check(status: int, name: str) -> None:
    if status != CB_OK:
        raise CoulombError(status, f"{name}: {last_error()}")


def _prec(p) -> int:
    if isinstance(p, str):
        return PRECISIONS[p]
    return int(p)


def _op(o) -> int:
    return OPS[o] if isinstance(o, str) else int(o)


def make_trap(d: dict | None) -> Trap:
    t = Trap()
    for name, _ in Trap._fields_:
        setattr(t, name, (d or {}).get(name, 0))
    return t


def _dev_f64(*ts):
    dev = None
    for t in ts:
        if t is None:
            continue
        if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_cuda:
            raise TypeError("expected float64 ROCm tensors")
        if not t.is_contiguous():
            raise ValueError("expected contiguous tensors")
        if dev is None:
            dev = t.device
        elif t.device != dev:
            raise ValueError("tensors are on different devices")
    return dev


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


_ws_cache: dict = {}


def workspace_size(op, n: int, nrun: int = 1, nvec: int = 1, prec="fp64") -> int:
    return int(lib().cb_workspace_size(_op(op), int(n), int(nrun), int(nvec), _prec(prec)))


def _workspace(op, n, nrun=1, nvec=1, prec="fp64", device=None):
    need = workspace_size(op, n, nrun, nvec, prec)
    if need == 0:
        raise CoulombError(CB_EINVAL, "cb_workspace_size rejected the request")
    key = (device, torch.cuda.current_stream(device).cuda_stream)
    buf = _ws_cache.get(key)
    if buf is None or buf.numel() < need:
        buf = torch.empty(need, dtype=torch.uint8, device=device)
        _ws_cache[key] = buf
    return buf


def reset_config(op, n: int, prec="fp64") -> None:
    set_config(op, n, prec, 0, 0, 0, 0)


def clear_workspace_cache() -> None:
    _ws_cache.clear()


# ------------------------------------------------------------------- calls
def coulomb_forces(x, y, z, q, eps2: float = 0.0, prec="fp64", out=None):
    """Forces (N) on every ion; returns (fx, fy, fz)."""
    dev = _dev_f64(x, y, z, q)
    n = x.numel()
    fx, fy, fz = out if out is not None else (torch.empty_like(x), torch.empty_like(x), torch.empty_like(x))
    ws = _workspace("forces", n, prec=prec, device=dev)
    _check(lib().coulomb_forces(n, x.data_ptr(), y.data_ptr(), z.data_ptr(), q.data_ptr(), float(eps2), _prec(prec),
                                fx.data_ptr(), fy.data_ptr(), fz.data_ptr(), ws.data_ptr(), ws.numel(), _stream()),
           "coulomb_forces")
    return fx, fy, fz


def coulomb_forces_noalloc(x, y, z, q, eps2: float = 0.0, prec="fp64", out=None):
    """Forces (N) on every ion without a workspace (the library's static
    per-GPU scratch); returns (fx, fy, fz).  Pass `out` to allocate nothing."""
    _dev_f64(x, y, z, q)
    n = x.numel()
    fx, fy, fz = out if out is not None else (torch.empty_like(x), torch.empty_like(x), torch.empty_like(x))
    _dev_f64(fx, fy, fz)
    _check(lib().coulomb_forces_noalloc(n, x.data_ptr(), y.data_ptr(), z.data_ptr(), q.data_ptr(), float(eps2),
                                        _prec(prec), fx.data_ptr(), fy.data_ptr(), fz.data_ptr(), _stream()),
           "coulomb_forces_noalloc")
    return fx, fy, fz


def coulomb_forces_range(x, y, z, q, i0: int, i1: int, eps2: float = 0.0, prec="fp64", out=None):
    """Forces (N) on the ions i0 .. i1-1 from all ions; returns (fx, fy, fz)
    of length i1 - i0."""
    dev = _dev_f64(x, y, z, q)
    n = x.numel()
    ni = int(i1) - int(i0)
    if out is not None:
        fx, fy, fz = out
    else:
        fx, fy, fz = (torch.empty(max(ni, 0), dtype=torch.float64, device=dev) for _ in range(3))
    ws = _workspace("forces", n, prec=prec, device=dev)
    _check(lib().coulomb_forces_range(n, int(i0), int(i1), x.data_ptr(), y.data_ptr(), z.data_ptr(), q.data_ptr(),
                                      float(eps2), _prec(prec), fx.data_ptr(), fy.data_ptr(), fz.data_ptr(),
                                      ws.data_ptr(), ws.numel(), _stream()),
           "coulomb_forces_range")
    return fx, fy, fz


def coulomb_pair_stage(x, y, z, q, eps2: float = 0.0, prec="fp64"):
    """Runs only the all-pairs kernel (partials into the cached workspace);
    returns (workspace tensor, number of j-splits)."""
    dev = _dev_f64(x, y, z, q)
    n = x.numel()
    ws = _workspace("forces", n, prec=prec, device=dev)
    S = C.c_int32(0)
    _check(lib().coulomb_pair_stage(n, x.data_ptr(), y.data_ptr(), z.data_ptr(), q.data_ptr(), float(eps2),
                                    _prec(prec), C.byref(S), ws.data_ptr(), ws.numel(), _stream()),
           "coulomb_pair_stage")
    return ws, int(S.value)


def coulomb_energy(x, y, z, q, eps2: float = 0.0, prec="fp64", out=None):
    """Coulomb energy U_C (J) as a one-element device tensor."""
    dev = _dev_f64(x, y, z, q)
    n = x.numel()
    u = out if out is not None else torch.empty(1, dtype=torch.float64, device=dev)
    ws = _workspace("energy", n, prec=prec, device=dev)
    _check(lib().coulomb_energy(n, x.data_ptr(), y.data_ptr(), z.data_ptr(), q.data_ptr(), float(eps2), _prec(prec),
                                u.data_ptr(), ws.data_ptr(), ws.numel(), _stream()), "coulomb_energy")
    return u


def trap_k(trap: dict | None, t: float = 0.0):
    """The trap's spring constants per unit mass (kx, ky, kz) at time t, from
    the library (cb_trap_k); (0, 0, 0) for no trap."""
    if trap is None:
        return (0.0, 0.0, 0.0)
    tr = make_trap(trap)
    k = (C.c_double * 3)()
    _check(lib().cb_trap_k(C.byref(tr), float(t), k), "cb_trap_k")
    return (k[0], k[1], k[2])


def coulomb_trap_grad(x, y, z, q, m=None, trap: dict | None = None, t: float = 0.0, eps2: float = 0.0,
                      prec="fp64", grad: bool = True, energy: bool = False, out=None):
    """Gradient g = dU/dr = -F + m k(t) r (a (3, n) tensor) and/or the energy
    U = U_C + U_trap(t) (a one-element tensor) of the Coulomb + trap
    potential; m = None gives the Coulomb part alone.  Returns (g or None,
    U or None).  out: an optional contiguous (3, n) float64 tensor for g."""
    dev = _dev_f64(x, y, z, q, m)
    n = x.numel()
    g = None
    if grad:
        g = out if out is not None else torch.empty((3, n), dtype=torch.float64, device=dev)
        _dev_f64(g)
        if tuple(g.shape) != (3, n):
            raise ValueError("out must have shape (3, n)")
    u = torch.empty(1, dtype=torch.float64, device=dev) if energy else None
    tr = make_trap(trap)
    ws = _workspace("grad", n, prec=prec, device=dev)
    gp = [g[c].data_ptr() for c in range(3)] if g is not None else [None, None, None]
    _check(lib().coulomb_trap_grad(n, x.data_ptr(), y.data_ptr(), z.data_ptr(), q.data_ptr(),
                                   m.data_ptr() if m is not None else None, C.byref(tr), float(t), float(eps2),
                                   _prec(prec), *gp, u.data_ptr() if u is not None else None, ws.data_ptr(),
                                   ws.numel(), _stream()), "coulomb_trap_grad")
    return g, u


def _state(st) -> State:
    if isinstance(st, dict):
        ts = [st[k] for k in STATE_KEYS]
    else:
        ts = list(st)
        if len(ts) == 1:
            ts = list(ts[0])
    if len(ts) != 9:
        raise ValueError("state needs nine arrays x y z vx vy vz ax ay az")
    _dev_f64(*ts)
    s = State()
    for k, t in zip(STATE_KEYS, ts):
        setattr(s, k, t.data_ptr())
    return s


def md_step(state, q, m, trap: dict, t: float, dt: float, eps2: float = 0.0, prec="fp64"):
    """One velocity-Verlet step, in place on `state` (dict or 9 tensors, or a
    (9, n) tensor)."""
    s = _state(state)
    dev = _dev_f64(q, m)
    n = q.numel()
    tr = make_trap(trap)
    ws = _workspace("md_step", n, prec=prec, device=dev)
    _check(lib().md_step(n, C.byref(s), q.data_ptr(), m.data_ptr(), C.byref(tr), float(t), float(dt), float(eps2),
                         _prec(prec), ws.data_ptr(), ws.numel(), _stream()), "md_step")


def md_run(state, q, m, traps, t0: float, dt: float, nsteps: int, offsets=None, eps2: float = 0.0, prec="fp64",
           init_accel: bool = True, every: int = 0, out=None):
    """nsteps velocity-Verlet steps in place.  traps: one dict, or one per run
    with offsets (sequence of nrun+1 ints).  Returns the energies tensor
    [nrun][nsteps//every + 1][4] (K, U_C, U_trap, E) when every > 0 (written
    into `out` when given: contiguous float64 on the device, that shape)."""
    s = _state(state)
    dev = _dev_f64(q, m)
    n = q.numel()
    if offsets is None:
        offsets = [0, n]
    offs = (C.c_int64 * len(offsets))(*[int(o) for o in offsets])
    nrun = len(offsets) - 1
    if isinstance(traps, dict):
        traps = [traps] * nrun
    if len(traps) != nrun:
        raise ValueError("need one trap per run")
    tarr = (Trap * nrun)(*[make_trap(t) for t in traps])
    en = None
    if every:
        shape = (nrun, nsteps // every + 1, 4)
        if out is not None:
            if tuple(out.shape) != shape or out.dtype != torch.float64 or not out.is_contiguous():
                raise ValueError(f"out must be a contiguous float64 tensor of shape {shape}")
            _dev_f64(q, m, out)
            en = out
        else:
            en = torch.empty(shape, dtype=torch.float64, device=dev)
    ws = _workspace("md_run", n, nrun=nrun, prec=prec, device=dev)
    _check(lib().md_run(nrun, offs, C.byref(s), q.data_ptr(), m.data_ptr(), tarr, float(t0), float(dt), int(nsteps),
                        float(eps2), _prec(prec), CB_INIT_ACCEL if init_accel else 0,
                        en.data_ptr() if en is not None else None, int(every), ws.data_ptr(), ws.numel(), _stream()),
           "md_run")
    return en


def coulomb_hvp(x, y, z, q, v, m=None, trap: dict | None = None, t: float = 0.0, eps2: float = 0.0, prec="fp64",
                out=None):
    """Hessian-vector products; v is (nvec, 3, n) or (3, n)."""
    dev = _dev_f64(x, y, z, q, v, m)
    n = x.numel()
    single = v.dim() == 2
    vv = v.reshape(-1, 3, n)
    nvec = vv.shape[0]
    hv = out if out is not None else torch.empty_like(vv)
    tr = make_trap(trap)
    ws = _workspace("hvp", n, nvec=nvec, prec=prec, device=dev)
    _check(lib().coulomb_hvp(n, x.data_ptr(), y.data_ptr(), z.data_ptr(), q.data_ptr(), nvec, vv.data_ptr(),
                             hv.data_ptr(), m.data_ptr() if m is not None else None, C.byref(tr), float(t),
                             float(eps2), _prec(prec), ws.data_ptr(), ws.numel(), _stream()), "coulomb_hvp")
    return hv.reshape(3, n) if single else hv


def md_adjoint_step(x, y, z, q, m, trap: dict, dt: float, lam, dldw, eps2: float = 0.0, prec="fp64",
                    final: bool = False):
    """One reverse step of the discrete adjoint (in place on lam [9][n] and
    dldw [3])."""
    dev = _dev_f64(x, y, z, q, m, lam, dldw)
    n = x.numel()
    tr = make_trap(trap)
    ws = _workspace("adjoint", n, prec=prec, device=dev)
    _check(lib().md_adjoint_step(n, x.data_ptr(), y.data_ptr(), z.data_ptr(), q.data_ptr(), m.data_ptr(),
                                 C.byref(tr), float(dt), float(eps2), _prec(prec), CB_ADJ_FINAL if final else 0,
                                 lam.data_ptr(), dldw.data_ptr(), ws.data_ptr(), ws.numel(), _stream()),
           "md_adjoint_step")


def poll_flags() -> int:
    """Synchronises the current stream and returns (and clears) the device
    flag word; bit 0 = a non-finite value was produced."""
    f = C.c_uint32(0)
    st = lib().cb_poll_flags(_stream(), C.byref(f))
    if st not in (CB_OK, CB_ENONFINITE):
        _check(st, "cb_poll_flags")
    return int(f.value)


def autotune(op, n: int, prec="fp64", cache_path: str | None = None) -> None:
    _check(lib().cb_autotune(_op(op), int(n), _prec(prec), cache_path.encode() if cache_path else None),
           "cb_autotune")


def load_tuning(cache_path: str) -> None:
    _check(lib().cb_load_tuning(cache_path.encode()), "cb_load_tuning")


def get_config(op, n: int, prec="fp64") -> dict:
    out = (C.c_int32 * 5)()
    _check(lib().cb_get_config(_op(op), int(n), _prec(prec), out), "cb_get_config")
    return dict(algo=out[0], p=out[1], wg=out[2], splits=out[3], tuned=bool(out[4]))


def set_config(op, n: int, prec="fp64", p: int = 1, wg: int = 256, splits: int = 1, algo: int = 0) -> None:
    """Force a launch configuration (algo = p = wg = splits = 0: back to the
    default).  algo 1 = the Newton's-third-law force kernel (n <= 2^18), with
    p in {2, 3, 4, 5, 6, 8}, wg = j's per reduction group = 4 and splits =
    segment length in {256, 512, 1024, 2048}; algo 2 = the same kernel with
    the per-j reactions summed through LDS; algo 4 = the same tiles run four
    i-blocks to a 256-thread workgroup that share one j-segment and sum their
    reactions in LDS before one write (p in {4, 6, 8}); algo 3 (md_step /
    md_run, n <= 8192) = one launch per step, p = 1, wg = 64, splits = j-parts
    in 1..32.
    op "md_ensemble" (n = total
    ions) picks the path of md_run with several runs: algo 0 with p = 4,
    wg = 512, splits = 1 is the persistent kernel; algo 2 with p in {4, 8},
    wg = 4, splits in {256, 512} is the stepped path."""
    _check(lib().cb_set_config(_op(op), int(n), _prec(prec), int(algo), int(p), int(wg), int(splits)),
           "cb_set_config")
