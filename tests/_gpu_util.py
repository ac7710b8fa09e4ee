"""Helpers shared by the GPU tests (no oracle arithmetic here)."""
import numpy as np
import torch

PREC_TOL = {"fp64": 1e-12, "ieee": 1e-12, "mixed": 1e-7}


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")


def host(t):
    return t.detach().cpu().numpy()


def per_ion_rel(F, ref):
    """Per-ion relative error |F_i - ref_i| / |ref_i| (vector 2-norms)."""
    return np.linalg.norm(F - ref, axis=0) / np.linalg.norm(ref, axis=0)


def report(name, err, kappa=None):
    worst = int(np.argmax(err))
    k = f" kappa_worst={kappa[worst]:.3g}" if kappa is not None else ""
    print(f"[{name}] max_rel={err.max():.3e} rms_rel={np.sqrt(np.mean(err ** 2)):.3e} worst_ion={worst}{k}",
          flush=True)


def state_tensors(st9):
    """Nine device tensors from a (9, n) numpy state."""
    return [dev(st9[k]) for k in range(9)]


def state_host(ts):
    return np.stack([host(t) for t in ts])
