"""torch.autograd Functions over the HIP kernels.

``energy(r, q, m, trap)`` is differentiable twice: its gradient is computed
by the force kernel and the gradient's backward by the Hessian-vector-product
kernel, so ``torch.autograd.grad`` of a gradient gives H v.

Positions are one (3, n) float64 tensor (rows x, y, z).  The trap energy is
sum_i m_i (kx x^2 + ky y^2 + kz z^2) / 2 with k from the trap at time t (see
include/coulomb.h); with m = None only the Coulomb part is used.
"""
from __future__ import annotations

import math

import torch

from . import api


def trap_k(trap: dict | None, t: float = 0.0):
    """Trap spring constants per unit mass (kx, ky, kz) at time t."""
    if trap is None:
        return (0.0, 0.0, 0.0)
    if int(trap.get("kind", 0)) == 1:
        w2 = trap["rf_omega"] ** 2
        kx = trap.get("rf_a", 0.0) * w2 / 4.0 + trap["rf_q"] * w2 / 2.0 * math.cos(
            trap["rf_omega"] * t + trap.get("rf_phase", 0.0))
        return (kx, -kx, trap["wz"] ** 2)
    wx, wy = trap["wx"], trap["wy"]
    t0, t1 = trap.get("t_ramp0", 0.0), trap.get("t_ramp1", 0.0)
    if t1 > t0:
        s = min(max((t - t0) / (t1 - t0), 0.0), 1.0)
        wx = wx + s * (trap["wx1"] - wx)
        wy = wy + s * (trap["wy1"] - wy)
    return (wx * wx, wy * wy, trap["wz"] ** 2)


def _k_tensor(trap, t, like):
    return torch.tensor(trap_k(trap, t), dtype=like.dtype, device=like.device).reshape(3, 1)


class CoulombTrapGrad(torch.autograd.Function):
    """G(r) = dU/dr = -F_C(r) + m k r; backward: H(r) w."""

    @staticmethod
    def forward(ctx, r, q, m, trap, t, eps2, prec):
        fx, fy, fz = api.coulomb_forces(r[0].contiguous(), r[1].contiguous(), r[2].contiguous(), q, eps2, prec)
        G = -torch.stack([fx, fy, fz])
        if m is not None:
            G = G + m.reshape(1, -1) * _k_tensor(trap, t, r) * r
        ctx.save_for_backward(r, q, m if m is not None else torch.empty(0))
        ctx.trap, ctx.t, ctx.eps2, ctx.prec, ctx.has_m = trap, t, eps2, prec, m is not None
        return G

    @staticmethod
    def backward(ctx, gG):
        r, q, m = ctx.saved_tensors
        hv = api.coulomb_hvp(r[0].contiguous(), r[1].contiguous(), r[2].contiguous(), q, gG.contiguous(),
                             m if ctx.has_m else None, ctx.trap, ctx.t, ctx.eps2, ctx.prec)
        return hv, None, None, None, None, None, None


class CoulombTrapEnergy(torch.autograd.Function):
    """U(r) = U_C(r) + U_trap(r); backward through CoulombTrapGrad (so that
    a second derivative uses the HVP kernel)."""

    @staticmethod
    def forward(ctx, r, q, m, trap, t, eps2, prec):
        u = api.coulomb_energy(r[0].contiguous(), r[1].contiguous(), r[2].contiguous(), q, eps2, prec)[0]
        if m is not None:
            u = u + 0.5 * (m.reshape(1, -1) * _k_tensor(trap, t, r) * r * r).sum()
        ctx.save_for_backward(r, q, m if m is not None else torch.empty(0))
        ctx.args = (trap, t, eps2, prec, m is not None)
        return u

    @staticmethod
    def backward(ctx, gU):
        r, q, m = ctx.saved_tensors
        trap, t, eps2, prec, has_m = ctx.args
        G = CoulombTrapGrad.apply(r, q, m if has_m else None, trap, t, eps2, prec)
        return gU * G, None, None, None, None, None, None


def energy(r, q, m=None, trap=None, t=0.0, eps2=0.0, prec="fp64"):
    return CoulombTrapEnergy.apply(r, q, m, trap, t, eps2, prec)


def gradient(r, q, m=None, trap=None, t=0.0, eps2=0.0, prec="fp64"):
    return CoulombTrapGrad.apply(r, q, m, trap, t, eps2, prec)
