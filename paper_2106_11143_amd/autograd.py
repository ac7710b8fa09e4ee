"""torch.autograd Functions over the HIP kernels.

``energy(r, q, m, trap)`` is differentiable twice: its gradient is computed
by the force kernel and the gradient's backward by the Hessian-vector-product
kernel, so ``torch.autograd.grad`` of a gradient gives H v.

Positions are one (3, n) float64 tensor (rows x, y, z).  The trap energy is
sum_i m_i (kx x^2 + ky y^2 + kz z^2) / 2 with k from the trap at time t (see
include/coulomb.h); with m = None only the Coulomb part is used.
"""
from __future__ import annotations

import torch

from . import api

# the trap's spring constants per unit mass (kx, ky, kz) at time t, from the library
trap_k = api.trap_k


class CoulombTrapGrad(torch.autograd.Function):
    """G(r) = dU/dr = -F_C(r) + m k r; backward: H(r) w."""

    @staticmethod
    def forward(ctx, r, q, m, trap, t, eps2, prec):
        G, _ = api.coulomb_trap_grad(r[0].contiguous(), r[1].contiguous(), r[2].contiguous(), q, m, trap, t, eps2,
                                     prec)
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
        _, u = api.coulomb_trap_grad(r[0].contiguous(), r[1].contiguous(), r[2].contiguous(), q, m, trap, t, eps2,
                                     prec, grad=False, energy=True)
        u = u[0]
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
