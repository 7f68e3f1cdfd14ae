"""Reverse mode through the series Newton solve, as torch.autograd.Functions.

Tensors here are multiple-double planes (2, m, *S), float64, on the GPU.  A
gradient that flows between these Functions is itself md-valued: its planes
hold G = dL/dRe z + i dL/dIm z for every complex entry z, the value of G
being the sum of the limbs (not one partial derivative per limb).  Generic
torch operations on planes do not follow that convention, so a loss is
taken with the Functions of this module (``sum_abs2``).

``newton_solve(coef, sysd, x0, iters)`` runs ``iters`` Newton steps on
truncated series (Section 4) from x0 with the system's coefficients taken
from ``coef`` and returns the series x and the status flags.  Its backward treats x as the
converged root of the truncated system and calls ``md_newton_adjoint``: one
QR of A_0, the staggered stages in reverse, and the contraction with every
term's monomial series, stored by the evaluation pass (``store_monomials``)
or recomputed per term.  The coefficient gradient comes back in double
double: limbs 0 and 1 of the returned planes, zeros above.  Every step runs
in the HIP library; torch only allocates and orders the work.
"""
from __future__ import annotations

import torch

from . import binding as B


class NewtonSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, coef, sysd, x0, iters, store_monomials):
        sd = sysd.with_coef(coef.detach().contiguous())
        x = x0.detach().clone().contiguous()
        _, _, status = B.newton(sd, x, iters)
        ctx.sd = sd
        ctx.store = bool(store_monomials)
        ctx.status = status  # MD_ST_* flags of the forward, then of the backward
        ctx.save_for_backward(x)
        ctx.mark_non_differentiable(status)
        return x, status

    @staticmethod
    def backward(ctx, grad_x, _grad_status):
        (x,) = ctx.saved_tensors
        sd = ctx.sd
        g2, _ = B.md_newton_adjoint(sd, x, grad_x.contiguous(), ctx.store, status=ctx.status)
        m = sd.m
        grad = torch.zeros_like(sd.coef)
        k = min(2, m)
        grad[:, :k] = g2[:, :k]
        return grad, None, None, None, None


class SumAbs2(torch.autograd.Function):
    """L = sum of |z|^2 over the entries of md planes; forward returns the
    leading double of L (from md_norm2), backward the md-valued 2 g z: the
    real and imaginary planes each multiplied by the double 2 g in the
    library (md_elementwise's md x double product, renormalised), so the
    gradient keeps all m limbs for any upstream g."""

    @staticmethod
    def forward(ctx, z):
        ctx.save_for_backward(z)
        m = z.shape[1]
        nrm = B.md_norm2(z.reshape(2, m, -1).contiguous())
        return (nrm[0, 0] * nrm[0, 0]).reshape(())

    @staticmethod
    def backward(ctx, g):
        (z,) = ctx.saved_tensors
        m = z.shape[1]
        zf = z.reshape(2, m, -1).contiguous()
        count = zf.shape[2]
        # the scale as the leading limb of an md operand (2 g is exact)
        scale = torch.zeros((m, count), dtype=torch.float64, device=z.device)
        scale[0] = (2.0 * g.to(torch.float64)).reshape(())
        out = torch.empty_like(zf)
        for part in range(2):
            out[part] = B.md_elementwise("muld", zf[part].contiguous(), scale)
        return out.reshape(z.shape)


def newton_solve(coef: torch.Tensor, sysd: B.DeviceSystem, x0: torch.Tensor, iters: int,
                 store_monomials: bool = True) -> torch.Tensor:
    """(x, status): x after iters Newton steps from x0 with coefficients coef
    (planes (2, m, M, dc+1)), differentiable in coef; status the int32 MD_ST_*
    flags on the device (the backward ors its own into the same tensor)."""
    return NewtonSolve.apply(coef, sysd, x0, iters, store_monomials)


def sum_abs2(z: torch.Tensor) -> torch.Tensor:
    """sum |z|^2 of md planes (2, m, ...), differentiable."""
    return SumAbs2.apply(z)
