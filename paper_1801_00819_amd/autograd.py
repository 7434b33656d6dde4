"""Differentiable Born modelling: ``torch.autograd.Function`` over the
library's operator pair.

forward  d = A m   (eq. 1 of the paper without noise; Born modelling over the
                    context's current window of shots)
backward g_m = A^T g_d   (eq. 2: the library's exact discrete adjoint)

The context should be opened with background checkpoints (``ckpt_interval``
-1 gives ceil(sqrt(nt)) steps between checkpoints): the forward pass then
advances the background wavefield alongside the Born field, and the backward
pass recomputes the background segment by segment from its checkpoints
instead of keeping every time step. All computation runs in the HIP library;
this module only passes device pointers.

The same function differentiates the split-step Fourier pair: a
device-pointer ``paper_1801_00819_amd.ssf.SsfContext`` has the same
``apply_born`` / ``apply_adjoint`` (its data are the window's frequency-
domain (re, im) pairs).
"""
from __future__ import annotations

import torch


class BornFn(torch.autograd.Function):
    """``d = BornFn.apply(m, ctx)`` with ``m`` a float32 CUDA tensor of the
    model shape and ``ctx`` a device-pointer :class:`Context` (or
    split-step context)."""

    @staticmethod
    def forward(fctx, m: torch.Tensor, lib_ctx) -> torch.Tensor:
        if not lib_ctx.device:
            raise ValueError("BornFn needs a context opened with device=True")
        fctx.lib_ctx = lib_ctx
        fctx.generation = lib_ctx.generation
        return lib_ctx.apply_born(m.detach().contiguous())

    @staticmethod
    def backward(fctx, grad_d: torch.Tensor):
        # the adjoint must belong to the window the forward pass modelled
        if fctx.lib_ctx.generation != fctx.generation:
            raise RuntimeError(
                "BornFn.backward: the context's window changed (update or "
                "downdate) after the forward pass; the adjoint would belong "
                "to another operator")
        g = fctx.lib_ctx.apply_adjoint(grad_d.detach().contiguous())
        return g, None


def born(m: torch.Tensor, lib_ctx) -> torch.Tensor:
    return BornFn.apply(m, lib_ctx)


def misfit(m: torch.Tensor, d: torch.Tensor, lib_ctx) -> torch.Tensor:
    """0.5 ||A m - d||^2, accumulated in float64."""
    r = born(m, lib_ctx) - d
    return 0.5 * torch.sum(r.double() * r.double())
