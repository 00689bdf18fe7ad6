"""torch.autograd.Function wrappers of the forward and adjoint kernels.

For the holomorphic maps g = H x^{m-1} and f = H x^m, complex autograd hands
the backward the cotangents of g and f and expects J^H applied to them; the
adjoint entry points of the library compute exactly that (spectral
correlations on the forward product's padded grid).  Where the shape has the
spectral layout (complex, d_H > 4096), the forward keeps x^ = fft(pad x)
(written by the forward's row pass as it transforms x) and the backward
reuses it instead of transforming x again.
"""
from __future__ import annotations

import torch

from .binding import (hankel_tvp, hankel_tvp_backward, hankel_tvp_backward_spectral,
                      hankel_tvp_backward_spectral_strided_batched, hankel_tvp_backward_strided_batched,
                      hankel_tvp_save_spectrum, hankel_tvp_strided_batched)


def _spectral(h: torch.Tensor, x: torch.Tensor, m: int) -> bool:
    """The forward can keep x^ for the backward: complex data and the
    three-pass spectral layout (d_H above 4096)."""
    return h.is_complex() and x.is_complex() and m * (x.shape[-1] - 1) + 1 > 4096


class HankelTVPFunction(torch.autograd.Function):
    """(h, x) -> (g, f) = (H x^{m-1}, H x^m) for a square Hankel tensor of order m.

    h and x are 1D (one product) or 2D (a batch: h (B, d_H), x (B, n))."""

    @staticmethod
    def forward(ctx, h, x, m: int):
        ctx.m = m
        ctx.n = x.shape[-1]
        ctx.spectral = any(ctx.needs_input_grad[:2]) and _spectral(h, x, m)
        if ctx.spectral:
            g, f, x_spec = hankel_tvp_save_spectrum(h, x, m, True, True)
            ctx.save_for_backward(h, x_spec)
        else:
            if x.dim() == 1:
                g, f = hankel_tvp(h, x, m, True, True)
            else:
                g, f = hankel_tvp_strided_batched(h, x, m, True, True)
            ctx.save_for_backward(h, x)
        return g, f

    @staticmethod
    def backward(ctx, grad_g, grad_f):
        h, xs = ctx.saved_tensors
        if not (h.is_complex() and xs.is_complex()):
            raise TypeError("the adjoint kernels are implemented for complex dtypes")
        want_h, want_x = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        if not (want_h or want_x):
            return None, None, None
        if ctx.spectral:
            if h.dim() == 1:
                gx, gh = hankel_tvp_backward_spectral(h, xs, ctx.m, ctx.n, grad_g, grad_f, want_x, want_h)
            else:
                gx, gh = hankel_tvp_backward_spectral_strided_batched(h, xs, ctx.m, ctx.n, grad_g, grad_f, want_x,
                                                                      want_h)
        elif xs.dim() == 1:
            gx, gh = hankel_tvp_backward(h, xs, ctx.m, grad_g, grad_f, want_x, want_h)
        else:
            gx, gh = hankel_tvp_backward_strided_batched(h, xs, ctx.m, grad_g, grad_f, want_x, want_h)
        return gh, gx, None


def hankel_tvp_autograd(h: torch.Tensor, x: torch.Tensor, m: int):
    """Differentiable (H x^{m-1}, H x^m)."""
    return HankelTVPFunction.apply(h, x, m)
