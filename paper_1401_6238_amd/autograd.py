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

from .binding import (block_hankel_tvp, block_hankel_tvp_backward, hankel_mode_products,
                      hankel_mode_products_backward, hankel_tvp, hankel_tvp_backward, hankel_tvp_backward_spectral,
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


class HankelModeProductsFunction(torch.autograd.Function):
    """(h, x_1, ..., x_m) -> (y, alpha) = (H x_2 ... x_m, H x_1 ... x_m) for the
    general Hankel tensor of size dims (distinct vectors); the backward is the
    library's distinct-vector adjoint."""

    @staticmethod
    def forward(ctx, h, dims, *xs):
        ctx.dims = list(dims)
        y, a = hankel_mode_products(h, list(xs), ctx.dims, True, True)
        ctx.save_for_backward(h, *xs)
        return y, a

    @staticmethod
    def backward(ctx, grad_y, grad_alpha):
        h, *xs = ctx.saved_tensors
        want = list(ctx.needs_input_grad[2:])
        want_h = ctx.needs_input_grad[0]
        if not (want_h or any(want)):
            return (None, None) + (None,) * len(xs)
        gv, gh = hankel_mode_products_backward(h, xs, ctx.dims, grad_y, grad_alpha, want, want_h)
        return (gh, None) + tuple(gv)


class BlockHankelTVPFunction(torch.autograd.Function):
    """(H, vec(X_1), ..., vec(X_m)) -> (vec(Y), alpha) for the BHHB tensor with
    blocks of size inner_dims and block counts block_dims (distinct vectors)."""

    @staticmethod
    def forward(ctx, H, inner_dims, block_dims, *xs):
        ctx.inner, ctx.blocks = list(inner_dims), list(block_dims)
        y, a = block_hankel_tvp(H, list(xs), ctx.inner, ctx.blocks, True, True)
        ctx.save_for_backward(H, *xs)
        return y, a

    @staticmethod
    def backward(ctx, grad_y, grad_alpha):
        H, *xs = ctx.saved_tensors
        want = list(ctx.needs_input_grad[3:])
        want_h = ctx.needs_input_grad[0]
        if not (want_h or any(want)):
            return (None, None, None) + (None,) * len(xs)
        gv, gh = block_hankel_tvp_backward(H, xs, ctx.inner, ctx.blocks, grad_y, grad_alpha, want, want_h)
        return (gh, None, None) + tuple(gv)


def hankel_mode_products_autograd(h: torch.Tensor, vectors, dims=None):
    """Differentiable (H x_2 ... x_m, H x_1 ... x_m) with distinct vectors."""
    dims = [v.numel() for v in vectors] if dims is None else list(dims)
    return HankelModeProductsFunction.apply(h, dims, *vectors)


def block_hankel_tvp_autograd(H: torch.Tensor, vectors, inner_dims, block_dims):
    """Differentiable BHHB products (vec(Y), alpha) with distinct vectors."""
    return BlockHankelTVPFunction.apply(H, list(inner_dims), list(block_dims), *vectors)
