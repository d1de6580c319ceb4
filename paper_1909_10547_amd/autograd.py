"""torch.autograd wrappers: the network PDF on the x-grid (forward =
fk_mlp_forward, backward = the reverse pass fk_mlp_backward), the
convolution (forward = fk_conv_dis/had, backward = the hand-written adjoint
fk_conv_backward) and the FP64 chi2 (backward = its gradient
2 C^{-1}(sigma - D)): the chain a gradient-descent PDF fit differentiates
(Section 2: the fit trains a network by gradient descent; Section 3: the
network generates the PDF on the grid, and the custom operator returns the
convolution and its gradient)."""
from __future__ import annotations

import torch

from . import fkconv


class _Mlp(torch.autograd.Function):
    @staticmethod
    def forward(ctx, params, fkctx, mlp, nflav, nx):
        p = params.contiguous()
        ctx.save_for_backward(p)
        ctx.fk = (fkctx, mlp)
        return fkconv.fk_mlp_forward(fkctx, mlp, p, nflav, nx)

    @staticmethod
    def backward(ctx, gpdf):
        (p,) = ctx.saved_tensors
        fkctx, mlp = ctx.fk
        return fkconv.fk_mlp_backward(fkctx, mlp, p, gpdf.contiguous()), None, None, None, None


def mlp_pdf(fkctx, mlp: int, params: torch.Tensor, nflav: int, nx: int) -> torch.Tensor:
    """Differentiable PDF [nflav][nx][R] of the networks params [R][P]."""
    return _Mlp.apply(params, fkctx, mlp, nflav, nx)


class _Conv(torch.autograd.Function):
    @staticmethod
    def forward(ctx, pdf, fkctx, table, kind):
        fn = fkconv.fk_conv_had if kind == fkconv.FK_HAD else fkconv.fk_conv_dis
        out = fn(fkctx, table, pdf.contiguous())
        ctx.save_for_backward(pdf)
        ctx.fk = (fkctx, table, kind)
        return out

    @staticmethod
    def backward(ctx, gout):
        (pdf,) = ctx.saved_tensors
        fkctx, table, kind = ctx.fk
        g = fkconv.fk_conv_backward(fkctx, table, pdf.contiguous() if kind == fkconv.FK_HAD else None,
                                    gout.contiguous())
        return g, None, None, None


def fk_conv(fkctx, table: int, pdf: torch.Tensor) -> torch.Tensor:
    """Differentiable observables [ndata][R] of a table or group."""
    kind = fkconv.fk_table_info(fkctx, table)["kind"]
    return _Conv.apply(pdf, fkctx, table, kind)


class _Chi2(torch.autograd.Function):
    @staticmethod
    def forward(ctx, sigma, fkctx, cov, data):
        chi2, d = fkconv.fk_chi2(fkctx, cov, sigma.contiguous(), data, want_grad=True)
        ctx.save_for_backward(d)
        return chi2

    @staticmethod
    def backward(ctx, gchi2):
        (d,) = ctx.saved_tensors
        return d * gchi2.to(d.dtype)[None, :], None, None, None


def fk_chi2(fkctx, cov: int, sigma: torch.Tensor, data: torch.Tensor) -> torch.Tensor:
    """Differentiable chi2 per replica (float64 [R])."""
    return _Chi2.apply(sigma, fkctx, cov, data)
