"""Differentiable w-projection forward model (model image -> predicted visibilities).

    V = A(I) = degrid(DFT(kappa kappa I))

forward:  wproj_image(IMAGE_TO_GRID) then wproj_degrid, both in the library's kernels.
backward: for a real image and complex visibilities, torch passes g = dL/dRe V + i dL/dIm V
          and the image gradient is Re(A^H g) = kappa kappa Re(IDFT(grid(g)))
          = wproj_grid of g with unit weights, then wproj_image(GRID_TO_IMAGE_RAW).
Degridding and gridding are exact adjoints of each other (same footprints, same taps,
conjugated), so the gradient of chi^2 = sum W |V_obs - A(I)|^2 is -2 Re(A^H (W r)).

The rows' binning depends on uvw only, so an imaging loop that evaluates the model many
times on the same rows can bin them once: pass a plan (make_plan) and the forward pass
degrids through it (wproj_degrid_planned) and the backward pass grids through it
(wproj_grid_planned) instead of binning the rows twice per evaluation.
"""

from __future__ import annotations

from typing import Optional

import torch

from . import wproj as W


class WProjPredict(torch.autograd.Function):
    @staticmethod
    def forward(ctx, image: torch.Tensor, k: W.Kernels, uvw: torch.Tensor,
                image_offsets: Optional[torch.Tensor] = None, plan: Optional[W.Plan] = None):
        n, ni = k.params["n"], k.params.get("n_images", 1)
        img = image.detach().to(k.real).reshape(ni, n, n).contiguous()
        nvis = uvw.shape[0]
        # with a plan the binning workspace is the plan's; the FFT needs only its own part
        ws = k.workspace(0 if plan is not None else nvis, device=image.device)
        g = torch.empty((k.n_grids, n, n), dtype=k.cplx, device=image.device)
        W.image(k, W.IMAGE_TO_GRID, g, img, workspace=ws)
        out = torch.empty(nvis, dtype=k.cplx, device=image.device)
        if plan is not None:
            plan.degrid(g, out)
        else:
            W.degrid(k, uvw, g, out, image_offsets=image_offsets, workspace=ws)
        ctx.k = k
        ctx.plan = plan
        ctx.save_for_backward(uvw, image_offsets if image_offsets is not None else torch.empty(0))
        ctx.has_off = image_offsets is not None
        ctx.shape = image.shape
        ctx.dtype = image.dtype
        return out

    @staticmethod
    def backward(ctx, grad_out: torch.Tensor):
        k, plan = ctx.k, ctx.plan
        uvw, off = ctx.saved_tensors
        off = off if ctx.has_off else None
        n, ni = k.params["n"], k.params.get("n_images", 1)
        nvis = uvw.shape[0]
        g = grad_out.to(k.cplx).contiguous()
        ws = k.workspace(0 if plan is not None else nvis, device=g.device)
        grid = torch.zeros((k.n_grids, n, n), dtype=k.cplx, device=g.device)
        if plan is not None:
            plan.grid(g, grid)  # the plan's weights are 1
        else:
            ones = torch.ones(nvis, dtype=k.real, device=g.device)
            W.grid(k, uvw, g, ones, grid, image_offsets=off, workspace=ws)
        img = torch.empty((ni, n, n), dtype=k.real, device=g.device)
        W.image(k, W.GRID_TO_IMAGE_RAW, grid, img, workspace=ws)
        return img.reshape(ctx.shape).to(ctx.dtype), None, None, None, None


class Chi2Loss(torch.autograd.Function):
    """chi^2 = sum_j W_j |V_obs,j - V_j|^2 and its gradient with respect to V in one pass of
    the library's wproj_chi2 (FP64 sum in a fixed order)."""

    @staticmethod
    def forward(ctx, pred: torch.Tensor, vis_obs: torch.Tensor, weight: torch.Tensor):
        grad = torch.empty_like(pred)
        loss = W.chi2(vis_obs, pred, weight, grad=grad)
        ctx.save_for_backward(grad)
        return loss.reshape(())

    @staticmethod
    def backward(ctx, grad_out: torch.Tensor):
        (grad,) = ctx.saved_tensors
        return grad * grad_out.to(grad.real.dtype), None, None


def make_plan(k: W.Kernels, uvw: torch.Tensor,
              image_offsets: Optional[torch.Tensor] = None) -> W.Plan:
    """The rows' binning with unit weights, for predict and chi2 on these rows: it degrids
    every row wproj_degrid predicts and grids the gradient with weight 1, as the adjoint
    needs.  Free it (Plan.free) when the rows change."""
    ones = torch.ones(uvw.shape[0], dtype=k.real, device=uvw.device)
    return W.Plan(k, uvw, ones, image_offsets=image_offsets)


def predict(image: torch.Tensor, k: W.Kernels, uvw: torch.Tensor,
            image_offsets: Optional[torch.Tensor] = None, plan: Optional[W.Plan] = None) -> torch.Tensor:
    """A(I): differentiable with respect to the (real) model image.  plan: make_plan of
    the same k, uvw and image_offsets, or None to bin the rows in each call."""
    return WProjPredict.apply(image, k, uvw, image_offsets, plan)


def chi2(image: torch.Tensor, k: W.Kernels, uvw: torch.Tensor, vis_obs: torch.Tensor,
         weight: torch.Tensor, image_offsets: Optional[torch.Tensor] = None,
         plan: Optional[W.Plan] = None) -> torch.Tensor:
    """chi^2 = sum_j W_j |V_obs,j - A(I)_j|^2, accumulated in float64 (wproj_chi2)."""
    pred = predict(image, k, uvw, image_offsets, plan)
    return Chi2Loss.apply(pred, vis_obs.to(k.cplx).contiguous(), weight.to(k.real).contiguous())
