"""Differentiable w-projection forward model (model image -> predicted visibilities).

    V = A(I) = degrid(DFT(kappa kappa I))

forward:  wproj_image(IMAGE_TO_GRID) then wproj_degrid, both in the library's kernels.
backward: for a real image and complex visibilities, torch passes g = dL/dRe V + i dL/dIm V
          and the image gradient is Re(A^H g) = kappa kappa Re(IDFT(grid(g)))
          = wproj_grid of g with unit weights, then wproj_image(GRID_TO_IMAGE_RAW).
Degridding and gridding are exact adjoints of each other (same footprints, same taps,
conjugated), so the gradient of chi^2 = sum W |V_obs - A(I)|^2 is -2 Re(A^H (W r)).
"""

from __future__ import annotations

from typing import Optional

import torch

from . import wproj as W


class WProjPredict(torch.autograd.Function):
    @staticmethod
    def forward(ctx, image: torch.Tensor, k: W.Kernels, uvw: torch.Tensor,
                image_offsets: Optional[torch.Tensor] = None):
        n, ni = k.params["n"], k.params.get("n_images", 1)
        img = image.detach().to(k.real).reshape(ni, n, n).contiguous()
        nvis = uvw.shape[0]
        ws = k.workspace(nvis, device=image.device)
        g = torch.empty((k.n_grids, n, n), dtype=k.cplx, device=image.device)
        W.image(k, W.IMAGE_TO_GRID, g, img, workspace=ws)
        out = torch.empty(nvis, dtype=k.cplx, device=image.device)
        W.degrid(k, uvw, g, out, image_offsets=image_offsets, workspace=ws)
        ctx.k = k
        ctx.save_for_backward(uvw, image_offsets if image_offsets is not None else torch.empty(0))
        ctx.has_off = image_offsets is not None
        ctx.shape = image.shape
        ctx.dtype = image.dtype
        return out

    @staticmethod
    def backward(ctx, grad_out: torch.Tensor):
        k = ctx.k
        uvw, off = ctx.saved_tensors
        off = off if ctx.has_off else None
        n, ni = k.params["n"], k.params.get("n_images", 1)
        nvis = uvw.shape[0]
        g = grad_out.to(k.cplx).contiguous()
        ones = torch.ones(nvis, dtype=k.real, device=g.device)
        ws = k.workspace(nvis, device=g.device)
        grid = torch.zeros((k.n_grids, n, n), dtype=k.cplx, device=g.device)
        W.grid(k, uvw, g, ones, grid, image_offsets=off, workspace=ws)
        img = torch.empty((ni, n, n), dtype=k.real, device=g.device)
        W.image(k, W.GRID_TO_IMAGE_RAW, grid, img, workspace=ws)
        return img.reshape(ctx.shape).to(ctx.dtype), None, None, None


def predict(image: torch.Tensor, k: W.Kernels, uvw: torch.Tensor,
            image_offsets: Optional[torch.Tensor] = None) -> torch.Tensor:
    """A(I): differentiable with respect to the (real) model image."""
    return WProjPredict.apply(image, k, uvw, image_offsets)


def chi2(image: torch.Tensor, k: W.Kernels, uvw: torch.Tensor, vis_obs: torch.Tensor,
         weight: torch.Tensor, image_offsets: Optional[torch.Tensor] = None) -> torch.Tensor:
    """chi^2 = sum_j W_j |V_obs,j - A(I)_j|^2, accumulated in float64."""
    r = vis_obs - predict(image, k, uvw, image_offsets)
    return (weight.to(torch.float64) * (r.real.double() ** 2 + r.imag.double() ** 2)).sum()
