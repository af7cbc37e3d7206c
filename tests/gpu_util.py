"""Shared helpers of the GPU parity tests (inputs, running the library, oracle side)."""

import numpy as np
import torch

import paper_1905_03213_amd as W
from oracle import wproj_ref as R

RDT = {"f64": torch.float64, "f32": torch.float32, "f32_f16table": torch.float32}
CDT = {"f64": torch.complex128, "f32": torch.complex64, "f32_f16table": torch.complex64}


def as_gpu_inputs(uvw, vis, weight, prec):
    """Device tensors in the precision the path takes, plus the exact host values
    (float64/complex128) those tensors hold, for the oracle."""
    cd, rd = CDT[prec], RDT[prec]
    v = torch.as_tensor(np.asarray(vis)).to(cd)
    w = torch.as_tensor(np.asarray(weight, dtype=np.float64)).to(rd)
    u = torch.as_tensor(np.asarray(uvw, dtype=np.float64))
    host = (u.numpy(), v.to(torch.complex128).numpy(), w.to(torch.float64).numpy())
    return (u.cuda(), v.cuda(), w.cuda()), host


def run_grid(params, uvw, vis, weight, image_offsets=None, k=None):
    """Grid on the GPU; returns (grid c128 numpy [ni][n][n], sumw, counters, host inputs)."""
    prec = params["precision"]
    (u, v, w), host = as_gpu_inputs(uvw, vis, weight, prec)
    own = k is None
    if own:
        k = W.make_kernels(params)
    g = k.new_grid()
    ni = params.get("n_images", 1)
    sw = torch.zeros(ni, dtype=torch.float64, device="cuda")
    cnt = torch.zeros(3, dtype=torch.int64, device="cuda")
    off = None if image_offsets is None else torch.as_tensor(np.asarray(image_offsets), dtype=torch.int64).cuda()
    W.grid(k, u, v, w, g, image_offsets=off, weight_sum=sw, counters=cnt)
    torch.cuda.synchronize()
    out = (g.to(torch.complex128).cpu().numpy(), sw.cpu().numpy(), cnt.cpu().numpy(), host)
    if own:
        k.free()
    return out


def oracle_grid(params, host, image_offsets=None):
    plan = R.Plan(params)
    tabs = R.kernel_tables(plan)
    return R.grid(plan, tabs, *host, image_offsets), plan, tabs


def rel_max(a, b):
    """max |a - b| / max |b|"""
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / np.abs(np.asarray(b)).max())


def rel_rms(a, b):
    d = np.asarray(a) - np.asarray(b)
    return float(np.sqrt(np.mean(np.abs(d) ** 2)) / np.abs(np.asarray(b)).max())


def grad_bound(pred_err_rms, r_rms, base):
    """Error bound of an FP32 chi^2 gradient relative to its peak.  The gradient
    -2 kappa kappa Re IDFT(grid(W r)) is linear in the residual r = V_obs - A(I), so the
    FP32 prediction's error dA enters as a residual error of relative size
    rms|dA| / rms|r|; r and dA are both noise-like over the rows, so their images scale
    alike, with a factor 3 for max against rms.  The backward pass (FP32 gridding and
    transform) adds at most the FP32 gridding tolerance `base`."""
    return base + 3.0 * pred_err_rms / r_rms


def planted(wl, seed=0, n_bad=7):
    """Copies of a workload's arrays with random weights and planted special rows:
    zero weights, a negative and a NaN weight, non-finite uvw, an off-grid row."""
    rng = np.random.default_rng(seed)
    uvw = np.asarray(wl.uvw).astype(np.float64, copy=True)  # numpy or CPU tensor
    vis = np.asarray(wl.vis).astype(np.complex128, copy=True)
    wt = rng.uniform(0.25, 2.0, uvw.shape[0])
    idx = rng.choice(uvw.shape[0], n_bad, replace=False)
    wt[idx[0]] = 0.0
    wt[idx[1]] = -1.0
    wt[idx[2]] = np.nan
    uvw[idx[3], 0] = np.nan
    uvw[idx[4], 2] = np.inf
    uvw[idx[5], 1] = 1e12
    wt[idx[6]] = 0.0
    return uvw, vis, wt
