"""Binning with counts aggregated per block in an LDS hash table (bin_aggregate = 1)
against the FP64 oracle: the same bins and results as per-wavefront runs, for compact
and recomputed records, several images in one call, the Hermitian fold, degridding and
plans, and a block with more distinct bins than the table holds (its surplus runs fall
back to global atomics)."""

import numpy as np
import pytest
import torch

import paper_1905_03213_amd as W
import synth
from oracle import wproj_ref as R

from gpu_util import oracle_grid, planted, rel_max, run_grid

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5}


def _check(params, uvw, vis, wt, offs=None):
    G, sw, cnt, host = run_grid(params, uvw, vis, wt, offs)
    (Gr, swr, cr), _, _ = oracle_grid(params, host, offs)
    assert cnt.tolist() == cr.tolist()
    assert np.allclose(sw, swr, rtol=1e-12, atol=0)
    assert rel_max(G, Gr) <= TOL[params["precision"]]
    return G


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("which", ["tracks", "cfg1w_variable_support", "multi_image", "fold"])
def test_aggregated_binning_matches_oracle(which, prec):
    offs = None
    extra = {}
    if which == "tracks":
        wl = synth.small_tracks()
    elif which == "cfg1w_variable_support":
        wl = synth.cfg1w(n_w=9, s_max=10)  # per-plane supports: records recomputed in the scatter
    elif which == "multi_image":
        wl = synth.cfg1w(n_w=9, s_max=10)
        offs = np.array([100, 700, 700, 1500, 1900])
        extra = {"n_images": 4}
    else:
        wl = synth.small_tracks()
        extra = {"w_mode": "fold"}
    uvw, vis, wt = planted(wl)
    params = {**wl.params, **extra, "precision": prec, "algorithm": "tiled", "bin_aggregate": True}
    _check(params, uvw, vis, wt, offs)


def test_aggregated_binning_crowded_table():
    """2048 visibilities per block spread over 2048^2 cells (16-cell tiles) and 64
    planes: nearly every run has a bin of its own, as many as the table has entries, more
    than linear probing places within its probe limit, so some runs take global atomics
    of their own."""
    rng = np.random.default_rng(21)
    n, cell = 2048, 1e-5
    params = dict(n=n, cell_rad=cell, n_wplanes=64, w_max=500.0, support=8, oversample=8,
                  kernel_image_size=32, n_images=1, precision="f32", algorithm="tiled",
                  tile=16, chunk=1024, bin_aggregate=True)
    nvis = 3 * 4096 + 123
    umax = (n / 2 - 8) / (n * cell)
    uvw = np.stack([rng.uniform(-umax, umax, nvis), rng.uniform(-umax, umax, nvis),
                    rng.uniform(-500.0, 500.0, nvis)], axis=1)
    vis = rng.standard_normal(nvis) + 1j * rng.standard_normal(nvis)
    wt = rng.uniform(0.5, 1.5, nvis)
    G = _check(params, uvw, vis, wt)
    G0 = _check({**params, "bin_aggregate": False}, uvw, vis, wt)
    assert rel_max(G, G0) <= 1e-6


def test_aggregated_degrid_and_plan():
    wl = synth.small_tracks()
    params = {**wl.params, "precision": "f32", "algorithm": "tiled", "bin_aggregate": True}
    plan = R.Plan(params)
    tabs = R.kernel_tables(plan)
    rng = np.random.default_rng(9)
    M = (rng.standard_normal((1, plan.n, plan.n)) + 1j * rng.standard_normal((1, plan.n, plan.n)))
    k = W.make_kernels(params)
    uvw = torch.as_tensor(np.asarray(wl.uvw)).cuda()
    out = torch.empty(uvw.shape[0], dtype=torch.complex64, device="cuda")
    W.degrid(k, uvw, torch.as_tensor(M.astype(np.complex64)).cuda(), out)
    ref = R.degrid(plan, tabs, np.asarray(wl.uvw), M)
    assert rel_max(out.to(torch.complex128).cpu().numpy(), ref) <= TOL["f32"]
    # a plan binned with aggregated counts grids like the one-shot call
    wt = torch.ones(uvw.shape[0], dtype=torch.float32, device="cuda")
    v = torch.as_tensor(np.asarray(wl.vis).astype(np.complex64)).cuda()
    p = W.Plan(k, uvw, wt)
    g1 = k.new_grid()
    p.grid(v, g1)
    g2 = k.new_grid()
    W.grid(k, uvw, v, wt, g2)
    torch.cuda.synchronize()
    assert rel_max(g1.cpu().numpy(), g2.cpu().numpy()) <= 1e-6
    p.free()
    k.free()


def test_autotune_reports_binning_choice():
    wl = synth.small_tracks()
    params = {**wl.params, "precision": "f32", "algorithm": "tiled"}
    k = W.make_kernels(params)
    uvw = torch.as_tensor(np.asarray(wl.uvw)).cuda()
    v = torch.as_tensor(np.asarray(wl.vis).astype(np.complex64)).cuda()
    wt = torch.ones(uvw.shape[0], dtype=torch.float32, device="cuda")
    W.autotune(k, uvw, v, wt)
    tile, chunk, agg = k.tuning_all()
    assert tile in (16, 32, 64) and chunk in (1024, 2048, 4096, 8192, 16384) and agg in (0, 1)
    # the choice is cached per shape and restored on a new handle of that shape
    k2 = W.make_kernels(params)
    W.autotune(k2, uvw, v, wt)
    assert k2.tuning_all() == (tile, chunk, agg)
    k.free()
    k2.free()
