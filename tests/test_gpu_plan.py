"""Plans (a binning kept for repeated gridding and degridding of the same rows) against
the oracle and against the one-shot calls: the same grid for several sets of
visibilities through one plan, the same weight sums and counters, degridding of the
rows the plan grids (0 for the others), several images, and a plan that keeps its
tuning when the handle is re-tuned."""

import numpy as np
import pytest
import torch

import paper_1905_03213_amd as W
import synth
from oracle import wproj_ref as R

from gpu_util import CDT, RDT, oracle_grid, planted, rel_max

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5, "f32_f16table": 1e-3}


def _workload(which):
    if which == "cfg1":
        return synth.cfg1()
    if which == "cfg1w":
        return synth.cfg1w()
    wl = synth.small_tracks()
    wl.uvw, wl.vis, wl.weight = wl.uvw.numpy(), wl.vis.numpy(), wl.weight.numpy()
    return wl


@pytest.mark.parametrize("prec", ["f64", "f32", "f32_f16table"])
@pytest.mark.parametrize("which", ["cfg1", "cfg1w", "tracks"])
def test_planned_grid_matches_oracle_for_several_vis(which, prec):
    wl = _workload(which)
    uvw, vis, wt = planted(wl)
    params = {**wl.params, "precision": prec, "algorithm": "tiled"}
    k = W.make_kernels(params)
    u = torch.as_tensor(uvw).cuda()
    w_t = torch.as_tensor(wt).to(RDT[prec]).cuda()
    sw = torch.zeros(1, dtype=torch.float64, device="cuda")
    cnt = torch.zeros(3, dtype=torch.int64, device="cuda")
    plan = W.Plan(k, u, w_t, weight_sum=sw, counters=cnt)
    rng = np.random.default_rng(7)
    for rep in range(3):
        v = vis * (1.0 + rep) + (rng.standard_normal(vis.shape[0]) + 1j * rng.standard_normal(vis.shape[0]))
        v_t = torch.as_tensor(v).to(CDT[prec]).cuda()
        g = k.new_grid()
        plan.grid(v_t, g)
        torch.cuda.synchronize()
        host = (uvw, v_t.to(torch.complex128).cpu().numpy(), w_t.double().cpu().numpy())
        (Gr, swr, cr), _, _ = oracle_grid(params, host)
        assert rel_max(g.to(torch.complex128).cpu().numpy(), Gr) <= TOL[prec]
    assert np.allclose(sw.cpu().numpy(), swr, rtol=1e-12, atol=0)
    assert cnt.cpu().tolist() == cr.tolist()
    plan.free()
    k.free()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_planned_degrid_predicts_gridded_rows(prec):
    wl = synth.cfg1w(n_w=9, s_max=10)
    uvw, _, wt = planted(wl)
    params = {**wl.params, "precision": prec, "algorithm": "tiled"}
    plan_o = R.Plan(params)
    tabs = R.kernel_tables(plan_o)
    n = plan_o.n
    rng = np.random.default_rng(4)
    M = rng.standard_normal((1, n, n)) + 1j * rng.standard_normal((1, n, n))
    M_t = torch.as_tensor(M).to(CDT[prec]).cuda()
    k = W.make_kernels(params)
    w_t = torch.as_tensor(wt).to(RDT[prec]).cuda()
    plan = W.Plan(k, torch.as_tensor(uvw).cuda(), w_t)
    out = torch.full((uvw.shape[0],), 7.0 + 7.0j, dtype=CDT[prec], device="cuda")
    plan.degrid(M_t, out)
    ref = R.degrid(plan_o, tabs, uvw, M_t.to(torch.complex128).cpu().numpy())
    gridded = R.snap(plan_o, uvw, w_t.double().cpu().numpy())["valid"]
    ref[~gridded] = 0.0  # rows the plan does not grid (flagged, bad weight, dropped)
    got = out.to(torch.complex128).cpu().numpy()
    assert rel_max(got, ref) <= TOL[prec]
    assert np.count_nonzero(got) == np.count_nonzero(ref)
    plan.free()
    k.free()


def test_planned_multi_image_and_empty():
    wl = synth.cfg1w(n_w=9, s_max=10)
    offs = np.array([100, 700, 700, 1500, 1900])
    params = {**wl.params, "precision": "f64", "algorithm": "tiled", "n_images": 4}
    k = W.make_kernels(params)
    u = torch.as_tensor(wl.uvw).cuda()
    w_t = torch.as_tensor(wl.weight).cuda()
    off_t = torch.as_tensor(offs).cuda()
    plan = W.Plan(k, u, w_t, image_offsets=off_t)
    g = k.new_grid()
    v_t = torch.as_tensor(wl.vis).cuda()
    plan.grid(v_t, g)
    torch.cuda.synchronize()
    (Gr, _, _), _, _ = oracle_grid(params, (wl.uvw, wl.vis, wl.weight), offs)
    assert rel_max(g.cpu().numpy(), Gr) <= 1e-12
    plan.free()
    empty = W.Plan(k, u[:0], w_t[:0], image_offsets=torch.zeros(5, dtype=torch.int64, device="cuda"))
    g2 = k.new_grid()
    empty.grid(v_t[:0], g2)
    torch.cuda.synchronize()
    assert not g2.any()
    empty.free()
    k.free()


def test_plan_keeps_its_tuning():
    wl = synth.small_tracks(n=256, cell=8e-5, n_chan=8, hours=2.0, dt_s=30.0)
    params = {**wl.params, "precision": "f32", "algorithm": "tiled", "tile": 16, "chunk": 1024}
    k = W.make_kernels(params)
    u = wl.uvw.cuda()
    v_t = wl.vis.to(torch.complex64).cuda()
    w_t = wl.weight.float().cuda()
    plan = W.Plan(k, u, w_t)
    W.autotune(k, u, v_t, w_t)  # re-tunes the handle; the plan's binning stays valid
    g = k.new_grid()
    plan.grid(v_t, g)
    g1 = k.new_grid()
    W.grid(k, u, v_t, w_t, g1)
    torch.cuda.synchronize()
    assert rel_max(g.to(torch.complex128).cpu().numpy(), g1.to(torch.complex128).cpu().numpy()) <= 1e-5
    plan.free()
    k.free()
