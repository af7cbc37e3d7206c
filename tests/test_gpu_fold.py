"""Hermitian-fold w modes on the GPU against the FP64 oracle, through the C ABI.

With a fold a row with w < 0 is gridded as conj(V) at (-u, -v, -w), so the planes only
cover [0, w_max]: spaced evenly in w ("fold") or in sqrt(w) ("fold_sqrt").  Covered:
kernel tables at the folded plane values, per-row footprints and the fold flag, binned
gridding (fixed support with packed records, per-plane supports with the recomputing
scatter), the plain gridder, tiled and plain degridding (conjugate for folded rows),
plans (the fold carried by the sign of the kept weight), and a full-size run on the
2048^2 benchmark tracks with half the planes."""

import os

import numpy as np
import pytest
import torch

import paper_1905_03213_amd as W
import synth
from oracle import cref
from oracle import wproj_ref as R

from gpu_util import CDT, RDT, oracle_grid, planted, rel_max, run_grid

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5, "f32_f16table": 1e-3}
MODES = ["fold", "fold_sqrt"]


def _wl(which):
    if which == "cfg1":
        wl = synth.cfg1()
    elif which == "cfg1w":
        wl = synth.cfg1w(n_w=17)
    else:
        wl = synth.small_tracks()
        wl.uvw, wl.vis, wl.weight = wl.uvw.numpy(), wl.vis.numpy(), wl.weight.numpy()
    return wl


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("prec", ["f64", "f32", "f32_f16table"])
def test_fold_tables_match_oracle(mode, prec):
    wl = _wl("cfg1w")
    params = {**wl.params, "precision": prec, "algorithm": "tiled", "w_mode": mode}
    k = W.make_kernels(params)
    plan = R.Plan(params)
    flat, offs = R.flat_tables(R.kernel_tables(plan))
    raw = k.export(W._lib.EXPORT_TABLES)
    if prec == "f64":
        got = raw.view(torch.complex128).cpu().numpy()
        tol = 1e-12
    elif prec == "f32":
        got = raw.view(torch.complex64).cpu().numpy().astype(np.complex128)
        tol = 2 ** -23
    else:
        h = raw.view(torch.float16).cpu().numpy().astype(np.float64)
        got = h[0::2] + 1j * h[1::2]
        tol = 2 ** -10
    assert np.abs(got - flat).max() <= tol * np.abs(flat).max()
    k.free()


@pytest.mark.parametrize("mode", MODES)
def test_fold_footprints_match_oracle(mode):
    wl = _wl("cfg1w")
    uvw, _, wt = planted(wl)
    params = {**wl.params, "precision": "f64", "algorithm": "tiled", "w_mode": mode}
    k = W.make_kernels(params)
    out = W.footprints(k, torch.as_tensor(uvw).cuda(), torch.as_tensor(wt).cuda()).cpu().numpy()
    geo = R.snap(R.Plan(params), uvw, wt)
    val = geo["valid"]
    assert np.array_equal(np.isin(out[:, 5], (0, 4)), val)
    assert np.array_equal(out[:, 5] == 4, geo["fold"])
    assert geo["fold"].sum() > 0 and (val & ~geo["fold"]).sum() > 0
    for i, key in enumerate(("x0", "y0", "ou", "ov", "p")):
        assert np.array_equal(out[val, i], geo[key][val]), key
    k.free()


# the plain path is the FP64 comparison path: it runs in FP64 only
ALGO_PREC = [("tiled", "f64"), ("tiled", "f32"), ("tiled", "f32_f16table"), ("plain", "f64")]


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("which", ["cfg1", "cfg1w", "tracks"])
@pytest.mark.parametrize("algo,prec", ALGO_PREC)
def test_fold_grid_matches_oracle(algo, prec, which, mode):
    wl = _wl(which)
    uvw, vis, wt = planted(wl)
    params = {**wl.params, "precision": prec, "algorithm": algo, "w_mode": mode}
    G, sw, cnt, host = run_grid(params, uvw, vis, wt)
    (Gr, swr, cr), _, _ = oracle_grid(params, host)
    assert cnt.tolist() == cr.tolist()
    assert np.allclose(sw, swr, rtol=1e-12, atol=0)
    assert rel_max(G, Gr) <= TOL[prec]


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("which", ["cfg1", "cfg1w"])
@pytest.mark.parametrize("algo", ["tiled", "plain"])
def test_fold_degrid_matches_oracle(algo, which, mode):
    wl = _wl(which)
    prec = "f32" if algo == "tiled" else "f64"
    params = {**wl.params, "precision": prec, "algorithm": algo, "w_mode": mode}
    plan = R.Plan(params)
    tabs = R.kernel_tables(plan)
    n = plan.n
    rng = np.random.default_rng(13)
    M = (rng.standard_normal((1, n, n)) + 1j * rng.standard_normal((1, n, n))).astype(
        np.complex64 if prec == "f32" else np.complex128)
    k = W.make_kernels(params)
    uvw = np.asarray(wl.uvw, dtype=np.float64)
    out = torch.full((uvw.shape[0],), 7.0 + 7.0j, dtype=CDT[prec], device="cuda")
    W.degrid(k, torch.as_tensor(uvw).cuda(), torch.as_tensor(M).cuda(), out)
    ref = R.degrid(plan, tabs, uvw, M.astype(np.complex128))
    got = out.to(torch.complex128).cpu().numpy()
    assert rel_max(got, ref) <= TOL[prec]
    assert np.count_nonzero(got) == np.count_nonzero(ref)
    assert R.snap(plan, uvw, np.ones(len(uvw)))["fold"].sum() > 0
    k.free()


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_fold_plan_grid_and_degrid(prec, mode):
    wl = _wl("tracks")
    uvw, vis, wt = planted(wl)
    params = {**wl.params, "precision": prec, "algorithm": "tiled", "w_mode": mode}
    k = W.make_kernels(params)
    u = torch.as_tensor(uvw).cuda()
    w_t = torch.as_tensor(wt).to(RDT[prec]).cuda()
    plan = W.Plan(k, u, w_t)
    v_t = torch.as_tensor(vis).to(CDT[prec]).cuda()
    g = k.new_grid()
    plan.grid(v_t, g)
    out = torch.full((uvw.shape[0],), 7.0 + 7.0j, dtype=CDT[prec], device="cuda")
    plan.degrid(g, out)
    torch.cuda.synchronize()
    host = (uvw, v_t.to(torch.complex128).cpu().numpy(), w_t.double().cpu().numpy())
    (Gr, _, _), oplan, tabs = oracle_grid(params, host)
    G = g.to(torch.complex128).cpu().numpy()
    assert rel_max(G, Gr) <= TOL[prec]
    geo = R.snap(oplan, uvw, host[2])
    ref = np.where(geo["valid"], R.degrid(oplan, tabs, uvw, G), 0.0)
    assert rel_max(out.to(torch.complex128).cpu().numpy(), ref) <= TOL[prec]
    plan.free()
    k.free()


def test_fold_full_size_half_the_planes():
    """The benchmark tracks (2048^2, 6.47e7 visibilities, S = 8) folded onto 64 planes over
    [0, w_max] (the plane spacing of 128 linear planes over [-w_max, w_max], half the
    tables): FP32 binned gridding against the C oracle at every cell."""
    threads = max(1, min(16, len(os.sched_getaffinity(0))))
    wl = synth.cfg2(device="cuda")
    params = {**wl.params, "precision": "f32", "algorithm": "tiled", "n_wplanes": 64, "w_mode": "fold"}
    k = W.make_kernels(params)
    vis = wl.vis.to(torch.complex64)
    wt = wl.weight.to(torch.float32)
    W.autotune(k, wl.uvw, vis, wt)
    g = k.new_grid()
    sw = torch.zeros(1, dtype=torch.float64, device="cuda")
    cnt = torch.zeros(3, dtype=torch.int64, device="cuda")
    W.grid(k, wl.uvw, vis, wt, g, weight_sum=sw, counters=cnt)
    torch.cuda.synchronize()
    plan = R.Plan({**params, "precision": "f64"})
    tabs = R.kernel_tables(plan)
    Gr, swr, cr = cref.grid(plan, tabs, wl.uvw.cpu().numpy(), vis.to(torch.complex128).cpu().numpy(),
                            wt.double().cpu().numpy(), nthreads=threads)
    G = g.to(torch.complex128).cpu().numpy()
    del g
    e = rel_max(G, Gr)
    print(f"[fold full size] 64 folded planes: grid rel max {e:.3e}", flush=True)
    assert cnt.cpu().tolist() == cr.tolist()
    assert np.allclose(sw.cpu().numpy(), swr, rtol=1e-9, atol=0)
    assert e <= TOL["f32"]
    k.free()
