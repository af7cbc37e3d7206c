"""w-stacking hybrid (w_mode "stack") on the GPU against the FP64 oracle, through the C ABI.

Layers of width 2 w_max / L, each with its own grid; a row is gridded onto its layer's
grid with the kernel of its residual w - w_l.  Covered: residual-plane tables, per-row
footprints (plane counted across layers), binned and plain gridding with several images,
the layer-combining grid -> image pass, image -> grids, tiled and plain degridding, plans,
the chi^2 gradient, and the 2048^2 benchmark tracks on 16 layers at full size."""

import os

import numpy as np
import pytest
import torch

import paper_1905_03213_amd as W
import synth
from oracle import cref
from oracle import wproj_ref as R
from paper_1905_03213_amd.autograd import chi2

from gpu_util import CDT, RDT, as_gpu_inputs, oracle_grid, planted, rel_max, run_grid

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5, "f32_f16table": 1e-3}


def _params(which, prec, algo="tiled", L=6, n_w=5):
    wl = synth.cfg1w(n_w=9, s_max=7) if which == "cfg1w" else synth.small_tracks()
    if which != "cfg1w":
        wl.uvw, wl.vis, wl.weight = wl.uvw.numpy(), wl.vis.numpy(), wl.weight.numpy()
    params = {**wl.params, "precision": prec, "algorithm": algo, "w_mode": "stack",
              "n_wlayers": L, "n_wplanes": n_w, "support_per_plane": None,
              "support": wl.params["support"]}
    return wl, params


@pytest.mark.parametrize("prec", ["f64", "f32", "f32_f16table"])
def test_stack_tables_match_oracle(prec):
    _, params = _params("cfg1w", prec)
    k = W.make_kernels(params)
    flat, _ = R.flat_tables(R.kernel_tables(R.Plan(params)))
    raw = k.export(W._lib.EXPORT_TABLES)
    if prec == "f64":
        got, tol = raw.view(torch.complex128).cpu().numpy(), 1e-12
    elif prec == "f32":
        got, tol = raw.view(torch.complex64).cpu().numpy().astype(np.complex128), 2 ** -23
    else:
        h = raw.view(torch.float16).cpu().numpy().astype(np.float64)
        got, tol = h[0::2] + 1j * h[1::2], 2 ** -10
    assert np.abs(got - flat).max() <= tol * np.abs(flat).max()
    k.free()


def test_stack_footprints_match_oracle():
    wl, params = _params("cfg1w", "f64")
    uvw, _, wt = planted(wl)
    k = W.make_kernels(params)
    out = W.footprints(k, torch.as_tensor(uvw).cuda(), torch.as_tensor(wt).cuda()).cpu().numpy()
    geo = R.snap(R.Plan(params), uvw, wt)
    val = geo["valid"]
    assert np.array_equal(out[:, 5] == 0, val)
    assert np.array_equal(out[val, 4], geo["layer"][val] * params["n_wplanes"] + geo["p"][val])
    for i, key in enumerate(("x0", "y0", "ou", "ov")):
        assert np.array_equal(out[val, i], geo[key][val]), key
    assert len(np.unique(geo["layer"][val])) == params["n_wlayers"]
    k.free()


# the plain path is the FP64 comparison path: it runs in FP64 only
ALGO_PREC = [("tiled", "f64"), ("tiled", "f32"), ("tiled", "f32_f16table"), ("plain", "f64")]


@pytest.mark.parametrize("which", ["cfg1w", "tracks"])
@pytest.mark.parametrize("algo,prec", ALGO_PREC)
def test_stack_grid_and_image_match_oracle(algo, prec, which):
    wl, params = _params(which, prec, algo)
    uvw, vis, wt = planted(wl)
    G, sw, cnt, host = run_grid(params, uvw, vis, wt)
    (Gr, swr, cr), plan, _ = oracle_grid(params, host)
    assert G.shape == Gr.shape == (params["n_wlayers"], plan.n, plan.n)
    assert cnt.tolist() == cr.tolist()
    assert np.allclose(sw, swr, rtol=1e-12, atol=0)
    assert rel_max(G, Gr) <= TOL[prec]
    # grid -> image combines the layers: GPU transform of the GPU grid against the oracle's
    k = W.make_kernels(params)
    g = torch.as_tensor(G).to(CDT[prec]).cuda()
    g_in = g.to(torch.complex128).cpu().numpy()  # the transform below runs in place
    img = torch.empty((1, plan.n, plan.n), dtype=RDT[prec], device="cuda")
    W.image(k, W.GRID_TO_IMAGE, g, img, torch.as_tensor(sw).cuda())
    ref = R.grid_to_image(plan, g_in, sw)[0]
    q = plan.n // 4
    got = img[0].double().cpu().numpy()
    e = rel_max(got[q:-q, q:-q], ref[q:-q, q:-q])
    assert e <= (1e-12 if prec == "f64" else 1e-5), e
    k.free()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_stack_image_to_grids_and_degrid(prec):
    wl, params = _params("cfg1w", prec)
    plan = R.Plan(params)
    tabs = R.kernel_tables(plan)
    rng = np.random.default_rng(17)
    n = plan.n
    q = n // 4
    I = np.zeros((1, n, n))
    I[0, q:-q, q:-q] = rng.standard_normal((n - 2 * q, n - 2 * q))
    I = I.astype(np.float64 if prec == "f64" else np.float32)
    for algo in ("tiled", "plain"):
        k = W.make_kernels({**params, "algorithm": algo})
        g = k.new_grid()
        W.image(k, W.IMAGE_TO_GRID, g, torch.as_tensor(I).cuda())
        M = R.image_to_grid(plan, I.astype(np.float64))
        assert g.shape[0] == params["n_wlayers"]
        assert rel_max(g.to(torch.complex128).cpu().numpy(), M) <= TOL[prec]
        out = torch.full((wl.nvis,), 7.0 + 7.0j, dtype=CDT[prec], device="cuda")
        W.degrid(k, torch.as_tensor(wl.uvw).cuda(), g, out)
        ref = R.degrid(plan, tabs, wl.uvw, g.to(torch.complex128).cpu().numpy())
        assert rel_max(out.to(torch.complex128).cpu().numpy(), ref) <= TOL[prec]
        k.free()


def test_stack_plan_and_chi2_gradient():
    wl, params = _params("tracks", "f64")
    plan = R.Plan(params)
    tabs = R.kernel_tables(plan)
    uvw, vis, wt = planted(wl)
    k = W.make_kernels(params)
    (u, v, w), host = as_gpu_inputs(uvw, vis, wt, "f64")
    pl = W.Plan(k, u, w)
    g = k.new_grid()
    pl.grid(v, g)
    Gr = R.grid(plan, tabs, *host)[0]
    assert rel_max(g.cpu().numpy(), Gr) <= 1e-12
    pl.free()
    # chi^2 gradient of a model image against the oracle's adjoint (FP64)
    keep = R.snap(plan, uvw, np.ones(len(uvw)))["valid"]
    U = torch.as_tensor(uvw[keep]).cuda()
    rng = np.random.default_rng(19)
    n = plan.n
    q = n // 4
    img0 = np.zeros((n, n))
    img0[q:-q, q:-q] = 0.01 * rng.standard_normal((n - 2 * q, n - 2 * q))
    Vo = torch.as_tensor(vis[keep]).cuda()
    Wt = torch.as_tensor(rng.uniform(0.5, 2.0, int(keep.sum()))).cuda()
    I = torch.tensor(img0, device="cuda", requires_grad=True)
    chi2(I, k, U, Vo, Wt).backward()
    ref = R.chi2_grad(plan, tabs, uvw[keep], Vo.cpu().numpy(), Wt.cpu().numpy(), img0)[0]
    assert rel_max(I.grad.cpu().numpy()[q:-q, q:-q], ref[q:-q, q:-q]) <= 1e-9
    k.free()


def test_stack_full_size_sixteen_layers():
    """The benchmark tracks (2048^2, 6.47e7 visibilities, S = 8) on 16 layers with 9
    residual planes each: FP32 binned gridding against the C oracle at every cell of the
    16 grids, and the combined image on the inner half."""
    threads = max(1, min(16, len(os.sched_getaffinity(0))))
    wl = synth.cfg2(device="cuda")
    params = {**wl.params, "precision": "f32", "algorithm": "tiled", "w_mode": "stack",
              "n_wlayers": 16, "n_wplanes": 9}
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
    e = rel_max(G, Gr)
    assert cnt.cpu().tolist() == cr.tolist()
    assert np.allclose(sw.cpu().numpy(), swr, rtol=1e-9, atol=0)
    img = torch.empty((1, plan.n, plan.n), dtype=torch.float32, device="cuda")
    W.image(k, W.GRID_TO_IMAGE, g, img, sw)
    del G
    ref = R.grid_to_image(plan, Gr, swr)[0]
    q = plan.n // 4
    ei = rel_max(img[0].double().cpu().numpy()[q:-q, q:-q], ref[q:-q, q:-q])
    print(f"[stack full size] 16 layers: grid rel max {e:.3e}, image inner rel max {ei:.3e}", flush=True)
    assert e <= 1e-5 and ei <= 1e-5
    k.free()
