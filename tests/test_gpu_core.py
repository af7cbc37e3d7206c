"""GPU parity of the library's core steps against the FP64 oracle, through the C ABI.

Kernel tables, the plain (no binning) gridder, the grid<->image transforms and the
plain degridder, at sizes the oracle finishes in seconds.
"""

import numpy as np
import pytest
import torch

import paper_1905_03213_amd as W
import synth
from oracle import wproj_ref as R

from gpu_util import CDT, RDT, as_gpu_inputs, oracle_grid, planted, rel_max, run_grid

pytestmark = pytest.mark.gpu


def _flat_oracle_tables(params):
    plan = R.Plan(params)
    flat, offs = R.flat_tables(R.kernel_tables(plan))
    return plan, flat, offs


@pytest.mark.parametrize("prec", ["f64", "f32", "f32_f16table"])
@pytest.mark.parametrize("which", ["cfg1", "cfg1w"])
def test_tables_match_oracle(prec, which):
    wl = synth.cfg1() if which == "cfg1" else synth.cfg1w()
    params = {**wl.params, "precision": prec, "algorithm": "plain"}
    k = W.make_kernels(params)
    plan, flat, offs = _flat_oracle_tables(params)
    got_off = k.export(W._lib.EXPORT_TABLE_OFFSETS).view(torch.int64).cpu().numpy()
    assert got_off.tolist() == offs.tolist()
    raw = k.export(W._lib.EXPORT_TABLES)
    if prec == "f64":
        got = raw.view(torch.complex128).cpu().numpy()
        assert np.abs(got - flat).max() <= 1e-12 * np.abs(flat).max()
    elif prec == "f32":
        got = raw.view(torch.complex64).cpu().numpy().astype(np.complex128)
        ref = flat.astype(np.complex64).astype(np.complex128)
        # both sides round float64 values that agree to ~1e-15 of the peak tap once,
        # so they differ by at most one float32 ulp of the peak
        assert np.abs(got - ref).max() <= 2.0 ** -23 * np.abs(flat).max()
    else:
        h = raw.view(torch.float16).cpu().numpy().astype(np.float64)
        got = h[0::2] + 1j * h[1::2]
        ref = flat.real.astype(np.float16).astype(np.float64) + 1j * flat.imag.astype(np.float16).astype(np.float64)
        assert np.abs(got - ref).max() <= 2.0 ** -10 * np.abs(flat).max()
    kap = k.export(W._lib.EXPORT_KAPPA).view(torch.float64).cpu().numpy()
    assert np.abs(kap - R.kappa(plan)).max() <= 1e-12 * np.abs(R.kappa(plan)).max()
    sup = k.export(W._lib.EXPORT_SUPPORTS).view(torch.int32).cpu().numpy()
    assert sup.tolist() == plan.supports
    k.free()


@pytest.mark.parametrize("which", ["cfg1", "cfg1w"])
def test_plain_grid_f64(which):
    wl = synth.cfg1() if which == "cfg1" else synth.cfg1w()
    uvw, vis, wt = planted(wl)
    params = {**wl.params, "precision": "f64", "algorithm": "plain"}
    G, sw, cnt, host = run_grid(params, uvw, vis, wt)
    (Gr, swr, cr), _, _ = oracle_grid(params, host)
    assert rel_max(G, Gr) <= 1e-12
    assert abs(sw[0] - swr[0]) <= 1e-12 * swr[0]
    assert cnt.tolist() == cr.tolist() and cr[0] >= 3 and cr[2] == 2


@pytest.mark.parametrize("prec,tol", [("f32", 1e-5), ("f32_f16table", 1e-3)])
def test_plain_grid_reduced_precision(prec, tol):
    wl = synth.cfg1()
    params = {**wl.params, "precision": prec, "algorithm": "plain"}
    G, sw, cnt, host = run_grid(params, wl.uvw, wl.vis, wl.weight)
    (Gr, swr, cr), plan, _ = oracle_grid(params, host)
    assert rel_max(G, Gr) <= tol
    assert cnt.tolist() == cr.tolist()


def test_plain_grid_multi_image_and_empty_ranges():
    wl = synth.cfg1w(n_w=9, s_max=10)
    params = {**wl.params, "precision": "f64", "algorithm": "plain", "n_images": 4}
    offs = np.array([100, 700, 700, 1500, 1900])  # rows 0..99 and 1900.. belong to no image
    G, sw, cnt, host = run_grid(params, wl.uvw, wl.vis, wl.weight, offs)
    (Gr, swr, cr), _, _ = oracle_grid(params, host, offs)
    assert rel_max(G, Gr) <= 1e-12
    assert np.abs(G[1]).max() == 0.0
    assert np.allclose(sw, swr, rtol=1e-12, atol=0)


@pytest.mark.parametrize("algo", ["plain", "tiled"])
def test_grid_empty_input_leaves_grid(algo):
    """No visibilities: the grid is left as it was and degridding writes nothing (the
    tiled path then has no records, no work items and an empty work order)."""
    wl = synth.cfg1()
    params = {**wl.params, "precision": "f32", "algorithm": algo}
    k = W.make_kernels(params)
    g = k.new_grid() + 1.5
    uvw0 = torch.empty((0, 3), dtype=torch.float64, device="cuda")
    W.grid(k, uvw0, torch.empty(0, dtype=torch.complex64, device="cuda"),
           torch.empty(0, dtype=torch.float32, device="cuda"), g)
    torch.cuda.synchronize()
    assert bool((g == 1.5).all())
    out = torch.empty(0, dtype=torch.complex64, device="cuda")
    W.degrid(k, uvw0, g, out)
    torch.cuda.synchronize()
    k.free()


@pytest.mark.parametrize("prec,tol", [("f64", 1e-12), ("f32", 2e-6)])
def test_grid_to_image_and_back(prec, tol):
    wl = synth.cfg1w()
    params = {**wl.params, "precision": prec, "algorithm": "plain", "n_images": 2}
    plan = R.Plan(params)
    rng = np.random.default_rng(3)
    n = plan.n
    Gin = rng.standard_normal((2, n, n)) + 1j * rng.standard_normal((2, n, n))
    Gin = Gin.astype(np.complex64 if prec != "f64" else np.complex128).astype(np.complex128)
    sw = np.array([123.0, 4.5])
    k = W.make_kernels(params)
    g = torch.as_tensor(Gin).to(CDT[prec]).cuda()
    img = torch.empty((2, n, n), dtype=RDT[prec], device="cuda")
    W.image(k, W.GRID_TO_IMAGE, g, img, torch.as_tensor(sw).cuda())
    ref = R.grid_to_image(plan, Gin, sw)
    got = img.double().cpu().numpy()
    q = n // 4
    inner = (slice(None), slice(q, n - q), slice(q, n - q))
    assert rel_max(got[inner], ref[inner]) <= tol
    # raw direction (no weight sum), whole image including the kappa-amplified edge
    g = torch.as_tensor(Gin).to(CDT[prec]).cuda()
    W.image(k, W.GRID_TO_IMAGE_RAW, g, img)
    ref = R.grid_to_image(plan, Gin, None)
    got = img.double().cpu().numpy()
    assert np.all(np.abs(got - ref) <= tol * 10 * np.abs(R.centred_idft(Gin)).max()
                  * np.outer(R.kappa(plan), R.kappa(plan))[None] + 1e-300)
    # image -> grid
    I = rng.standard_normal((2, n, n)).astype(np.float32 if prec != "f64" else np.float64)
    W.image(k, W.IMAGE_TO_GRID, g, torch.as_tensor(I).cuda())
    M = R.image_to_grid(plan, I.astype(np.float64))
    assert rel_max(g.to(torch.complex128).cpu().numpy(), M) <= tol
    k.free()


@pytest.mark.parametrize("prec,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_plain_degrid(prec, tol):
    wl = synth.cfg1w(n_w=9, s_max=10)
    params = {**wl.params, "precision": prec, "algorithm": "plain"}
    plan = R.Plan(params)
    tabs = R.kernel_tables(plan)
    rng = np.random.default_rng(4)
    n = plan.n
    M = rng.standard_normal((1, n, n)) + 1j * rng.standard_normal((1, n, n))
    M = M.astype(np.complex64 if prec != "f64" else np.complex128).astype(np.complex128)
    uvw, _, _ = planted(wl)
    k = W.make_kernels(params)
    out = torch.empty(uvw.shape[0], dtype=CDT[prec], device="cuda")
    W.degrid(k, torch.as_tensor(uvw).cuda(), torch.as_tensor(M).to(CDT[prec]).cuda(), out)
    ref = R.degrid(plan, tabs, uvw, M)
    got = out.to(torch.complex128).cpu().numpy()
    assert rel_max(got, ref) <= tol
    assert np.count_nonzero(got) == np.count_nonzero(ref)
    k.free()


def test_unit_point_source_images_to_delta_centre():
    wl = synth.cfg1()
    params = {**wl.params, "precision": "f64", "algorithm": "plain"}
    k = W.make_kernels(params)
    n = params["n"]
    ones = torch.ones(wl.nvis, dtype=torch.complex128, device="cuda")
    g = k.new_grid()
    sw = torch.zeros(1, dtype=torch.float64, device="cuda")
    W.grid(k, torch.as_tensor(wl.uvw).cuda(), ones, torch.as_tensor(wl.weight).cuda(), g,
           weight_sum=sw)
    img = torch.empty((1, n, n), dtype=torch.float64, device="cuda")
    W.image(k, W.GRID_TO_IMAGE, g, img, sw)
    assert abs(img[0, n // 2, n // 2].item() - 1.0) < 1e-12
    k.free()


@pytest.mark.parametrize("algo", ["tiled", "plain"])
def test_empty_image_is_zero_and_reported(algo):
    """An image that receives no gridded weight (every weight 0 here, or every row of
    image 1 flagged) comes out of GRID_TO_IMAGE as zeros, and wproj_check_weights reports
    WPROJ_EEMPTY for it; images with weight pass."""
    wl = synth.cfg1w(n_w=9, s_max=10)
    offs = np.array([0, 600, 1200, 2000])
    params = {**wl.params, "precision": "f32", "algorithm": algo, "n_images": 3}
    k = W.make_kernels(params)
    n = params["n"]
    wt = np.ones(len(wl.vis))
    wt[600:1200] = 0.0  # image 1: all flagged
    (u, v, w), _ = as_gpu_inputs(wl.uvw, wl.vis, wt, "f32")
    off = torch.as_tensor(offs, dtype=torch.int64).cuda()
    g = k.new_grid()
    sw = torch.zeros(3, dtype=torch.float64, device="cuda")
    W.grid(k, u, v, w, g, image_offsets=off, weight_sum=sw)
    img = torch.full((3, n, n), 7.0, dtype=torch.float32, device="cuda")
    W.image(k, W.GRID_TO_IMAGE, g, img, sw)
    with pytest.raises(W.WprojError) as ei:
        W.check_weights(k, sw)
    assert ei.value.code == -7 and "image 1" in str(ei.value)
    got = img.cpu().numpy()
    assert sw.cpu().tolist()[1] == 0.0
    assert not np.any(got[1])
    assert np.all(np.isfinite(got)) and np.abs(got[0]).max() > 0 and np.abs(got[2]).max() > 0
    # every image with weight: OK
    sw2 = torch.ones(3, dtype=torch.float64, device="cuda")
    W.check_weights(k, sw2)
    sw2[2] = float("nan")
    with pytest.raises(W.WprojError) as ei:
        W.check_weights(k, sw2)
    assert ei.value.code == -1
    k.free()
