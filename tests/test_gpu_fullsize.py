"""Parity at the benchmark's full sizes, in the launch configuration bench.py times.

The plain C oracle (FP64, OpenMP per-thread grids) computes the complete grid on the
host in seconds, so these compare every cell and every pixel, not a sample:
  cfg2  2048^2, 6.47e7 visibilities, S=8, 128 planes: FP32 tiled (the bench path) and
        FP64 plain (the comparison path)
  cfg4  64 images of 1024^2, ~4e7 visibilities, S=8, 64 planes: FP32 tiled
  cfg3  4096^2, 5.05e7 visibilities, supports 4..16, 256 planes: FP16 tables, FP32 tiled
  cfg5  2048^2 model -> 1.01e7 predicted visibilities: FP32 degridding
Image errors are max and RMS |GPU - oracle| / max|oracle| over the inner half (the
edge correction amplifies rounding by up to ~1e6 there) and over the whole uncorrected
image.
"""

import os

import numpy as np
import pytest
import torch

import paper_1905_03213_amd as W
import synth
from oracle import cref
from oracle import wproj_ref as R

from gpu_util import grad_bound, rel_max, rel_rms

pytestmark = pytest.mark.gpu

THREADS = max(1, min(16, len(os.sched_getaffinity(0))))


def _gpu_grid(wl, prec, algo):
    k = W.make_kernels({**wl.params, "precision": prec, "algorithm": algo})
    cd = torch.complex128 if prec == "f64" else torch.complex64
    rd = torch.float64 if prec == "f64" else torch.float32
    vis = wl.vis.to(cd)
    wt = wl.weight.to(rd)
    if algo == "tiled":
        # the tile and chunk bench.py would time on this data
        tile, chunk = W.autotune(k, wl.uvw, vis, wt, image_offsets=wl.image_offsets)
        print(f"[fullsize] autotuned tile {tile}, chunk {chunk}", flush=True)
    g = k.new_grid()
    ni = wl.params.get("n_images", 1)
    sw = torch.zeros(ni, dtype=torch.float64, device="cuda")
    cnt = torch.zeros(3, dtype=torch.int64, device="cuda")
    W.grid(k, wl.uvw, vis, wt, g, image_offsets=wl.image_offsets, weight_sum=sw, counters=cnt)
    torch.cuda.synchronize()
    return k, g, sw, cnt, vis.to(torch.complex128).cpu().numpy(), wt.double().cpu().numpy()


def _report(name, **kv):
    print(f"[fullsize] {name}: " + ", ".join(f"{k}={v:.3e}" if isinstance(v, float) else f"{k}={v}"
                                             for k, v in kv.items()), flush=True)


def _image_errors(plan, G, Gr, sw):
    n = plan.n
    q = n // 4
    img = R.grid_to_image(plan, G, sw)
    ref = R.grid_to_image(plan, Gr, sw)
    inner = (slice(None), slice(q, n - q), slice(q, n - q))
    raw = R.centred_idft(G).real / sw.reshape(-1, 1, 1)
    rawr = R.centred_idft(Gr).real / sw.reshape(-1, 1, 1)
    return (rel_max(img[inner], ref[inner]), rel_rms(img[inner], ref[inner]),
            rel_max(raw, rawr), rel_rms(raw, rawr))


@pytest.mark.parametrize("prec,algo,tol", [("f32", "tiled", 1e-5), ("f64", "plain", 1e-12)])
def test_cfg2_full(prec, algo, tol):
    wl = synth.cfg2(device="cuda")
    k, g, sw, cnt, vis_h, wt_h = _gpu_grid(wl, prec, algo)
    plan = R.Plan({**wl.params, "precision": "f64"})
    tabs = R.kernel_tables(plan)
    Gr, swr, cr = cref.grid(plan, tabs, wl.uvw.cpu().numpy(), vis_h, wt_h, nthreads=THREADS)
    G = g.to(torch.complex128).cpu().numpy()
    assert cnt.cpu().tolist() == cr.tolist()
    assert abs(sw.item() - swr[0]) <= 1e-9 * swr[0]
    gmax = rel_max(G, Gr)
    emax, erms, rmax, rrms = _image_errors(plan, G, Gr, swr)
    _report(f"cfg2 {prec} {algo}", grid_max=gmax, img_max=emax, img_rms=erms,
            raw_max=rmax, raw_rms=rrms, nvis=wl.nvis, gridded=int(swr[0]))
    assert emax <= tol and rmax <= tol
    if prec == "f64":
        assert gmax <= tol
    # the image the library itself produces (rocFFT + correction) on this grid
    img = torch.empty((1, plan.n, plan.n), dtype=k.real, device="cuda")
    W.image(k, W.GRID_TO_IMAGE, g, img, sw)
    got = img.double().cpu().numpy()
    ref = R.grid_to_image(plan, Gr, swr)
    q = plan.n // 4
    e_lib = rel_max(got[:, q:-q, q:-q], ref[:, q:-q, q:-q])
    _report(f"cfg2 {prec} {algo} library image", img_max=e_lib)
    assert e_lib <= (1e-12 if prec == "f64" else 2e-5)
    k.free()


def test_cfg4_full_batched():
    wl = synth.cfg4(device="cuda")
    k, g, sw, cnt, vis_h, wt_h = _gpu_grid(wl, "f32", "tiled")
    plan = R.Plan({**wl.params, "precision": "f64"})
    tabs = R.kernel_tables(plan)
    offs = wl.image_offsets.cpu().numpy()
    Gr, swr, cr = cref.grid(plan, tabs, wl.uvw.cpu().numpy(), vis_h, wt_h, offs,
                            nthreads=THREADS)
    G = g.to(torch.complex128).cpu().numpy()
    assert cnt.cpu().tolist() == cr.tolist()
    assert np.allclose(sw.cpu().numpy(), swr, rtol=1e-9, atol=0)
    worst = 0.0
    for i in range(0, plan.n_images, 8):  # transforms in slices to bound host memory
        sl = slice(i, i + 8)
        e = _image_errors(plan, G[sl], Gr[sl], swr[sl])
        worst = max(worst, e[0], e[2])
    _report("cfg4 f32 tiled", grid_max=rel_max(G, Gr), img_max_worst=worst, nvis=wl.nvis)
    assert worst <= 1e-5
    k.free()


def test_cfg3_full_fp16_tables_variable_support():
    wl = synth.cfg3(device="cuda")
    k, g, sw, cnt, vis_h, wt_h = _gpu_grid(wl, "f32_f16table", "tiled")
    plan = R.Plan({**wl.params, "precision": "f64"})
    tabs = R.kernel_tables(plan)
    Gr, swr, cr = cref.grid(plan, tabs, wl.uvw.cpu().numpy(), vis_h, wt_h, nthreads=THREADS)
    G = g.to(torch.complex128).cpu().numpy()
    del g
    assert cnt.cpu().tolist() == cr.tolist()
    emax, erms, rmax, rrms = _image_errors(plan, G, Gr, swr)
    _report("cfg3 f16-table tiled", grid_max=rel_max(G, Gr), img_max=emax, img_rms=erms,
            raw_max=rmax, raw_rms=rrms, nvis=wl.nvis)
    assert emax <= 1e-3 and rmax <= 1e-3
    k.free()


def test_cfg5_full_degrid():
    wl = synth.cfg5(device="cuda")
    n = wl.params["n"]
    model = synth.cfg5_model_image(n)
    plan = R.Plan({**wl.params, "precision": "f64"})
    tabs = R.kernel_tables(plan)
    k = W.make_kernels({**wl.params, "precision": "f32", "algorithm": "tiled"})
    img = torch.as_tensor(model, dtype=torch.float32, device="cuda")[None]
    g = k.new_grid()
    W.image(k, W.IMAGE_TO_GRID, g, img)
    out = torch.empty(wl.nvis, dtype=torch.complex64, device="cuda")
    W.degrid(k, wl.uvw, g, out)
    torch.cuda.synchronize()
    M = R.image_to_grid(plan, model.astype(np.float32).astype(np.float64)[None])
    ref = cref.degrid(plan, tabs, wl.uvw.cpu().numpy(), M, nthreads=THREADS)
    got = out.to(torch.complex128).cpu().numpy()
    e = rel_max(got, ref)
    _report("cfg5 f32 degrid", vis_max=e, vis_rms=rel_rms(got, ref), nvis=wl.nvis)
    assert e <= 1e-5
    k.free()


def test_cfg5_full_chi2_gradient():
    """chi^2 gradient of the 2048^2 FP32 model over 1.01e7 visibilities against the
    oracle's adjoint (O9: -2 kappa kappa Re IDFT(grid(W r)), with the C oracle for the
    gridding and degridding), at I = 0 and at a perturbed image, plus central differences
    through the GPU path (chi^2 is quadratic in I, so they carry no truncation error)."""
    from paper_1905_03213_amd.autograd import chi2

    wl = synth.cfg5(device="cuda")
    n = wl.params["n"]
    q = n // 4
    inner = (slice(q, n - q), slice(q, n - q))
    plan = R.Plan({**wl.params, "precision": "f64"})
    tabs = R.kernel_tables(plan)
    uvw_h = wl.uvw.cpu().numpy()
    truth = synth.cfg5_model_image(n)
    rng = np.random.default_rng(55)
    v_true = cref.degrid(plan, tabs, uvw_h, R.image_to_grid(plan, truth[None]), nthreads=THREADS)
    Vo = torch.as_tensor(v_true, device="cuda") + wl.vis  # plus the workload's noise (sigma 0.01)
    Vo = Vo.to(torch.complex64)
    Wt = torch.as_tensor(rng.uniform(0.5, 2.0, wl.nvis), dtype=torch.float32, device="cuda")
    vo_h = Vo.to(torch.complex128).cpu().numpy()
    wt_h = Wt.double().cpu().numpy()
    k = W.make_kernels({**wl.params, "precision": "f32", "algorithm": "tiled"})
    U = wl.uvw
    kap = R.kappa(plan)
    for name, img0 in (("zero", np.zeros((n, n))), ("perturbed", 0.9 * truth)):
        img32 = img0.astype(np.float32)
        I = torch.tensor(img32, device="cuda", requires_grad=True)
        loss = chi2(I, k, U, Vo, Wt)
        loss.backward()
        got = I.grad.double().cpu().numpy()
        # oracle: r = V_obs - A(I) in FP64 from the same FP32 image and FP32-rounded V_obs
        a_ref = cref.degrid(plan, tabs, uvw_h, R.image_to_grid(plan, img32.astype(np.float64)[None]),
                            nthreads=THREADS)
        r = vo_h - a_ref
        G, _, _ = cref.grid(plan, tabs, uvw_h, r, wt_h, nthreads=THREADS)
        ref = -2.0 * R.grid_to_image(plan, G, None)[0]
        del G
        with torch.no_grad():
            from paper_1905_03213_amd.autograd import predict
            a_gpu = predict(I, k, U).to(torch.complex128).cpu().numpy()
        d_rms = float(np.sqrt(np.mean(np.abs(a_gpu - a_ref) ** 2)))
        r_rms = float(np.sqrt(np.mean(np.abs(r) ** 2)))
        bound = grad_bound(d_rms, r_rms, 1e-5)
        e_max = rel_max(got[inner], ref[inner])
        e_rms = rel_rms(got[inner], ref[inner])
        _report(f"cfg5 chi2 gradient at {name}", grad_max=e_max, grad_rms=e_rms, bound=bound,
                pred_err_rms=d_rms, resid_rms=r_rms, nvis=wl.nvis)
        assert e_max <= bound, (e_max, bound)
        assert abs(loss.item() - float(np.sum(wt_h * np.abs(r) ** 2))) <= 1e-4 * loss.item()
        # central differences at a few inner pixels: chi^2(I +- h e) computed by the GPU path.
        # Each chi^2 carries the FP32 prediction error: |d chi^2| <= 2 sqrt(sum W^2 |r|^2) rms|dA|
        # (a sum of 1e7 independent terms) with r the residual at I +- h e, 4 sigma margin.
        h = 1.0
        for _ in range(3):
            y, x = (int(v) for v in rng.integers(q, n - q, 2))
            e = torch.zeros((n, n), dtype=torch.float32, device="cuda")
            e[y, x] = h
            with torch.no_grad():
                fp = chi2(I + e, k, U, Vo, Wt).item()
                fm = chi2(I - e, k, U, Vo, Wt).item()
            fd = (fp - fm) / (2 * h)
            # |A(h e)| per row is about h kappa(x) kappa(y) (taps normalised to sum 1)
            hk = h * kap[x] * kap[y]
            r_h = np.sqrt(np.sum(wt_h ** 2 * (np.abs(r) ** 2 + hk * hk)))
            tol = 4.0 * 2.0 * r_h * d_rms * 2.0 / (2 * h) + bound * np.abs(ref[inner]).max()
            _report(f"cfg5 fd at {name} ({y},{x})", fd=fd, grad=float(got[y, x]), tol=float(tol))
            assert abs(fd - got[y, x]) <= tol
        I.grad = None
    k.free()
