"""The largest grid the library accepts (n = 32768, 8.6 GB as complex64) against the
oracle, and sizes it must refuse.

Visibilities are spread over the whole uv plane, so that footprints touch the first and
last rows and columns and many fall off the grid; a few are placed exactly at the first
and last footprint positions that still fit.  The host cannot hold a dense FP64 oracle
grid of this size, so the oracle accumulates only the touched cells
(oracle.wproj_ref.grid_cells) and evaluates the image at sample pixels by a direct sum
(oracle.wproj_ref.image_pixels); the device grid is compared at every touched cell, and
its count of non-zero cells must equal the oracle's (no stray writes)."""

import ctypes

import numpy as np
import pytest
import torch

import paper_1905_03213_amd as W
from paper_1905_03213_amd import _lib
from oracle import wproj_ref as R

pytestmark = pytest.mark.gpu

N = 32768
PARAMS = dict(n=N, cell_rad=1e-6, n_wplanes=8, w_max=1000.0, support=8, oversample=8,
              kernel_image_size=32, n_images=1)


def _inputs():
    rng = np.random.default_rng(21)
    fov = N * PARAMS["cell_rad"]
    umax = (N / 2) / fov
    n_rand = 30_000
    u = rng.uniform(-umax, umax, n_rand)
    v = rng.uniform(-umax, umax, n_rand)
    w = rng.uniform(-1.1, 1.1, n_rand) * PARAMS["w_max"]
    # first and last on-grid footprints: q = S O/2 - O (x0 = 0) and q = (N - S) O + S O/2 - 1
    O, S = PARAMS["oversample"], PARAMS["support"]
    half = S * O // 2
    qs = np.array([half - O, half - O + 3, (N - S) * O + half - 1, (N - S) * O + half - 4])
    ge = (qs / O - N / 2) / fov
    eu, ev = np.meshgrid(ge, ge)
    edge = np.stack([eu.ravel(), ev.ravel(), np.zeros(eu.size)], axis=1)
    uvw = np.concatenate([np.stack([u, v, w], axis=1), edge])
    vis = rng.standard_normal(uvw.shape[0]) + 1j * rng.standard_normal(uvw.shape[0])
    return uvw, vis


@pytest.fixture(scope="module")
def oracle_cells():
    uvw, vis = _inputs()
    plan = R.Plan({**PARAMS, "precision": "f64"})
    tabs = R.kernel_tables(plan)
    cells, vals, sw, cnt = R.grid_cells(plan, tabs, uvw, vis, np.ones(uvw.shape[0]))
    geo = R.snap(plan, uvw, np.ones(uvw.shape[0]))
    v = geo["valid"]
    assert geo["x0"][v].min() == 0 and geo["y0"][v].min() == 0
    assert geo["x0"][v].max() == N - 8 and geo["y0"][v].max() == N - 8
    return plan, uvw, vis, cells, vals, sw, cnt


@pytest.mark.parametrize("prec,algo,tol", [("f32", "tiled", 1e-5), ("f64", "plain", 1e-12)])
def test_max_grid_size(oracle_cells, prec, algo, tol):
    plan, uvw, vis, cells, vals, sw_ref, cnt_ref = oracle_cells
    params = {**PARAMS, "precision": prec, "algorithm": algo}
    if algo == "tiled":
        params["tile"] = 32
    k = W.make_kernels(params)
    cd = torch.complex128 if prec == "f64" else torch.complex64
    rd = torch.float64 if prec == "f64" else torch.float32
    g = k.new_grid()
    sw = torch.zeros(1, dtype=torch.float64, device="cuda")
    cnt = torch.zeros(3, dtype=torch.int64, device="cuda")
    uvw_t = torch.as_tensor(uvw).cuda()
    vis_t = torch.as_tensor(vis).to(cd).cuda()
    wt_t = torch.ones(uvw.shape[0], dtype=rd, device="cuda")
    W.grid(k, uvw_t, vis_t, wt_t, g, weight_sum=sw, counters=cnt)
    torch.cuda.synchronize()
    assert cnt.cpu().tolist() == cnt_ref.tolist()
    assert sw.item() == sw_ref
    flat = g.view(-1)
    got = flat[torch.as_tensor(cells).cuda()].to(torch.complex128).cpu().numpy()
    scale = np.abs(vals).max()
    err = np.abs(got - vals).max() / scale
    print(f"[limits] n={N} {prec} {algo}: touched={cells.size} grid_max={err:.3e}", flush=True)
    assert err <= tol
    nz = int(torch.view_as_real(g).ne(0).any(dim=-1).sum().item())
    assert nz == cells.size
    if algo == "tiled":
        img = torch.empty((1, N, N), dtype=rd, device="cuda")
        ws = k.workspace(0)
        W.image(k, W.GRID_TO_IMAGE, g, img, sw, workspace=ws)
        torch.cuda.synchronize()
        rng = np.random.default_rng(3)
        ys = np.concatenate([[N // 2], rng.integers(N // 4, 3 * N // 4, 31)])
        xs = np.concatenate([[N // 2], rng.integers(N // 4, 3 * N // 4, 31)])
        ref = R.image_pixels(plan, cells, vals, sw_ref, ys, xs)
        got_px = img[0][torch.as_tensor(ys).cuda(), torch.as_tensor(xs).cuda()].double().cpu().numpy()
        e_img = np.abs(got_px - ref).max() / np.abs(ref).max()
        print(f"[limits] n={N} image at 32 pixels: max err {e_img:.3e}", flush=True)
        assert e_img <= tol
        del img, ws
    del g
    k.free()


def test_sizes_beyond_the_limits_are_refused():
    with pytest.raises(W.WprojError):
        W.make_kernels({**PARAMS, "n": 2 * N, "precision": "f32", "algorithm": "tiled"})
    # the tiled path takes at most 2^32 - 2 visibilities per call (32-bit record offsets);
    # the check runs before any pointer is used
    k = W.make_kernels({**PARAMS, "n": 256, "cell_rad": 1e-4, "precision": "f32",
                        "algorithm": "tiled"})
    L = _lib.lib()
    fake = ctypes.c_void_p(256)
    huge = 1 << 32
    rc = L.wproj_grid(k.handle, huge, fake, fake, fake, None, fake, None, None, fake, 1 << 62, None)
    assert rc == -1 and b"2^32" in L.wproj_last_error()
    k.free()
