"""GPU parity of the binned (tiled) gridder against the FP64 oracle, through the C ABI.

Covers fixed and per-plane supports, every precision, tile sizes 16/32/64 (results must
not depend on the tile), several images per call, and a hot tile that is split into
several work items.
"""

import numpy as np
import pytest

import synth

from gpu_util import oracle_grid, planted, rel_max, run_grid

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5, "f32_f16table": 1e-3}


def _check(params, uvw, vis, wt, offs=None):
    G, sw, cnt, host = run_grid(params, uvw, vis, wt, offs)
    (Gr, swr, cr), _, _ = oracle_grid(params, host, offs)
    err = rel_max(G, Gr)
    assert err <= TOL[params["precision"]], err
    assert np.allclose(sw, swr, rtol=1e-12, atol=0)
    assert cnt.tolist() == cr.tolist()
    return G, err


@pytest.mark.parametrize("prec", ["f64", "f32", "f32_f16table"])
@pytest.mark.parametrize("which", ["cfg1", "cfg1w", "tracks"])
def test_tiled_grid_matches_oracle(prec, which):
    if which == "cfg1":
        wl = synth.cfg1()
    elif which == "cfg1w":
        wl = synth.cfg1w()
    else:
        wl = synth.small_tracks()
        wl.uvw, wl.vis, wl.weight = wl.uvw.numpy(), wl.vis.numpy(), wl.weight.numpy()
    uvw, vis, wt = planted(wl)
    _check({**wl.params, "precision": prec, "algorithm": "tiled"}, uvw, vis, wt)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_tile_size_invariance(prec):
    wl = synth.cfg1()
    outs = []
    for tile in (16, 32, 64):
        G, _ = _check({**wl.params, "precision": prec, "algorithm": "tiled", "tile": tile},
                      wl.uvw, wl.vis, wl.weight)
        outs.append(G)
    tol = TOL[prec]
    for G in outs[1:]:
        assert rel_max(G, outs[0]) <= tol


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_tiled_multi_image(prec):
    wl = synth.cfg1w(n_w=9, s_max=10)
    offs = np.array([100, 700, 700, 1500, 1900])
    params = {**wl.params, "precision": prec, "algorithm": "tiled", "n_images": 4}
    G, _ = _check(params, wl.uvw, wl.vis, wl.weight, offs)
    assert np.abs(G[1]).max() == 0.0


@pytest.mark.parametrize("prec,chunk", [("f64", 0), ("f32", 0), ("f32", 1024), ("f32", 16384)])
def test_hot_tile_split_into_chunks(prec, chunk):
    # 30000 visibilities inside one 64-cell tile: several work items of different sizes
    # (30 of 1024 records down to one full and one partial item of 16384) accumulate the
    # same cells, handed out largest first.
    rng = np.random.default_rng(12)
    wl = synth.cfg1(n_vis=30000)
    fov = wl.params["n"] * wl.params["cell_rad"]
    r = 20.0 * np.sqrt(rng.random(30000)) / fov
    th = 2 * np.pi * rng.random(30000)
    uvw = np.stack([r * np.cos(th) + 30.0 / fov, r * np.sin(th) + 30.0 / fov,
                    rng.uniform(-500, 500, 30000)], axis=1)
    _check({**wl.params, "precision": prec, "algorithm": "tiled", "chunk": chunk}, uvw, wl.vis, wl.weight)


def test_autotune_picks_a_candidate_and_keeps_parity():
    import paper_1905_03213_amd as W
    import torch

    wl = synth.small_tracks(n=256, cell=8e-5, n_chan=8, hours=2.0, dt_s=30.0)
    params = {**wl.params, "precision": "f32", "algorithm": "tiled"}
    k = W.make_kernels(params)
    uvw = wl.uvw.cuda()
    vis = wl.vis.to(torch.complex64).cuda()
    wt = wl.weight.float().cuda()
    tile, chunk = W.autotune(k, uvw, vis, wt)
    assert tile in (16, 32) and chunk in (1024, 2048, 4096, 8192, 16384)
    # a second handle of the same shape reuses the cached choice
    k2 = W.make_kernels(params)
    assert W.autotune(k2, uvw, vis, wt) == (tile, chunk)
    G, sw, cnt, host = run_grid(params, wl.uvw.numpy(), wl.vis.numpy(), wl.weight.numpy(), k=k)
    (Gr, swr, cr), _, _ = oracle_grid(params, host)
    assert rel_max(G, Gr) <= TOL["f32"]
    k.free()
    k2.free()


@pytest.mark.parametrize("prec", ["f64", "f32", "f32_f16table"])
@pytest.mark.parametrize("which", ["cfg1w", "tracks"])
def test_tiled_degrid_matches_oracle(prec, which):
    import torch

    import paper_1905_03213_amd as W
    from oracle import wproj_ref as R

    if which == "cfg1w":
        wl = synth.cfg1w(n_w=9, s_max=10)
    else:
        wl = synth.small_tracks()
        wl.uvw, wl.vis, wl.weight = wl.uvw.numpy(), wl.vis.numpy(), wl.weight.numpy()
    uvw, _, _ = planted(wl)
    params = {**wl.params, "precision": prec, "algorithm": "tiled"}
    plan = R.Plan(params)
    tabs = R.kernel_tables(plan)
    rng = np.random.default_rng(4)
    n = plan.n
    cd = torch.complex128 if prec == "f64" else torch.complex64
    M = rng.standard_normal((1, n, n)) + 1j * rng.standard_normal((1, n, n))
    M = M.astype(np.complex128 if prec == "f64" else np.complex64).astype(np.complex128)
    k = W.make_kernels(params)
    out = torch.full((uvw.shape[0],), 7.0 + 7.0j, dtype=cd, device="cuda")
    W.degrid(k, torch.as_tensor(uvw).cuda(), torch.as_tensor(M).to(cd).cuda(), out)
    ref = R.degrid(plan, tabs, uvw, M)
    got = out.to(torch.complex128).cpu().numpy()
    assert rel_max(got, ref) <= TOL[prec]
    assert np.count_nonzero(got) == np.count_nonzero(ref)  # dropped rows come back as 0
    k.free()


def test_tiled_degrid_multi_image():
    import torch

    import paper_1905_03213_amd as W
    from oracle import wproj_ref as R

    wl = synth.cfg1w(n_w=9, s_max=10)
    offs = np.array([100, 700, 700, 1500, 1900])
    params = {**wl.params, "precision": "f64", "algorithm": "tiled", "n_images": 4}
    plan = R.Plan(params)
    tabs = R.kernel_tables(R.Plan({**params, "n_images": 1}))
    rng = np.random.default_rng(5)
    M = rng.standard_normal((4, plan.n, plan.n)) + 1j * rng.standard_normal((4, plan.n, plan.n))
    k = W.make_kernels(params)
    out = torch.empty(wl.nvis, dtype=torch.complex128, device="cuda")
    W.degrid(k, torch.as_tensor(wl.uvw).cuda(), torch.as_tensor(M).cuda(), out,
             image_offsets=torch.as_tensor(offs).cuda())
    ref = R.degrid(plan, tabs, wl.uvw, M, offs)
    assert rel_max(out.cpu().numpy(), ref) <= 1e-12
    k.free()
