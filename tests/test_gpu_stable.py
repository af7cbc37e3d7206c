"""Stable binning (stable_bins = 1) and the binned order a plan keeps (wproj_plan_rows).

The paper's regroup is a counting sort that keeps each baseline's rows in time order
(Eq. 5 and 6); the library's binning is the same pattern keyed by (image, uv-tile,
w-plane).  These tests pin the binned order itself against the oracle's footprints:
  * with stable bins, the rows of a plan in bin order are exactly a stable argsort of
    the oracle's bin keys (bit-exact index check), across one to three radix passes;
  * with count atomics, every bin holds exactly the oracle's rows (its order is free);
and then the consequences: gridding and degridding with stable bins against the FP64
oracle, and FP32 grids that are identical bit for bit from run to run, under a HIP graph
replay, and after any reordering of the input that keeps each bin's rows in order.
"""

import numpy as np
import pytest
import torch

import paper_1905_03213_amd as W
import synth
from oracle import wproj_ref as R

from gpu_util import oracle_grid, planted, rel_max, run_grid

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5, "f32_f16table": 1e-3}


def _crowded():
    """~12k visibilities over 2048^2 cells in 16-cell tiles and 64 planes: 2^20 bins, so
    the keys need three 8-bit radix passes."""
    rng = np.random.default_rng(21)
    n, cell = 2048, 1e-5
    params = dict(n=n, cell_rad=cell, n_wplanes=64, w_max=500.0, support=8, oversample=8,
                  kernel_image_size=32, n_images=1, algorithm="tiled", tile=16, chunk=1024)
    nvis = 3 * 4096 + 123
    umax = (n / 2 - 8) / (n * cell)
    uvw = np.stack([rng.uniform(-umax, umax, nvis), rng.uniform(-umax, umax, nvis),
                    rng.uniform(-500.0, 500.0, nvis)], axis=1)
    vis = rng.standard_normal(nvis) + 1j * rng.standard_normal(nvis)
    wt = rng.uniform(0.5, 1.5, nvis)
    return params, uvw, vis, wt, None


def _case(which):
    """(params without precision, uvw, vis, weight, image offsets)"""
    offs = None
    extra = {"tile": 16, "chunk": 256}
    if which == "crowded":
        return _crowded()
    if which == "tracks":
        wl = synth.small_tracks()
    elif which == "variable_support":
        wl = synth.cfg1w(n_w=9, s_max=10)  # per-plane supports: records recomputed, not compact
    elif which == "multi_image":
        wl = synth.cfg1w(n_w=9, s_max=10)
        offs = np.array([100, 700, 700, 1500, 1900])
        extra["n_images"] = 4
    else:  # fold
        wl = synth.small_tracks()
        extra["w_mode"] = "fold"
    uvw, vis, wt = planted(wl)
    return {**wl.params, **extra, "algorithm": "tiled"}, uvw, vis, wt, offs


def _bin_keys(params, uvw, wt, offs):
    """Each row's bin key from the oracle's footprints, in the library's key order:
    ((image, tile row, tile column), w-plane); int64 max for rows not gridded."""
    plan = R.Plan(params)
    g = R.snap(plan, uvw, wt)
    n, tile = params["n"], params["tile"]
    nt = (n + tile - 1) // tile
    ni = params.get("n_images", 1)
    assert ni * nt * nt * plan.n_w <= 1 << 25  # planes are binned apart at this size
    rows = np.arange(uvw.shape[0])
    if offs is None:
        img = np.zeros(rows.shape, dtype=np.int64)
        inside = np.ones(rows.shape, dtype=bool)
    else:
        offs = np.asarray(offs)
        img = np.searchsorted(offs, rows, side="right") - 1
        inside = (rows >= offs[0]) & (rows < offs[-1])
        img = np.clip(img, 0, ni - 1)
    key = ((img * nt + g["y0"] // tile) * nt + g["x0"] // tile) * plan.n_w + g["p"]
    return np.where(g["valid"] & inside, key, np.iinfo(np.int64).max)


def _plan_rows(params, uvw, wt, offs):
    k = W.make_kernels(params)
    u = torch.as_tensor(uvw).cuda()
    w = torch.as_tensor(wt).to(k.real).cuda()
    off = None if offs is None else torch.as_tensor(offs, dtype=torch.int64).cuda()
    p = W.Plan(k, u, w, image_offsets=off)
    rows = p.rows()
    torch.cuda.synchronize()
    out = rows.cpu().numpy().astype(np.int64) & 0xFFFFFFFF
    p.free()
    k.free()
    return out


@pytest.mark.parametrize("agg", [False, True])
@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("which", ["tracks", "variable_support", "multi_image", "fold", "crowded"])
def test_stable_bins_keep_input_order(which, prec, agg):
    """Either key pass (per-wavefront runs, or counts aggregated per block) feeds the
    stable sort the same keys."""
    params, uvw, vis, wt, offs = _case(which)
    params = {**params, "precision": prec, "stable_bins": True, "bin_aggregate": agg}
    key = _bin_keys(params, uvw, wt, offs)
    n_in = int((key != np.iinfo(np.int64).max).sum())
    want = np.argsort(key, kind="stable")[:n_in]
    rows = _plan_rows(params, uvw, wt, offs)
    assert np.array_equal(rows[:n_in], want)
    assert (rows[n_in:] == 0xFFFFFFFF).all()


@pytest.mark.parametrize("agg", [False, True])
@pytest.mark.parametrize("which", ["tracks", "variable_support", "multi_image", "crowded"])
def test_atomic_bins_hold_the_oracle_rows(which, agg):
    params, uvw, vis, wt, offs = _case(which)
    params = {**params, "precision": "f32", "bin_aggregate": agg}
    key = _bin_keys(params, uvw, wt, offs)
    n_in = int((key != np.iinfo(np.int64).max).sum())
    rows = _plan_rows(params, uvw, wt, offs)
    got = rows[:n_in]
    assert (rows[n_in:] == 0xFFFFFFFF).all()
    # bins in key order, each holding exactly its rows (in any order)
    assert np.all(np.diff(key[got]) >= 0)
    assert np.array_equal(np.sort(got), np.sort(np.argsort(key, kind="stable")[:n_in]))


@pytest.mark.parametrize("prec", ["f64", "f32", "f32_f16table"])
@pytest.mark.parametrize("which", ["tracks", "variable_support", "multi_image", "fold", "crowded"])
def test_stable_grid_matches_oracle(which, prec):
    params, uvw, vis, wt, offs = _case(which)
    params = {**params, "precision": prec, "stable_bins": True}
    G, sw, cnt, host = run_grid(params, uvw, vis, wt, offs)
    (Gr, swr, cr), _, _ = oracle_grid(params, host, offs)
    assert cnt.tolist() == cr.tolist()
    assert np.allclose(sw, swr, rtol=1e-12, atol=0)
    assert rel_max(G, Gr) <= TOL[prec]


def test_stable_degrid_matches_oracle():
    params, uvw, _, _, _ = _case("tracks")
    params = {**params, "precision": "f32", "stable_bins": True}
    plan = R.Plan(params)
    tabs = R.kernel_tables(plan)
    rng = np.random.default_rng(9)
    M = rng.standard_normal((1, plan.n, plan.n)) + 1j * rng.standard_normal((1, plan.n, plan.n))
    k = W.make_kernels(params)
    u = torch.as_tensor(uvw).cuda()
    out = torch.empty(u.shape[0], dtype=torch.complex64, device="cuda")
    W.degrid(k, u, torch.as_tensor(M.astype(np.complex64)).cuda(), out)
    torch.cuda.synchronize()
    ref = R.degrid(plan, tabs, uvw, M)
    assert rel_max(out.to(torch.complex128).cpu().numpy(), ref) <= TOL["f32"]
    k.free()


def test_stable_fp32_grid_is_reproducible_bit_for_bit():
    """Two runs, a HIP graph replay and an input reordered bin by bin (each bin's rows
    kept in their order) give the same FP32 grid to the last bit."""
    params, uvw, vis, wt, _ = _case("tracks")
    params = {**params, "precision": "f32", "stable_bins": True}
    k = W.make_kernels(params)
    u = torch.as_tensor(uvw).cuda()
    v = torch.as_tensor(vis.astype(np.complex64)).cuda()
    w = torch.as_tensor(wt.astype(np.float32)).cuda()
    ws = k.workspace(u.shape[0])
    g = k.new_grid()

    def once(uu, vv, ww):
        g.zero_()
        W.grid(k, uu, vv, ww, g, workspace=ws)

    once(u, v, w)
    torch.cuda.synchronize()
    first = g.clone()
    once(u, v, w)
    torch.cuda.synchronize()
    assert torch.equal(g, first)
    # rows grouped bin by bin, each bin's rows in their input order
    key = _bin_keys(params, uvw, wt, None)
    perm = torch.as_tensor(np.argsort(key, kind="stable")).cuda()
    once(u[perm].contiguous(), v[perm].contiguous(), w[perm].contiguous())
    torch.cuda.synchronize()
    assert torch.equal(g, first)
    # captured once, replayed after eager work
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        once(u, v, w)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        once(u, v, w)
    torch.cuda.synchronize()
    for _ in range(3):
        g.fill_(1.0)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(g, first)
    # against the oracle as well
    (Gr, _, _), _, _ = oracle_grid(params, (uvw, v.to(torch.complex128).cpu().numpy(),
                                            w.to(torch.float64).cpu().numpy()))
    assert rel_max(first.to(torch.complex128).cpu().numpy(), Gr) <= TOL["f32"]
    k.free()


@pytest.mark.parametrize("n", [1, 7, 4095, 4096, 4097])
@pytest.mark.parametrize("flagged", [False, True])
def test_stable_bins_edge_sizes(n, flagged):
    """One radix block exactly, one row more or less, a single row, and inputs where no
    row is gridded (every weight 0): the binned order is still the oracle's."""
    params, uvw, vis, wt, _ = _crowded()
    params = {**params, "precision": "f32", "stable_bins": True}
    uvw, vis, wt = uvw[:n].copy(), vis[:n].copy(), wt[:n].copy()
    if flagged:
        wt[:] = 0.0
    key = _bin_keys(params, uvw, wt, None)
    n_in = int((key != np.iinfo(np.int64).max).sum())
    assert n_in == (0 if flagged else n)
    rows = _plan_rows(params, uvw, wt, None)
    assert np.array_equal(rows[:n_in], np.argsort(key, kind="stable")[:n_in])
    assert (rows[n_in:] == 0xFFFFFFFF).all()
    G, sw, cnt, host = run_grid(params, uvw, vis, wt)
    if flagged:
        assert not np.any(G) and sw[0] == 0.0
    else:
        (Gr, _, _), _, _ = oracle_grid(params, host)
        assert rel_max(G, Gr) <= TOL["f32"]
