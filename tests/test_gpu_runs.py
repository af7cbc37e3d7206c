"""Register accumulation over runs of a shared footprint origin, and the channel-major
visibility order it is meant for, on the GPU against the oracle.

wproj_regroup_channels turns rows regrouped by baseline (Eqs. 5 and 6) into the order
baseline, channel, time (oracle/eq56.py: channel_major_order), bit for bit; gathers
apply it to uvw, visibilities and weights.  With accumulate_runs the FP32 fixed-support
gridders keep each lane's grid cell in a register while consecutive records of a work
item share the footprint origin: checked against the FP64 oracle on a track workload in
measurement-set order and in channel-major order (where most consecutive samples share
an origin), at one-, two- and four-pass supports, FP32 and FP16 tables, one-shot and
planned gridding."""

import numpy as np
import pytest
import torch

import paper_1905_03213_amd as W
import synth
from oracle import eq56
from oracle import wproj_ref as R

from gpu_util import oracle_grid, rel_max, run_grid

pytestmark = pytest.mark.gpu

TOL = {"f32": 1e-5, "f32_f16table": 1e-3}


def _oracle_vis_order(a1, a2, n_ant, n_chan):
    a1 = np.asarray(a1, dtype=np.int64)
    a2 = np.asarray(a2, dtype=np.int64)
    n_b = n_ant * (n_ant + 1) // 2
    ok = (a1 >= 0) & (a2 >= 0) & (a1 < n_ant) & (a2 < n_ant)
    b = np.full(a1.shape[0], n_b, dtype=np.int64)
    b[ok] = eq56.baseline_index(a1[ok], a2[ok], n_ant)
    perm = eq56.regroup_order(b, n_b + 1)
    return eq56.channel_major_order(perm, b, n_b + 1, n_chan)


def _device_vis_order(a1, a2, n_ant, n_chan):
    t1 = torch.as_tensor(np.asarray(a1, dtype=np.int32), device="cuda")
    t2 = torch.as_tensor(np.asarray(a2, dtype=np.int32), device="cuda")
    perm, start, counts = W.regroup_rows(t1, t2, n_ant)
    return W.regroup_channels(perm, start, counts, n_ant, n_chan)


@pytest.mark.parametrize("case", ["random_invalid", "track"])
def test_regroup_channels_matches_oracle(case):
    if case == "random_invalid":
        rng = np.random.default_rng(31)
        n_ant, n_chan = 10, 7
        a1 = rng.integers(-1, 11, 3000)
        a2 = rng.integers(0, 10, 3000)
    else:
        _, b1, b2 = synth.array_tracks(np.random.default_rng(2), hours=2.0, dt_s=10.0)
        n_t = 720
        a1, a2 = np.tile(b1, n_t), np.tile(b2, n_t)
        n_ant, n_chan = 27, 4
    got = _device_vis_order(a1, a2, n_ant, n_chan).cpu().numpy()
    assert np.array_equal(got, _oracle_vis_order(a1, a2, n_ant, n_chan))


def test_gather_small_and_wide_rows():
    """uvw rows (24 bytes), complex64 visibilities (8) and float32 weights (4) gathered by
    a visibility permutation, against torch indexing."""
    rng = np.random.default_rng(4)
    n = 50000
    perm = torch.as_tensor(rng.permutation(n), device="cuda")
    for t in (torch.randn(n, 3, dtype=torch.float64), torch.randn(n, dtype=torch.complex64),
              torch.rand(n, dtype=torch.float32)):
        src = t.cuda()
        assert torch.equal(W.gather_rows(perm, src), src[perm])


def _channel_major_tracks():
    """A 1 h track at 10 s on a 128^2 grid (4 channels), in measurement-set order and in
    baseline/channel/time order: uvw, vis, weight as host arrays."""
    wl = synth.small_tracks(hours=1.0, dt_s=10.0)
    src = wl.sources
    n_t, n_bl, n_ch = int(src["n_time"]), int(src["n_bl"]), int(src["n_chan"])
    a1, a2 = np.tile(src["ant1"], n_t), np.tile(src["ant2"], n_t)
    n_ant = int(max(a1.max(), a2.max())) + 1
    order = _oracle_vis_order(a1, a2, n_ant, n_ch)
    uvw, vis = wl.uvw.numpy(), wl.vis.numpy()
    wt = np.random.default_rng(5).uniform(0.5, 2.0, len(vis))
    return wl, (uvw, vis, wt), (uvw[order], vis[order], wt[order]), order


def _same_origin_fraction(params, uvw, wt):
    geo = R.snap(R.Plan(params), uvw, wt)
    v = geo["valid"]
    key = np.stack([geo["x0"], geo["y0"], geo["p"]], axis=1)
    same = (key[1:] == key[:-1]).all(axis=1) & v[1:] & v[:-1]
    return float(same.sum()) / max(int(v.sum()), 1)


@pytest.mark.parametrize("prec", ["f32", "f32_f16table"])
@pytest.mark.parametrize("support", [3, 8, 9, 16])
@pytest.mark.parametrize("order", ["ms", "channel_major"])
def test_run_accumulation_matches_oracle(order, support, prec):
    wl, ms, cm, _ = _channel_major_tracks()
    uvw, vis, wt = ms if order == "ms" else cm
    m = max(wl.params["kernel_image_size"], 2 * support)
    params = {**wl.params, "support": support, "kernel_image_size": m, "precision": prec,
              "algorithm": "tiled", "accumulate_runs": True}
    if order == "channel_major" and support == 8:
        # most consecutive samples of one baseline and channel share the origin
        frac = _same_origin_fraction(params, uvw, wt)
        print(f"[runs] same-origin fraction in channel-major order: {frac:.3f}", flush=True)
        assert frac > 0.5
    G, sw, cnt, host = run_grid(params, uvw, vis, wt)
    (Gr, swr, cr), _, _ = oracle_grid(params, host)
    assert cnt.tolist() == cr.tolist()
    assert np.allclose(sw, swr, rtol=1e-12, atol=0)
    assert rel_max(G, Gr) <= TOL[prec]


def test_run_accumulation_planned_and_unchanged_grid():
    """A plan on a run-accumulating handle grids like the oracle; the grid agrees with
    the same rows gridded without the mode to FP32 rounding (the binning order differs
    between calls, so the two agree to rounding, not bit for bit)."""
    wl, _, cm, _ = _channel_major_tracks()
    uvw, vis, wt = cm
    base = {**wl.params, "precision": "f32", "algorithm": "tiled"}
    grids = []
    for runs in (False, True):
        k = W.make_kernels({**base, "accumulate_runs": runs})
        u = torch.as_tensor(uvw).cuda()
        plan = W.Plan(k, u, torch.as_tensor(wt).to(torch.float32).cuda())
        v = torch.as_tensor(vis).to(torch.complex64).cuda()
        g = k.new_grid()
        plan.grid(v, g)
        torch.cuda.synchronize()
        grids.append(g.to(torch.complex128).cpu().numpy())
        plan.free()
        k.free()
    host = (uvw, torch.as_tensor(vis).to(torch.complex64).to(torch.complex128).numpy(),
            torch.as_tensor(wt).to(torch.float32).double().numpy())
    (Gr, _, _), _, _ = oracle_grid(base, host)
    assert rel_max(grids[1], Gr) <= TOL["f32"]
    assert rel_max(grids[1], grids[0]) <= TOL["f32"]


@pytest.mark.parametrize("prec", ["f32", "f32_f16table"])
@pytest.mark.parametrize("support", [3, 8, 9, 16])
def test_run_accumulation_is_bit_identical_with_stable_bins(support, prec):
    """With stable bins both handles see every bin's records in input order, so the
    register-accumulating gridder, which makes the same multiply-adds in the same order,
    gives the plain gridder's FP32 grid bit for bit (channel-major rows, where most
    consecutive records share their origin)."""
    wl, _, cm, _ = _channel_major_tracks()
    uvw, vis, wt = cm
    m = max(wl.params["kernel_image_size"], 2 * support)
    base = {**wl.params, "support": support, "kernel_image_size": m, "precision": prec,
            "algorithm": "tiled", "tile": 16, "chunk": 1024, "stable_bins": True}
    u = torch.as_tensor(uvw).cuda()
    v = torch.as_tensor(vis).to(torch.complex64).cuda()
    w = torch.as_tensor(wt).to(torch.float32).cuda()
    grids = []
    for runs in (False, True):
        k = W.make_kernels({**base, "accumulate_runs": runs})
        g = k.new_grid()
        W.grid(k, u, v, w, g)
        torch.cuda.synchronize()
        grids.append(g.clone())
        k.free()
    assert torch.equal(grids[0], grids[1])
