"""The gridding step captured in a HIP graph and replayed.

Every launch of wproj_grid and wproj_image is stream-ordered and clears its counters
and queues with fill kernels (no memset nodes), so it can be captured once and
replayed.  Each replay runs after eager work that changes the inputs in place and is
checked against an eager run on the same inputs: gridding alone, then the whole step
(gridding, rocFFT inverse, correction) in one graph.  Record order inside a tile follows
the binning's atomic slot assignment, so FP32 grids of two runs agree to rounding
(~1e-7), not bit for bit; images are compared on the inner half, away from the edge
pixels where the grid correction kappa^2 (~1e6) amplifies that rounding.
"""

import numpy as np
import pytest
import torch

import paper_1905_03213_amd as W
import synth

from gpu_util import rel_max

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n_images", [1, 3])
def test_graph_replays_match_eager(n_images):
    wl = synth.small_tracks(n=256, cell=8e-5, n_chan=8, hours=2.0, dt_s=30.0)
    nv = wl.nvis
    offs = None
    if n_images > 1:
        offs = torch.as_tensor(np.linspace(0, nv, n_images + 1).astype(np.int64), device="cuda")
    k = W.make_kernels({**wl.params, "precision": "f32", "algorithm": "tiled", "n_images": n_images})
    n = wl.params["n"]
    uvw = wl.uvw.cuda()
    vis = wl.vis.to(torch.complex64).cuda()
    wt = wl.weight.float().cuda()
    ws = k.workspace(nv)
    g = k.new_grid()
    sw = torch.zeros(n_images, dtype=torch.float64, device="cuda")
    img = torch.empty((n_images, n, n), dtype=torch.float32, device="cuda")

    def grid_part():
        g.zero_()
        sw.zero_()
        W.grid(k, uvw, vis, wt, g, image_offsets=offs, weight_sum=sw, workspace=ws)

    def image_part():
        W.image(k, W.GRID_TO_IMAGE, g, img, sw, workspace=ws)

    def capture(fn):
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            fn()  # warm up on the capture stream
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            fn()
        torch.cuda.synchronize()
        return graph

    # 1) gridding alone in a graph
    gg = capture(grid_part)
    rng = np.random.default_rng(1)
    for rep in range(4):
        vis.mul_(float(rng.uniform(0.5, 2.0)))  # eager work between replays, in place
        wt.add_(0.125 * rep)
        torch.cuda.synchronize()
        gg.replay()
        torch.cuda.synchronize()
        got_g, got_sw = g.clone(), sw.clone()
        grid_part()
        torch.cuda.synchronize()
        assert torch.allclose(got_sw, sw, rtol=1e-12, atol=0)
        assert rel_max(got_g.to(torch.complex128).cpu().numpy(), g.to(torch.complex128).cpu().numpy()) <= 1e-6
    # 2) the whole step (gridding, FFT, correction) in one graph
    def step():
        grid_part()
        image_part()

    gs = capture(step)
    for rep in range(3):
        vis.mul_(float(rng.uniform(0.5, 2.0)))
        torch.cuda.synchronize()
        gs.replay()
        torch.cuda.synchronize()
        got_img = img.clone()
        step()
        torch.cuda.synchronize()
        q = n // 4
        assert rel_max(got_img[:, q:-q, q:-q].double().cpu().numpy(),
                       img[:, q:-q, q:-q].double().cpu().numpy()) <= 1e-5
    k.free()


def test_planned_step_replays_match_eager():
    """A kept plan's gridding plus imaging, captured once and replayed for new visibilities
    (the body of an imaging loop)."""
    wl = synth.small_tracks(n=256, cell=8e-5, n_chan=8, hours=2.0, dt_s=30.0)
    k = W.make_kernels({**wl.params, "precision": "f32", "algorithm": "tiled"})
    n = wl.params["n"]
    uvw = wl.uvw.cuda()
    vis = wl.vis.to(torch.complex64).cuda()
    wt = wl.weight.float().cuda()
    sw = torch.zeros(1, dtype=torch.float64, device="cuda")
    plan = W.Plan(k, uvw, wt, weight_sum=sw)
    ws = k.workspace(0)
    g = k.new_grid()
    img = torch.empty((1, n, n), dtype=torch.float32, device="cuda")

    def step():
        g.zero_()
        plan.grid(vis, g)
        W.image(k, W.GRID_TO_IMAGE, g, img, sw, workspace=ws)

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step()
    torch.cuda.synchronize()
    rng = np.random.default_rng(2)
    q = n // 4
    for rep in range(3):
        vis.mul_(float(rng.uniform(0.5, 2.0)))
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        got = img.clone()
        step()
        torch.cuda.synchronize()
        assert rel_max(got[:, q:-q, q:-q].double().cpu().numpy(),
                       img[:, q:-q, q:-q].double().cpu().numpy()) <= 1e-5
    plan.free()
    k.free()
