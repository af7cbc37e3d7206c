"""GPU checks of wproj_grid_noalloc (gridding with the library's fixed per-GPU scratch
array instead of a caller workspace) against wproj_grid, through the C ABI: two calls
in a row, the second on a smaller input, so the second runs on scratch memory that
still holds the first call's contents."""

import ctypes

import numpy as np
import pytest
import torch

import paper_1905_03213_amd as W
import synth
from paper_1905_03213_amd import _lib

from gpu_util import as_gpu_inputs, planted, rel_max

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5, "f32_f16table": 1e-3}


def _both(k, ni, u, v, w, off=None):
    """(grid, weight sums, counters) from wproj_grid and from wproj_grid_noalloc."""
    out = []
    for fn in (W.grid, W.grid_noalloc):
        g = k.new_grid()
        sw = torch.zeros(ni, dtype=torch.float64, device="cuda")
        cnt = torch.zeros(3, dtype=torch.int64, device="cuda")
        fn(k, u, v, w, g, image_offsets=off, weight_sum=sw, counters=cnt)
        torch.cuda.synchronize()
        out.append((g.to(torch.complex128).cpu().numpy(), sw.cpu().numpy(), cnt.cpu().numpy()))
    return out


@pytest.mark.parametrize("prec", ["f64", "f32", "f32_f16table"])
def test_noalloc_matches_grid_two_calls(prec):
    wl = synth.cfg1()
    uvw, vis, wt = planted(wl)
    params = {**wl.params, "precision": prec, "algorithm": "tiled"}
    k = W.make_kernels(params)
    assert k.workspace_size(len(wt)) <= W.noalloc_scratch_bytes()
    for n_rows in (len(wt), len(wt) // 3):  # second call smaller than the first
        (u, v, w), _ = as_gpu_inputs(uvw[:n_rows], vis[:n_rows], wt[:n_rows], prec)
        (G, sw, c), (Gn, swn, cn) = _both(k, 1, u, v, w)
        print(f"noalloc {prec} rows {n_rows}: rel max {rel_max(Gn, G):.2e}", flush=True)
        assert rel_max(Gn, G) <= TOL[prec]
        assert np.allclose(swn, sw, rtol=1e-12, atol=0)
        assert cn.tolist() == c.tolist()
    k.free()


def test_noalloc_multi_image_fixed_support():
    """Several images in one call and the fixed-support packed-record path."""
    wl = synth.cfg1w(n_w=9, s_max=8)
    params = {**wl.params, "precision": "f32", "algorithm": "tiled", "n_images": 4,
              "support_per_plane": None, "support": 8}
    k = W.make_kernels(params)
    uvw, vis, wt = planted(wl)
    for offs in ([0, 500, 900, 1500, 2000], [100, 200, 200, 500, 600]):
        (u, v, w), _ = as_gpu_inputs(uvw, vis, wt, "f32")
        off = torch.as_tensor(np.asarray(offs), dtype=torch.int64).cuda()
        (G, sw, c), (Gn, swn, cn) = _both(k, 4, u, v, w, off)
        assert rel_max(Gn, G) <= TOL["f32"]
        assert np.allclose(swn, sw, rtol=1e-12, atol=0)
        assert cn.tolist() == c.tolist()
    k.free()


def test_noalloc_refuses_oversized_request():
    """A request whose workspace exceeds the scratch array is refused on the host before
    anything is enqueued (the pointers are never read)."""
    wl = synth.cfg1()
    k = W.make_kernels({**wl.params, "precision": "f32", "algorithm": "tiled"})
    cap = W.noalloc_scratch_bytes()
    nvis = 1
    while k.workspace_size(nvis) <= cap:
        nvis *= 2
    dummy = torch.zeros(16, dtype=torch.float64, device="cuda")
    g = k.new_grid()
    p = ctypes.c_void_p(dummy.data_ptr())
    rc = _lib.lib().wproj_grid_noalloc(k.handle, nvis, p, p, p, None, ctypes.c_void_p(g.data_ptr()),
                                       None, None, None)
    assert rc == -5  # WPROJ_EWORKSPACE
    assert b"scratch" in _lib.lib().wproj_last_error()
    torch.cuda.synchronize()
    assert not g.abs().any()
    k.free()
