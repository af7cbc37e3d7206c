"""Binned gridding and degridding on geometries the other tests do not reach, against
the FP64 oracle: a single w-plane (w ignored), odd and non-power-of-two oversampling
(5 and 6, so floor division is not a shift), support 7 with oversampling 4, odd per-plane
supports, a grid side that is not a multiple of the tile (ragged edge tiles), and more
sub-kernels than packed records can number (oversampling 256), each with footprints
reaching the grid edges."""

import numpy as np
import pytest
import torch

import paper_1905_03213_amd as W
from oracle import wproj_ref as R

from gpu_util import oracle_grid, rel_max, run_grid

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5, "f32_f16table": 1e-3}

GEOMETRIES = {
    "one_plane": dict(n=256, cell_rad=5e-5, n_wplanes=1, w_max=0.0, support=8, oversample=8,
                      kernel_image_size=16),
    "O5_S8": dict(n=192, cell_rad=6e-5, n_wplanes=9, w_max=300.0, support=8, oversample=5,
                  kernel_image_size=32),
    "O4_S7": dict(n=160, cell_rad=6e-5, n_wplanes=5, w_max=300.0, support=7, oversample=4,
                  kernel_image_size=32),
    "O6_odd_supports": dict(n=200, cell_rad=6e-5, n_wplanes=7, w_max=300.0, support=5,
                            support_per_plane=[5, 7, 9, 11, 9, 7, 5], oversample=6,
                            kernel_image_size=64),
    "ragged_n": dict(n=250, cell_rad=5e-5, n_wplanes=5, w_max=300.0, support=8, oversample=8,
                     kernel_image_size=32),
    # 5 x 256^2 sub-kernels: more than the 2^18 a record can carry above its LDS offset,
    # so this fixed support takes unpacked records, the recomputing scatter and the
    # general gridder and degridder paths
    "O256_many_subkernels": dict(n=128, cell_rad=6e-5, n_wplanes=5, w_max=300.0, support=4,
                                 oversample=256, kernel_image_size=32),
}


def _inputs(params, seed, nvis=20000):
    rng = np.random.default_rng(seed)
    n = params["n"]
    fov = n * params["cell_rad"]
    umax = (n / 2) / fov
    uv = rng.uniform(-umax, umax, (nvis, 2))  # includes footprints at and past the edges
    w = rng.uniform(-1.05, 1.05, nvis) * max(params["w_max"], 1.0)
    uvw = np.concatenate([uv, w[:, None]], axis=1)
    vis = rng.standard_normal(nvis) + 1j * rng.standard_normal(nvis)
    wt = rng.uniform(0.25, 2.0, nvis)
    return uvw, vis, wt


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("geom", list(GEOMETRIES))
def test_tiled_grid_geometries(geom, prec):
    params = {**GEOMETRIES[geom], "precision": prec, "algorithm": "tiled", "n_images": 1}
    uvw, vis, wt = _inputs(params, 1)
    G, sw, cnt, host = run_grid(params, uvw, vis, wt)
    (Gr, swr, cr), _, _ = oracle_grid(params, host)
    assert cnt.tolist() == cr.tolist()
    assert cr[0] > 0  # some footprints fell off the edges
    assert np.allclose(sw, swr, rtol=1e-12, atol=0)
    assert rel_max(G, Gr) <= TOL[prec]


@pytest.mark.parametrize("geom", list(GEOMETRIES))
def test_tiled_degrid_geometries(geom):
    params = {**GEOMETRIES[geom], "precision": "f32", "algorithm": "tiled", "n_images": 1}
    uvw, _, _ = _inputs(params, 2)
    plan = R.Plan(params)
    tabs = R.kernel_tables(plan)
    n = plan.n
    rng = np.random.default_rng(3)
    M = (rng.standard_normal((1, n, n)) + 1j * rng.standard_normal((1, n, n))).astype(np.complex64)
    k = W.make_kernels(params)
    out = torch.full((uvw.shape[0],), 7.0 + 7.0j, dtype=torch.complex64, device="cuda")
    W.degrid(k, torch.as_tensor(uvw).cuda(), torch.as_tensor(M).cuda(), out)
    ref = R.degrid(plan, tabs, uvw, M.astype(np.complex128))
    got = out.to(torch.complex128).cpu().numpy()
    assert rel_max(got, ref) <= TOL["f32"]
    assert np.count_nonzero(got) == np.count_nonzero(ref)
    k.free()


FIXED = list(range(3, 17))
# supports above 16 have no kernel of their own: the general (one record at a time) path
GENERAL = [20, 32]


def _fixed_params(s_full, prec):
    return dict(n=192, cell_rad=6e-5, n_wplanes=5, w_max=300.0, support=s_full, oversample=8,
                kernel_image_size=max(32, 2 * s_full), n_images=1, precision=prec, algorithm="tiled")


@pytest.mark.parametrize("prec", ["f64", "f32", "f32_f16table"])
@pytest.mark.parametrize("s_full", FIXED + GENERAL)
def test_tiled_grid_fixed_supports(s_full, prec):
    """Every fixed support from 3 to 16 has its own gridder kernel (one tap per lane in
    ceil(S^2 / 64) passes); 6 is the largest that fits one pass with lanes to spare, 9 the
    first with two passes, 16 the largest with its own kernel.  With FP32 arithmetic the
    taps of two records arrive in one load from a pair-ordered copy of the table; an odd
    number of taps in the last pass leaves one entry of that copy empty (S = 3, 5, 7, 9,
    11, 13, 15; 13 and 15 are the three- and four-pass kernels with an odd last pass).
    Supports 20 and 32 (the largest accepted) take the general path."""
    params = _fixed_params(s_full, prec)
    uvw, vis, wt = _inputs(params, 5)
    G, sw, cnt, host = run_grid(params, uvw, vis, wt)
    (Gr, swr, cr), _, _ = oracle_grid(params, host)
    assert cnt.tolist() == cr.tolist()
    assert np.allclose(sw, swr, rtol=1e-12, atol=0)
    assert rel_max(G, Gr) <= TOL[prec]


@pytest.mark.parametrize("s_full", FIXED + GENERAL)
def test_tiled_degrid_fixed_supports(s_full):
    params = _fixed_params(s_full, "f32")
    uvw, _, _ = _inputs(params, 6)
    plan = R.Plan(params)
    tabs = R.kernel_tables(plan)
    n = plan.n
    rng = np.random.default_rng(8)
    M = (rng.standard_normal((1, n, n)) + 1j * rng.standard_normal((1, n, n))).astype(np.complex64)
    k = W.make_kernels(params)
    out = torch.full((uvw.shape[0],), 7.0 + 7.0j, dtype=torch.complex64, device="cuda")
    W.degrid(k, torch.as_tensor(uvw).cuda(), torch.as_tensor(M).cuda(), out)
    ref = R.degrid(plan, tabs, uvw, M.astype(np.complex128))
    got = out.to(torch.complex128).cpu().numpy()
    assert rel_max(got, ref) <= TOL["f32"]
    assert np.count_nonzero(got) == np.count_nonzero(ref)
    k.free()


@pytest.mark.parametrize("s_full", [4, 7, 8])
@pytest.mark.parametrize("tile,chunk", [(16, 256), (32, 300), (32, 8192), (64, 1000)])
def test_tap_lane_degrid_tiles_and_chunks(s_full, tile, chunk):
    """The one-tap-per-lane degridder (FP32 tables, fixed support up to 8) reads cells at
    offsets set by the tile's row pitch, and a team of four wavefronts splits each work
    item into batches of 64 records: tiles 16, 32 and 64, and work items of 256, 300, 1000
    and 8192 records (ragged last batches, items shorter than one batch per wavefront)
    against the oracle, with dense hot tiles so that items split."""
    params = {**_fixed_params(s_full, "f32"), "tile": tile, "chunk": chunk}
    rng = np.random.default_rng(11)
    uvw, _, _ = _inputs(params, 12, nvis=30000)
    # a third of the rows in a small hot region, so its tiles hold several work items
    hot = rng.random(uvw.shape[0]) < 0.33
    uvw[hot, :2] = rng.uniform(-15.0, 15.0, (int(hot.sum()), 2))
    plan = R.Plan(params)
    tabs = R.kernel_tables(plan)
    n = plan.n
    M = (rng.standard_normal((1, n, n)) + 1j * rng.standard_normal((1, n, n))).astype(np.complex64)
    k = W.make_kernels(params)
    out = torch.full((uvw.shape[0],), 7.0 + 7.0j, dtype=torch.complex64, device="cuda")
    W.degrid(k, torch.as_tensor(uvw).cuda(), torch.as_tensor(M).cuda(), out)
    ref = R.degrid(plan, tabs, uvw, M.astype(np.complex128))
    got = out.to(torch.complex128).cpu().numpy()
    assert rel_max(got, ref) <= TOL["f32"]
    assert np.count_nonzero(got) == np.count_nonzero(ref)
    k.free()
