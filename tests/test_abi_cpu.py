"""Host-side checks of the C ABI: the library loads, exports every declared entry
point, and rejects bad arguments before touching the GPU."""

import ctypes
import os
import re

import pytest

from paper_1905_03213_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "wproj.h")).read()
    return sorted(set(re.findall(r"^\S[^\n(]*?\b(wproj_\w+)\(", src, re.M)))


def test_header_and_binding_agree():
    assert _declared() == sorted(_lib.EXPORTED)


def test_library_exports_every_declared_symbol():
    L = _lib.lib()
    for name in _declared():
        assert hasattr(L, name), name
    assert L.wproj_version() >= 100


def _params(**kw):
    P = _lib.Params()
    base = dict(n=64, n_wplanes=3, cell_rad=1e-3, w_max=10.0, support=7, oversample=8,
                kernel_image_size=32, precision=_lib.F32, n_images=1, algorithm=0, tile=0)
    base.update(kw)
    for k, v in base.items():
        setattr(P, k, v)
    return P


@pytest.mark.parametrize("bad", [dict(n=63), dict(cell_rad=0.1), dict(n_wplanes=0),
                                 dict(w_max=-1.0), dict(support=0), dict(support=7, oversample=1),
                                 dict(kernel_image_size=31), dict(precision=7), dict(n_images=0),
                                 dict(algorithm=5), dict(tile=48), dict(chunk=100),
                                 dict(w_mode=4), dict(w_mode=-1), dict(accumulate_runs=2),
                                 dict(bin_aggregate=2), dict(bin_aggregate=-1),
                                 dict(stable_bins=2), dict(stable_bins=-1),
                                 dict(n_wlayers=2), dict(w_mode=3, n_wlayers=-1),
                                 dict(w_mode=3, n_wlayers=4097)])
def test_make_kernels_rejects_invalid_params(bad):
    L = _lib.lib()
    h = ctypes.c_void_p()
    rc = L.wproj_make_kernels(ctypes.byref(_params(**bad)), None, ctypes.byref(h))
    assert rc == -1 and not h.value
    assert L.wproj_last_error()


def test_reserved_and_per_plane_support_checked():
    L = _lib.lib()
    P = _params()
    P.reserved[0] = 1
    h = ctypes.c_void_p()
    assert L.wproj_make_kernels(ctypes.byref(P), None, ctypes.byref(h)) == -1
    P = _params()
    spp = (ctypes.c_int32 * 3)(7, 33, 7)
    P.support_per_plane = spp
    assert L.wproj_make_kernels(ctypes.byref(P), None, ctypes.byref(h)) == -1
    assert b"support" in L.wproj_last_error()


def test_null_handle_paths():
    L = _lib.lib()
    assert L.wproj_workspace_size(None, 10) == -1
    assert L.wproj_grid(None, 0, None, None, None, None, None, None, None, None, 0, None) == -1
    assert L.wproj_degrid(None, 0, None, None, None, None, None, 0, None) == -1
    assert L.wproj_plan_rows(None, None, None) == -1
    assert L.wproj_image(None, 0, None, None, None, None, 0, None) == -1
    assert L.wproj_export(None, 0, None, 0, None, None) == -1
    assert L.wproj_footprints(None, 0, None, None, None, None) == -1
    out = ctypes.c_void_p(5)
    assert L.wproj_plan_create(None, 0, None, None, None, None, None, None, 0, None,
                               ctypes.byref(out)) == -1
    assert out.value is None  # cleared on failure
    assert L.wproj_grid_planned(None, None, None, None) == -1
    assert L.wproj_degrid_planned(None, None, None, None) == -1
    assert L.wproj_plan_free(None) == 0
    assert L.wproj_free_kernels(None) == 0


def test_regroup_and_gather_argument_checks():
    L = _lib.lib()
    assert L.wproj_regroup_workspace_size(-1, 27) == -1
    assert L.wproj_regroup_workspace_size(10, 0) == -1
    assert L.wproj_regroup_workspace_size(10, 256) == -4  # one LDS counter per baseline
    assert L.wproj_regroup_workspace_size(1 << 31, 27) == -1
    # workspace: per-block counts (blocks of >= 2048 rows), their scan and the scan's carries
    ws = L.wproj_regroup_workspace_size(1_010_880, 27)
    blocks = -(-1_010_880 // 2048)
    keys = 27 * 28 // 2 + 1
    assert ws >= 4 * (2 * keys * blocks + 1)
    assert L.wproj_regroup_workspace_size(0, 1) > 0
    # NULL outputs and a short workspace are rejected before any GPU work
    assert L.wproj_regroup_rows(4, None, None, 27, None, None, None, None, 0, None) == -1
    fake = ctypes.c_void_p(16)
    assert L.wproj_regroup_rows(4, fake, fake, 27, fake, fake, fake, fake, 8, None) == -5
    assert L.wproj_gather_rows(4, 6, fake, 4, fake, fake, None, None) == -1   # row_bytes % 4
    assert L.wproj_gather_rows(4, 0, fake, 4, fake, fake, None, None) == -1
    assert L.wproj_gather_rows(-1, 8, fake, 4, fake, fake, None, None) == -1
    assert L.wproj_gather_rows(4, 8, None, 4, fake, fake, None, None) == -1


def test_rate_measurements_check_arguments():
    L = _lib.lib()
    bps = ctypes.c_double(0.0)
    # invalid mode, width or rounds, or a NULL result, are refused before any GPU work
    assert L.wproj_measure_lds(3, 16, ctypes.byref(bps), None, None) == -1
    assert L.wproj_measure_lds(0, 0, ctypes.byref(bps), None, None) == -1
    assert L.wproj_measure_lds(0, 16, None, None, None) == -1
    assert L.wproj_measure_vmem(12, 16, ctypes.byref(bps), None, None) == -1
    assert L.wproj_measure_vmem(16, (1 << 20) + 1, ctypes.byref(bps), None, None) == -1
    assert L.wproj_measure_vmem(8, 16, None, None, None) == -1
    assert L.wproj_measure_vmem(2, 16, ctypes.byref(bps), None, None) == -1
    assert b"width" in L.wproj_last_error()


def test_chi2_argument_checks():
    L = _lib.lib()
    assert L.wproj_chi2_workspace_size() > 0
    d = ctypes.c_double()
    # unknown precision, negative count, no output, no inputs, no workspace
    assert L.wproj_chi2(7, 0, None, None, None, ctypes.byref(d), None, ctypes.byref(d), 1 << 20, None) == -1
    assert L.wproj_chi2(1, -1, None, None, None, ctypes.byref(d), None, ctypes.byref(d), 1 << 20, None) == -1
    assert L.wproj_chi2(1, 0, None, None, None, None, None, ctypes.byref(d), 1 << 20, None) == -1
    assert L.wproj_chi2(1, 5, None, None, None, ctypes.byref(d), None, ctypes.byref(d), 1 << 20, None) == -1
    assert L.wproj_chi2(1, 0, None, None, None, ctypes.byref(d), None, None, 0, None) == -5
