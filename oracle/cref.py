"""ctypes wrapper of the plain C oracle gridder/degridder (test infrastructure only)."""

import ctypes
import os

import numpy as np

from . import build as _build
from .wproj_ref import W_MODES, Plan, flat_tables

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = ctypes.CDLL(_build.LIB)
        vp, i64, i32, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double
        L.wref_grid.argtypes = [i32, dbl, i32, dbl, i32, i32, vp, i32, vp, vp, i64, vp, vp, vp,
                                i32, vp, vp, vp, vp, i32]
        L.wref_grid.restype = i32
        L.wref_degrid.argtypes = [i32, dbl, i32, dbl, i32, i32, vp, i32, vp, vp, i64, vp, i32, vp,
                                  vp, vp, i32]
        L.wref_degrid.restype = i32
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _prep(plan: Plan, tables):
    flat, offs = flat_tables(tables)
    flat = np.ascontiguousarray(flat.view(np.float64))
    supp = np.ascontiguousarray(np.asarray(plan.supports, dtype=np.int32))
    return flat, offs, supp


def grid(plan: Plan, tables, uvw, vis, weight, image_offsets=None, nthreads: int = 1, out=None):
    """Same contract as wproj_ref.grid, computed by the C loop."""
    flat, offs, supp = _prep(plan, tables)
    uvw = np.ascontiguousarray(uvw, dtype=np.float64)
    vis = np.ascontiguousarray(vis, dtype=np.complex128)
    wt = np.ascontiguousarray(weight, dtype=np.float64)
    G = out if out is not None else np.zeros((plan.n_grids, plan.n, plan.n), dtype=np.complex128)
    sumw = np.zeros(plan.n_images)
    cnt = np.zeros(3, dtype=np.int64)
    io = None if image_offsets is None else np.ascontiguousarray(image_offsets, dtype=np.int64)
    rc = lib().wref_grid(plan.n, plan.cell, plan.n_w, plan.w_max, W_MODES.index(plan.w_mode),
                         plan.n_layers, _p(supp), plan.O, _p(flat),
                         _p(offs), uvw.shape[0], _p(uvw), _p(vis.view(np.float64)), _p(wt),
                         plan.n_images, None if io is None else _p(io), _p(G.view(np.float64)),
                         _p(sumw), _p(cnt), int(nthreads))
    if rc != 0:
        raise MemoryError("wref_grid failed")
    return G, sumw, cnt


def degrid(plan: Plan, tables, uvw, M, image_offsets=None, nthreads: int = 1):
    flat, offs, supp = _prep(plan, tables)
    uvw = np.ascontiguousarray(uvw, dtype=np.float64)
    M = np.ascontiguousarray(M, dtype=np.complex128)
    out = np.zeros(uvw.shape[0], dtype=np.complex128)
    io = None if image_offsets is None else np.ascontiguousarray(image_offsets, dtype=np.int64)
    lib().wref_degrid(plan.n, plan.cell, plan.n_w, plan.w_max, W_MODES.index(plan.w_mode),
                      plan.n_layers, _p(supp), plan.O, _p(flat),
                      _p(offs), uvw.shape[0], _p(uvw), plan.n_images,
                      None if io is None else _p(io), _p(M.view(np.float64)),
                      _p(out.view(np.float64)), int(nthreads))
    return out
