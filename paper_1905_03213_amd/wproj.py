"""Python binding of the w-projection C ABI: argument marshalling only.

Tensors are passed by device pointer (torch supplies memory and the current
HIP stream); every step runs in the library's HIP kernels.  Function names
follow the C entry points (wproj_make_kernels -> make_kernels, ...).
"""

from __future__ import annotations

import ctypes
from typing import Optional

import torch

from . import _lib
from ._lib import (ALGO_PLAIN, ALGO_TILED, F32, F32_F16TABLE, F64, GRID_TO_IMAGE,  # noqa: F401
                   GRID_TO_IMAGE_RAW, IMAGE_TO_GRID, WprojError)

_PREC = {"f64": F64, "f32": F32, "f32_f16table": F32_F16TABLE}
_ALGO = {"tiled": ALGO_TILED, "plain": ALGO_PLAIN}
_WMODE = {"linear": _lib.W_LINEAR, "fold": _lib.W_FOLD, "fold_sqrt": _lib.W_FOLD_SQRT,
          "stack": _lib.W_STACK}


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def _ptr(t: Optional[torch.Tensor], name: str, dtype=None, numel=None):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if numel is not None and t.numel() < numel:
        raise ValueError(f"{name} holds {t.numel()} elements, {numel} needed")
    return ctypes.c_void_p(t.data_ptr())


class Kernels:
    """A built handle (kernel tables, grid correction, FFT plans) and its parameters."""

    def __init__(self, handle: ctypes.c_void_p, params: dict):
        self.handle = handle
        self.params = dict(params)
        prec = self.params["precision"]
        self.real = torch.float64 if prec == "f64" else torch.float32
        self.cplx = torch.complex128 if prec == "f64" else torch.complex64

    def free(self):
        if self.handle:
            _lib.lib().wproj_free_kernels(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def workspace_size(self, nvis: int) -> int:
        r = _lib.lib().wproj_workspace_size(self.handle, int(nvis))
        if r < 0:
            _lib.check("wproj_workspace_size", int(r))
        return int(r)

    def workspace(self, nvis: int, device="cuda") -> torch.Tensor:
        return torch.empty(max(1, self.workspace_size(nvis)), dtype=torch.uint8, device=device)

    def export(self, what: int, stream=None) -> torch.Tensor:
        L = _lib.lib()
        need = ctypes.c_int64(0)
        _lib.check("wproj_export", L.wproj_export(self.handle, int(what), None, 0,
                                                   ctypes.byref(need), None))
        out = torch.empty(need.value, dtype=torch.uint8, device="cuda")
        _lib.check("wproj_export", L.wproj_export(self.handle, int(what),
                                                   ctypes.c_void_p(out.data_ptr()), need.value,
                                                   None, _stream(stream)))
        return out

    def profile(self, enable: bool = True):
        """wproj_profile: record HIP events around each phase of this handle's calls."""
        _lib.check("wproj_profile", _lib.lib().wproj_profile(self.handle, int(bool(enable))))

    def profile_read(self) -> dict:
        """wproj_profile_read: {phase: (total_ms, n_intervals)} since the last read."""
        import numpy as np

        ms = np.zeros(len(_lib.PHASES), dtype=np.float64)
        cnt = np.zeros(len(_lib.PHASES), dtype=np.int64)
        _lib.check("wproj_profile_read", _lib.lib().wproj_profile_read(
            self.handle, ms.ctypes.data_as(ctypes.c_void_p), cnt.ctypes.data_as(ctypes.c_void_p)))
        return {name: (float(ms[i]), int(cnt[i])) for i, name in enumerate(_lib.PHASES)}

    def tuning(self) -> tuple:
        """wproj_tuning: (tile, chunk) of the tiled gridder."""
        return self.tuning_all()[:2]

    def tuning_all(self) -> tuple:
        """wproj_tuning: (tile, chunk, bin_aggregate)."""
        t, c, a = ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_int32(0)
        _lib.check("wproj_tuning", _lib.lib().wproj_tuning(self.handle, ctypes.byref(t), ctypes.byref(c),
                                                           ctypes.byref(a)))
        return int(t.value), int(c.value), int(a.value)

    def new_grid(self, device="cuda") -> torch.Tensor:
        return torch.zeros((self.n_grids, self.params["n"], self.params["n"]), dtype=self.cplx,
                           device=device)

    @property
    def n_grids(self) -> int:
        """Grids per call: one per image, or one per (image, w-stacking layer)."""
        stacked = self.params.get("w_mode") in ("stack", _lib.W_STACK)
        layers = max(1, int(self.params.get("n_wlayers", 1) or 1)) if stacked else 1
        return int(self.params.get("n_images", 1)) * layers


def make_kernels(params: dict, stream=None) -> Kernels:
    """wproj_make_kernels.  params keys: n, cell_rad, n_wplanes, w_max, support,
    support_per_plane (list or None), oversample, kernel_image_size, precision
    ("f64" | "f32" | "f32_f16table"), n_images, algorithm ("tiled" | "plain"), tile, chunk,
    w_mode ("linear" | "fold" | "fold_sqrt" | "stack"), n_wlayers (w-stacking layers),
    accumulate_runs (bool), bin_aggregate (bool), stable_bins (bool)."""
    P = _lib.Params()
    P.n = int(params["n"])
    P.n_wplanes = int(params["n_wplanes"])
    P.cell_rad = float(params["cell_rad"])
    P.w_max = float(params["w_max"])
    P.support = int(params["support"])
    P.oversample = int(params["oversample"])
    spp = params.get("support_per_plane")
    keep = None
    if spp is not None:
        keep = (ctypes.c_int32 * len(spp))(*[int(s) for s in spp])
        P.support_per_plane = keep
    P.kernel_image_size = int(params["kernel_image_size"])
    prec = params.get("precision", "f32")
    P.precision = _PREC[prec] if isinstance(prec, str) else int(prec)
    P.n_images = int(params.get("n_images", 1))
    algo = params.get("algorithm", "tiled")
    P.algorithm = _ALGO[algo] if isinstance(algo, str) else int(algo)
    P.tile = int(params.get("tile", 0))
    P.chunk = int(params.get("chunk", 0))
    wm = params.get("w_mode", "linear")
    P.w_mode = _WMODE[wm] if isinstance(wm, str) else int(wm)
    P.n_wlayers = int(params.get("n_wlayers", 0) or 0)
    P.accumulate_runs = int(bool(params.get("accumulate_runs", False)))
    P.bin_aggregate = int(bool(params.get("bin_aggregate", False)))
    P.stable_bins = int(bool(params.get("stable_bins", False)))
    h = ctypes.c_void_p()
    _lib.check("wproj_make_kernels",
               _lib.lib().wproj_make_kernels(ctypes.byref(P), _stream(stream), ctypes.byref(h)))
    del keep
    p = dict(params)
    p.setdefault("precision", "f32")
    p.setdefault("n_images", 1)
    return Kernels(h, p)


def grid(k: Kernels, uvw: torch.Tensor, vis: torch.Tensor, weight: torch.Tensor,
         grid_out: torch.Tensor, image_offsets: Optional[torch.Tensor] = None,
         weight_sum: Optional[torch.Tensor] = None, counters: Optional[torch.Tensor] = None,
         workspace: Optional[torch.Tensor] = None, stream=None):
    """wproj_grid: grid_out += gridded visibilities (weight_sum, counters accumulated)."""
    nvis = int(uvw.shape[0]) if uvw.dim() else 0
    n, ni = k.params["n"], k.params.get("n_images", 1)
    if workspace is None:
        workspace = k.workspace(nvis)
    _lib.check("wproj_grid", _lib.lib().wproj_grid(
        k.handle, nvis, _ptr(uvw, "uvw", torch.float64, 3 * nvis), _ptr(vis, "vis", k.cplx, nvis),
        _ptr(weight, "weight", k.real, nvis),
        _ptr(image_offsets, "image_offsets", torch.int64, ni + 1),
        _ptr(grid_out, "grid", k.cplx, k.n_grids * n * n),
        _ptr(weight_sum, "weight_sum", torch.float64, ni),
        _ptr(counters, "counters", torch.int64, 3),
        _ptr(workspace, "workspace", torch.uint8), workspace.numel(), _stream(stream)))


def chi2(vis_obs: torch.Tensor, pred: torch.Tensor, weight: Optional[torch.Tensor] = None,
         grad: Optional[torch.Tensor] = None, workspace: Optional[torch.Tensor] = None,
         stream=None) -> torch.Tensor:
    """wproj_chi2: sum_j w_j |o_j - p_j|^2 as a one-element float64 device tensor; if grad
    is given, -2 w_j (o_j - p_j) is written into it.  complex128 arrays run in FP64,
    complex64 in FP32 (weights of the matching real type)."""
    if pred.dtype not in (torch.complex64, torch.complex128):
        raise TypeError("pred must be complex64 or complex128")
    f64 = pred.dtype == torch.complex128
    real = torch.float64 if f64 else torch.float32
    nvis = int(pred.numel())
    out = torch.empty(1, dtype=torch.float64, device=pred.device)
    if workspace is None:
        workspace = torch.empty(int(_lib.lib().wproj_chi2_workspace_size()), dtype=torch.uint8,
                                device=pred.device)
    _lib.check("wproj_chi2", _lib.lib().wproj_chi2(
        _lib.F64 if f64 else _lib.F32, nvis, _ptr(vis_obs, "vis_obs", pred.dtype, nvis),
        _ptr(pred, "pred", pred.dtype, nvis), _ptr(weight, "weight", real, nvis),
        _ptr(out, "chi2", torch.float64, 1), _ptr(grad, "grad", pred.dtype, nvis),
        _ptr(workspace, "workspace", torch.uint8), workspace.numel(), _stream(stream)))
    return out


def check_weights(k: Kernels, weight_sum: torch.Tensor, stream=None):
    """wproj_check_weights: waits for the stream; raises WprojError (code WPROJ_EEMPTY = -7)
    when an image's sum of weights is 0 (that image comes out of GRID_TO_IMAGE as zeros)."""
    ni = k.params.get("n_images", 1)
    _lib.check("wproj_check_weights", _lib.lib().wproj_check_weights(
        k.handle, _ptr(weight_sum, "weight_sum", torch.float64, ni), _stream(stream)))


def measure_lds(mode: int, rounds: int = 4096, stream=None) -> tuple:
    """wproj_measure_lds: (bytes per second, kernel ms) of the LDS streaming kernel
    (mode 0 reads, 1 writes, 2 read-add-write of 64-bit words)."""
    bps, ms = ctypes.c_double(0.0), ctypes.c_double(0.0)
    _lib.check("wproj_measure_lds", _lib.lib().wproj_measure_lds(
        int(mode), int(rounds), ctypes.byref(bps), ctypes.byref(ms), _stream(stream)))
    return bps.value, ms.value


def measure_vmem(width: int, rounds: int = 4096, stream=None) -> tuple:
    """wproj_measure_vmem: (bytes per second, kernel ms) of L1-resident buffer loads of
    `width` (4, 8 or 16) bytes per lane."""
    bps, ms = ctypes.c_double(0.0), ctypes.c_double(0.0)
    _lib.check("wproj_measure_vmem", _lib.lib().wproj_measure_vmem(
        int(width), int(rounds), ctypes.byref(bps), ctypes.byref(ms), _stream(stream)))
    return bps.value, ms.value


def grid_noalloc(k: Kernels, uvw: torch.Tensor, vis: torch.Tensor, weight: torch.Tensor,
                 grid_out: torch.Tensor, image_offsets: Optional[torch.Tensor] = None,
                 weight_sum: Optional[torch.Tensor] = None, counters: Optional[torch.Tensor] = None,
                 stream=None):
    """wproj_grid_noalloc: wproj_grid with the library's fixed per-GPU scratch array as
    workspace (nothing allocated; overlapping calls on one GPU race)."""
    nvis = int(uvw.shape[0]) if uvw.dim() else 0
    n, ni = k.params["n"], k.params.get("n_images", 1)
    _lib.check("wproj_grid_noalloc", _lib.lib().wproj_grid_noalloc(
        k.handle, nvis, _ptr(uvw, "uvw", torch.float64, 3 * nvis), _ptr(vis, "vis", k.cplx, nvis),
        _ptr(weight, "weight", k.real, nvis),
        _ptr(image_offsets, "image_offsets", torch.int64, ni + 1),
        _ptr(grid_out, "grid", k.cplx, k.n_grids * n * n),
        _ptr(weight_sum, "weight_sum", torch.float64, ni),
        _ptr(counters, "counters", torch.int64, 3), _stream(stream)))


def noalloc_scratch_bytes() -> int:
    """wproj_noalloc_scratch_bytes: size of the per-GPU scratch array of grid_noalloc."""
    return int(_lib.lib().wproj_noalloc_scratch_bytes())


def autotune(k: Kernels, uvw: torch.Tensor, vis: torch.Tensor, weight: torch.Tensor,
             image_offsets: Optional[torch.Tensor] = None, workspace: Optional[torch.Tensor] = None,
             stream=None) -> tuple:
    """wproj_autotune on these visibilities; returns the chosen (tile, chunk)."""
    nvis = int(uvw.shape[0])
    n, ni = k.params["n"], k.params.get("n_images", 1)
    if workspace is None:
        workspace = k.workspace(nvis)
    scratch = k.new_grid(device=uvw.device)
    _lib.check("wproj_autotune", _lib.lib().wproj_autotune(
        k.handle, nvis, _ptr(uvw, "uvw", torch.float64, 3 * nvis), _ptr(vis, "vis", k.cplx, nvis),
        _ptr(weight, "weight", k.real, nvis),
        _ptr(image_offsets, "image_offsets", torch.int64, ni + 1),
        _ptr(scratch, "scratch_grid", k.cplx, k.n_grids * n * n),
        _ptr(workspace, "workspace", torch.uint8), workspace.numel(), _stream(stream)))
    return k.tuning()


def degrid(k: Kernels, uvw: torch.Tensor, model_grid: torch.Tensor, vis_out: torch.Tensor,
           image_offsets: Optional[torch.Tensor] = None, workspace: Optional[torch.Tensor] = None,
           stream=None):
    """wproj_degrid: vis_out = prediction from the model grid."""
    nvis = int(uvw.shape[0])
    n, ni = k.params["n"], k.params.get("n_images", 1)
    if workspace is None:
        workspace = k.workspace(nvis)
    _lib.check("wproj_degrid", _lib.lib().wproj_degrid(
        k.handle, nvis, _ptr(uvw, "uvw", torch.float64, 3 * nvis),
        _ptr(model_grid, "model_grid", k.cplx, k.n_grids * n * n),
        _ptr(image_offsets, "image_offsets", torch.int64, ni + 1),
        _ptr(vis_out, "vis_out", k.cplx, nvis),
        _ptr(workspace, "workspace", torch.uint8), workspace.numel(), _stream(stream)))


def image(k: Kernels, direction: int, grid_buf: torch.Tensor, image_buf: torch.Tensor,
          weight_sum: Optional[torch.Tensor] = None, workspace: Optional[torch.Tensor] = None,
          stream=None):
    """wproj_image: GRID_TO_IMAGE(_RAW) transforms grid_buf in place into image_buf;
    IMAGE_TO_GRID overwrites grid_buf from image_buf."""
    n, ni = k.params["n"], k.params.get("n_images", 1)
    if workspace is None:
        workspace = k.workspace(0)
    _lib.check("wproj_image", _lib.lib().wproj_image(
        k.handle, int(direction), _ptr(grid_buf, "grid", k.cplx, k.n_grids * n * n),
        _ptr(image_buf, "image", k.real, ni * n * n),
        _ptr(weight_sum, "weight_sum", torch.float64, ni),
        _ptr(workspace, "workspace", torch.uint8), workspace.numel(), _stream(stream)))


class Plan:
    """wproj_plan_create: the binning of one set of rows kept for repeated gridding and
    degridding.  Holds its workspace; free() releases the plan."""

    def __init__(self, k: Kernels, uvw: torch.Tensor, weight: torch.Tensor,
                 image_offsets: Optional[torch.Tensor] = None,
                 weight_sum: Optional[torch.Tensor] = None, counters: Optional[torch.Tensor] = None,
                 stream=None):
        self.k = k
        self.nvis = int(uvw.shape[0])
        ni = k.params.get("n_images", 1)
        self.workspace = k.workspace(self.nvis, device=uvw.device)
        h = ctypes.c_void_p()
        _lib.check("wproj_plan_create", _lib.lib().wproj_plan_create(
            k.handle, self.nvis, _ptr(uvw, "uvw", torch.float64, 3 * self.nvis),
            _ptr(weight, "weight", k.real, self.nvis),
            _ptr(image_offsets, "image_offsets", torch.int64, ni + 1),
            _ptr(weight_sum, "weight_sum", torch.float64, ni),
            _ptr(counters, "counters", torch.int64, 3),
            _ptr(self.workspace, "workspace", torch.uint8), self.workspace.numel(),
            _stream(stream), ctypes.byref(h)))
        self.handle = h

    def grid(self, vis: torch.Tensor, grid_buf: torch.Tensor, stream=None):
        n, ni = self.k.params["n"], self.k.params.get("n_images", 1)
        _lib.check("wproj_grid_planned", _lib.lib().wproj_grid_planned(
            self.handle, _ptr(vis, "vis", self.k.cplx, self.nvis),
            _ptr(grid_buf, "grid", self.k.cplx, self.k.n_grids * n * n), _stream(stream)))

    def degrid(self, model_grid: torch.Tensor, vis_out: torch.Tensor, stream=None):
        n, ni = self.k.params["n"], self.k.params.get("n_images", 1)
        _lib.check("wproj_degrid_planned", _lib.lib().wproj_degrid_planned(
            self.handle, _ptr(model_grid, "model_grid", self.k.cplx, self.k.n_grids * n * n),
            _ptr(vis_out, "vis_out", self.k.cplx, self.nvis), _stream(stream)))

    def rows(self, stream=None) -> torch.Tensor:
        """wproj_plan_rows: the row of each binned record in bin order, as int32 holding
        the uint32 rows (entries past the binned rows are 0xffffffff, i.e. -1)."""
        out = torch.empty(self.nvis, dtype=torch.int32, device=self.workspace.device)
        _lib.check("wproj_plan_rows", _lib.lib().wproj_plan_rows(
            self.handle, _ptr(out, "rows", torch.int32, self.nvis), _stream(stream)))
        return out

    def free(self):
        if self.handle is not None and self.handle.value:
            _lib.lib().wproj_plan_free(self.handle)
        self.handle = None
        self.workspace = None


def footprints(k: Kernels, uvw: torch.Tensor, weight: Optional[torch.Tensor] = None,
               stream=None) -> torch.Tensor:
    """wproj_footprints: int32 [nvis, 6] = (x0, y0, ou, ov, p, class) per visibility."""
    nvis = int(uvw.shape[0])
    out = torch.empty((nvis, 6), dtype=torch.int32, device=uvw.device)
    _lib.check("wproj_footprints", _lib.lib().wproj_footprints(
        k.handle, nvis, _ptr(uvw, "uvw", torch.float64, 3 * nvis),
        _ptr(weight, "weight", k.real, nvis), _ptr(out, "out", torch.int32, 6 * nvis),
        _stream(stream)))
    return out


def regroup_rows(ant1: torch.Tensor, ant2: torch.Tensor, n_ant: int, stream=None):
    """wproj_regroup_rows (Eqs. 5 and 6): returns (perm, start, counts), int64 device tensors;
    rows in increasing baseline number, time order kept inside each baseline."""
    n_rows = int(ant1.shape[0])
    if int(ant2.shape[0]) != n_rows:
        raise ValueError("ant1 and ant2 differ in length")
    n_keys = n_ant * (n_ant + 1) // 2 + 1
    need = int(_lib.lib().wproj_regroup_workspace_size(n_rows, int(n_ant)))
    if need < 0:
        raise _lib.WprojError("wproj_regroup_workspace_size", need, last_error())
    dev = ant1.device
    perm = torch.empty(n_rows, dtype=torch.int64, device=dev)
    start = torch.empty(n_keys, dtype=torch.int64, device=dev)
    counts = torch.empty(n_keys, dtype=torch.int64, device=dev)
    ws = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
    _lib.check("wproj_regroup_rows", _lib.lib().wproj_regroup_rows(
        n_rows, _ptr(ant1, "ant1", torch.int32, n_rows), _ptr(ant2, "ant2", torch.int32, n_rows),
        int(n_ant), _ptr(perm, "perm", torch.int64, n_rows), _ptr(start, "start", torch.int64, n_keys),
        _ptr(counts, "counts", torch.int64, n_keys), _ptr(ws, "workspace", torch.uint8), ws.numel(),
        _stream(stream)))
    return perm, start, counts


def regroup_channels(perm: torch.Tensor, start: torch.Tensor, counts: torch.Tensor, n_ant: int,
                     n_chan: int, stream=None) -> torch.Tensor:
    """wproj_regroup_channels: the visibility permutation (int64 [n_rows * n_chan]) that
    takes rows regrouped by baseline (regroup_rows) to baseline-, channel-, time-major order."""
    n_rows = int(perm.shape[0])
    n_keys = n_ant * (n_ant + 1) // 2 + 1
    out = torch.empty(n_rows * int(n_chan), dtype=torch.int64, device=perm.device)
    _lib.check("wproj_regroup_channels", _lib.lib().wproj_regroup_channels(
        n_rows, int(n_ant), int(n_chan), _ptr(perm, "perm", torch.int64, n_rows),
        _ptr(start, "start", torch.int64, n_keys), _ptr(counts, "counts", torch.int64, n_keys),
        _ptr(out, "vis_perm", torch.int64, n_rows * int(n_chan)), _stream(stream)))
    return out


def gather_rows(perm: torch.Tensor, src: torch.Tensor, out: Optional[torch.Tensor] = None,
                bad: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """wproj_gather_rows: out[k] = src[perm[k]] over the first dimension of src."""
    n_rows = int(perm.shape[0])
    n_src = int(src.shape[0])
    row_bytes = src[0].numel() * src.element_size() if n_src else src.element_size()
    if out is None:
        out = torch.empty((n_rows,) + tuple(src.shape[1:]), dtype=src.dtype, device=src.device)
    if not src.is_contiguous() or not out.is_contiguous():
        raise ValueError("src and out must be contiguous")
    _lib.check("wproj_gather_rows", _lib.lib().wproj_gather_rows(
        n_rows, row_bytes, _ptr(perm, "perm", torch.int64, n_rows), n_src,
        _ptr(src, "src") if n_src else None, _ptr(out, "out") if n_rows else None,
        _ptr(bad, "bad", torch.int64, 1), _stream(stream)))
    return out


def last_error() -> str:
    return _lib.lib().wproj_last_error().decode()


def version() -> int:
    return int(_lib.lib().wproj_version())
