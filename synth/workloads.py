"""Seeded synthetic workloads shaped like the paper's JVLA test.

The paper validates on an 8 h, L-band (1-2 GHz), D-array JVLA observation of
G55.7+3.4 imaged at 1024^2 with 23 w-planes and full support 9 (Section 3.1,
"Validation Test").  That measurement set is not available, so these
generators stand in for it: 27 antennas (as in the VLA) on random positions,
Earth-rotation tracks over 8 h at 10 s integrations, L-band channels, point
source skies plus Gaussian noise.  Rows come in measurement-set order
(time, baseline, channel), the order the paper says the data arrive in before
its GPU path regroups them by baseline (Section 2.2).

Randomness is drawn with numpy's PCG64 from fixed seeds (config index k uses
seed k for layouts/tracks and 100 + k for the sky), so the same arrays come out
on any machine.  The visibility sums are evaluated with torch in float64 on
the requested device; the values are inputs only and both the oracle and the
GPU path receive the very same arrays.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional

import numpy as np
import torch

C_LIGHT = 299792458.0


@dataclass
class Workload:
    """One synthetic imaging problem.

    ``params`` mirrors the C-ABI parameter block: n, cell_rad, n_wplanes,
    w_max, support, support_per_plane (list or None), oversample,
    kernel_image_size, precision ("f64", "f32", "f32_f16table"), n_images.
    Arrays are numpy on the host or torch tensors on ``device``.
    """

    name: str
    params: dict
    uvw: object  # [nvis, 3] float64, wavelengths
    vis: object  # [nvis] complex128
    weight: object  # [nvis] float64
    image_offsets: Optional[object] = None  # [n_images + 1] int64 CSR, or None
    sources: dict = field(default_factory=dict)

    @property
    def nvis(self) -> int:
        return int(self.uvw.shape[0])


# ---------------------------------------------------------------------------
# building blocks
# ---------------------------------------------------------------------------


def area_uniform_disk(rng: np.random.Generator, n: int, radius: float):
    """n points uniform in area inside a disk: r = R sqrt(U), theta = 2 pi U."""
    r = radius * np.sqrt(rng.random(n))
    th = 2.0 * np.pi * rng.random(n)
    return r * np.cos(th), r * np.sin(th)


def array_tracks(
    rng: np.random.Generator,
    n_ant: int = 27,
    radius_m: float = 10e3,
    height_m: float = 50.0,
    lat_deg: float = 34.08,
    dec_deg: float = 45.0,
    hours: float = 8.0,
    dt_s: float = 10.0,
):
    """Baseline (u,v,w) in metres for an Earth-rotation synthesis track.

    Antennas are placed area-uniformly in a disk (east, north) with heights
    uniform in +-height_m.  Local east/north/up offsets are rotated to
    equatorial components at the array latitude, then to (u,v,w) for each hour
    angle H and the source declination (the standard interferometry rotation).
    Time samples sit at the middle of each dt_s interval across [-hours/2,
    hours/2].  Baselines are the pairs a1 < a2 in lexicographic order.

    Returns (uvw_m [n_time, n_bl, 3], ant1 [n_bl], ant2 [n_bl]).
    """
    e, n = area_uniform_disk(rng, n_ant, radius_m)
    up = rng.uniform(-height_m, height_m, n_ant)
    lat = math.radians(lat_deg)
    X = -math.sin(lat) * n + math.cos(lat) * up
    Y = e
    Z = math.cos(lat) * n + math.sin(lat) * up
    a1, a2 = np.triu_indices(n_ant, k=1)
    bx, by, bz = X[a2] - X[a1], Y[a2] - Y[a1], Z[a2] - Z[a1]
    n_time = int(round(hours * 3600.0 / dt_s))
    t = -hours * 3600.0 / 2.0 + (np.arange(n_time) + 0.5) * dt_s
    H = t * (2.0 * np.pi / 86400.0)
    dec = math.radians(dec_deg)
    sH, cH = np.sin(H)[:, None], np.cos(H)[:, None]
    sd, cd = math.sin(dec), math.cos(dec)
    u = sH * bx + cH * by
    v = -sd * cH * bx + sd * sH * by + cd * bz
    w = cd * cH * bx - cd * sH * by + sd * bz
    return np.stack([u, v, w], axis=-1), a1.astype(np.int32), a2.astype(np.int32)


def point_source_vis(uvw, l, m, flux, device="cpu", chunk: int = 1 << 22):
    """V = sum_k S_k exp(-2 pi i (u l_k + v m_k + w (n_k - 1))), n_k = sqrt(1 - l^2 - m^2).

    The measurement equation for unresolved sources (no 1/n factor).  uvw is a
    float64 torch tensor or numpy array [nvis, 3]; the result is complex128 of
    the same kind on ``device``.
    """
    as_numpy = isinstance(uvw, np.ndarray)
    U = torch.as_tensor(uvw, dtype=torch.float64, device=device)
    lt = torch.as_tensor(np.asarray(l, dtype=np.float64), device=device)
    mt = torch.as_tensor(np.asarray(m, dtype=np.float64), device=device)
    nt = torch.sqrt(1.0 - lt * lt - mt * mt) - 1.0
    st = torch.as_tensor(np.asarray(flux, dtype=np.float64), device=device)
    out = torch.empty(U.shape[0], dtype=torch.complex128, device=device)
    for s in range(0, U.shape[0], chunk):
        blk = U[s : s + chunk]
        ph = -2.0 * math.pi * (
            blk[:, 0:1] * lt[None, :] + blk[:, 1:2] * mt[None, :] + blk[:, 2:3] * nt[None, :]
        )
        re = (torch.cos(ph) * st[None, :]).sum(1)
        im = (torch.sin(ph) * st[None, :]).sum(1)
        out[s : s + chunk] = torch.complex(re, im)
    return out.cpu().numpy() if as_numpy else out


def _noise(rng: np.random.Generator, n: int, sigma: float):
    z = rng.standard_normal((n, 2)) * sigma
    return z[:, 0] + 1j * z[:, 1]


def support_ramp(n_wplanes: int, s_min: int, s_max: int):
    """Full support growing linearly with |w|: S_p = s_min + floor((s_max-s_min)*|w_p|/w_max + 1/2).

    Plane p sits at w_p = -w_max + p * 2 w_max / (n_w - 1), so |w_p|/w_max =
    |2p/(n_w-1) - 1|.  Used by the variable-support workloads.
    """
    if n_wplanes == 1:
        return [int(s_min)]
    out = []
    for p in range(n_wplanes):
        frac = abs(2.0 * p / (n_wplanes - 1) - 1.0)
        out.append(int(s_min + math.floor((s_max - s_min) * frac + 0.5)))
    return out


def kernel_image_size_rule(w_max: float, fov: float, s_taper: int, s_max: int) -> int:
    """Smallest power of two >= max(2 S_max, ceil(w_max FoV^2) + S_taper).

    The w phase screen's local fringe rate at the field edge is w l_max cycles
    per unit l, so m samples across 2 l_max resolve it when m >= w FoV^2; the
    taper's own width adds S_taper.
    """
    need = max(2 * s_max, int(math.ceil(w_max * fov * fov)) + s_taper)
    m = 1
    while m < need:
        m *= 2
    return m


def _sky(rng: np.random.Generator, n_src: int, fov: float, frac: float = 0.45):
    flux = rng.uniform(0.1, 1.0, n_src)
    l = rng.uniform(-frac * fov, frac * fov, n_src)
    m = rng.uniform(-frac * fov, frac * fov, n_src)
    return l, m, flux


def _params(n, cell, n_w, w_max, support, oversample, m, precision, spp=None, n_images=1):
    return dict(
        n=int(n),
        cell_rad=float(cell),
        n_wplanes=int(n_w),
        w_max=float(w_max),
        support=int(support),
        support_per_plane=None if spp is None else [int(s) for s in spp],
        oversample=int(oversample),
        kernel_image_size=int(m),
        precision=precision,
        n_images=int(n_images),
    )


# ---------------------------------------------------------------------------
# the workloads
# ---------------------------------------------------------------------------


def cfg1(precision: str = "f64", n_vis: int = 20000) -> Workload:
    """256^2 grid, cell 5e-5 rad, 2e4 visibilities, u,v uniform in a 9000 lambda disk,
    w uniform in +-500 lambda, 32 w-planes, support 7, oversampling 8, five sources."""
    rng = np.random.default_rng(1)
    srng = np.random.default_rng(101)
    n, cell = 256, 5e-5
    fov = n * cell
    u, v = area_uniform_disk(rng, n_vis, 9000.0)
    w = rng.uniform(-500.0, 500.0, n_vis)
    uvw = np.stack([u, v, w], axis=1)
    l, m, flux = _sky(srng, 5, fov)
    vis = point_source_vis(uvw, l, m, flux) + _noise(srng, n_vis, 0.01)
    params = _params(n, cell, 32, 500.0, 7, 8, 16, precision)
    return Workload("cfg1", params, uvw, vis, np.ones(n_vis), None, dict(l=l, m=m, flux=flux))


def cfg1w(n_w: int = 33, oversample: int = 8, s_max: int = 12, m_img: int = 32,
          n_vis: int = 2000, noise: float = 0.0) -> Workload:
    """A w-dominated tiny field: 64^2 grid, cell 1e-3 rad, w uniform in +-1000 lambda,
    u,v uniform in a 350 lambda disk, taper support 7 with per-plane supports 7..s_max.
    Two sources: 1 Jy at (0.010, -0.012) and 0.5 Jy at (-0.020, 0.015)."""
    rng = np.random.default_rng(11)
    n, cell = 64, 1e-3
    u, v = area_uniform_disk(rng, n_vis, 350.0)
    w = rng.uniform(-1000.0, 1000.0, n_vis)
    uvw = np.stack([u, v, w], axis=1)
    l = np.array([0.010, -0.020])
    m = np.array([-0.012, 0.015])
    flux = np.array([1.0, 0.5])
    vis = point_source_vis(uvw, l, m, flux)
    if noise > 0:
        vis = vis + _noise(np.random.default_rng(111), n_vis, noise)
    spp = support_ramp(n_w, 7, s_max) if n_w > 1 else [7]
    params = _params(n, cell, n_w, 1000.0, 7, oversample, m_img, "f64", spp)
    return Workload("cfg1w", params, uvw, vis, np.ones(n_vis), None, dict(l=l, m=m, flux=flux))


def _track_workload(name, seed, n, cell, n_chan, f_lo, f_hi, n_w, support, spp, oversample,
                    precision, n_src, device, hours=8.0, dt_s=10.0, noise=0.01,
                    radius_m=10e3, m_img=None):
    rng = np.random.default_rng(seed)
    srng = np.random.default_rng(100 + seed)
    base, a1, a2 = array_tracks(rng, radius_m=radius_m, hours=hours, dt_s=dt_s)
    freqs = np.linspace(f_lo, f_hi, n_chan) if n_chan > 1 else np.array([f_lo])
    scale = torch.as_tensor(freqs / C_LIGHT, dtype=torch.float64, device=device)
    B = torch.as_tensor(base, dtype=torch.float64, device=device)  # [T, NB, 3]
    uvw = (B[:, :, None, :] * scale[None, None, :, None]).reshape(-1, 3).contiguous()
    fov = n * cell
    l, m, flux = _sky(srng, n_src, fov)
    vis = point_source_vis(uvw, l, m, flux, device=device)
    nv = uvw.shape[0]
    if noise > 0:
        z = torch.as_tensor(srng.standard_normal((nv, 2)) * noise, device=device)
        vis += torch.complex(z[:, 0].contiguous(), z[:, 1].contiguous())
    w_max = float(uvw[:, 2].abs().max())
    s_max = max(spp) if spp else support
    if m_img is None:
        m_img = kernel_image_size_rule(w_max, fov, support, s_max)
    params = _params(n, cell, n_w, w_max, support, oversample, m_img, precision, spp)
    weight = torch.ones(nv, dtype=torch.float64, device=device)
    return Workload(name, params, uvw, vis, weight, None,
                    dict(l=l, m=m, flux=flux, freqs=freqs, ant1=a1, ant2=a2,
                         n_time=base.shape[0], n_bl=base.shape[1], n_chan=n_chan))


def cfg2(device="cuda", precision: str = "f32", n_chan: int = 64, hours: float = 8.0) -> Workload:
    """2048^2 grid, cell 1e-5 rad; 27 antennas in a 10 km-radius disk, 351 baselines,
    8 h at 10 s, dec +45 deg, 64 channels over 1.0-1.5 GHz (6.47e7 visibilities);
    128 w-planes, S=8, oversampling 8, 50 point sources."""
    return _track_workload("cfg2", 2, 2048, 1e-5, n_chan, 1.0e9, 1.5e9, 128, 8, None, 8,
                           precision, 50, device, hours=hours)


def cfg3(device="cuda", precision: str = "f32_f16table", n_chan: int = 50,
         hours: float = 8.0) -> Workload:
    """4096^2 grid, cell 5e-6 rad, 50 channels of the same track generator (5.05e7
    visibilities); support 4..16 growing with |w|, 256 w-planes, oversampling 8."""
    spp = support_ramp(256, 4, 16)
    return _track_workload("cfg3", 3, 4096, 5e-6, n_chan, 1.0e9, 1.5e9, 256, 4, spp, 8,
                           precision, 50, device, hours=hours)


def cfg4(device="cuda", precision: str = "f32", n_images: int = 64,
         n_lo: float = 1e5, n_hi: float = 2e6) -> Workload:
    """64 channel images of 1024^2 (cell 7.5e-6 rad), one per channel over 1.0-1.5 GHz;
    per-channel visibility counts log-uniform in [n_lo, n_hi]; each channel's rows are a
    sorted random subset of its track rows (8 h at 5 s so that 2e6 rows exist);
    S=8, 64 w-planes, oversampling 8."""
    rng = np.random.default_rng(4)
    srng = np.random.default_rng(104)
    base, a1, a2 = array_tracks(rng, hours=8.0, dt_s=5.0)
    rows = base.reshape(-1, 3)
    n_rows = rows.shape[0]
    freqs = np.linspace(1.0e9, 1.5e9, n_images)
    counts = np.exp(rng.uniform(math.log(n_lo), math.log(n_hi), n_images)).astype(np.int64)
    counts = np.minimum(counts, n_rows)
    offsets = np.zeros(n_images + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(counts)
    parts = []
    for c in range(n_images):
        pick = np.sort(rng.choice(n_rows, size=int(counts[c]), replace=False))
        parts.append(torch.as_tensor(rows[pick] * (freqs[c] / C_LIGHT), device=device))
    uvw = torch.cat(parts).contiguous()
    n, cell = 1024, 7.5e-6
    l, m, flux = _sky(srng, 50, n * cell)
    vis = point_source_vis(uvw, l, m, flux, device=device)
    z = torch.as_tensor(srng.standard_normal((uvw.shape[0], 2)) * 0.01, device=device)
    vis += torch.complex(z[:, 0].contiguous(), z[:, 1].contiguous())
    w_max = float(uvw[:, 2].abs().max())
    m_img = kernel_image_size_rule(w_max, n * cell, 8, 8)
    params = _params(n, cell, 64, w_max, 8, 8, m_img, precision, None, n_images)
    weight = torch.ones(uvw.shape[0], dtype=torch.float64, device=device)
    return Workload("cfg4", params, uvw, vis, weight,
                    torch.as_tensor(offsets, device=device),
                    dict(l=l, m=m, flux=flux, freqs=freqs, counts=counts))


def cfg5_model_image(n: int = 2048, seed: int = 105, n_pts: int = 50, n_blobs: int = 10):
    """Sparse sky image: n_pts point sources (0.1-1 Jy on random pixels) plus n_blobs
    Gaussian blobs (sigma 2-10 px, peak 0.01-0.1), float64 [n, n] indexed [y][x]."""
    rng = np.random.default_rng(seed)
    img = np.zeros((n, n), dtype=np.float64)
    lo, hi = n // 8, n - n // 8
    ys = rng.integers(lo, hi, n_pts)
    xs = rng.integers(lo, hi, n_pts)
    np.add.at(img, (ys, xs), rng.uniform(0.1, 1.0, n_pts))
    yy = np.arange(n)[:, None]
    xx = np.arange(n)[None, :]
    for _ in range(n_blobs):
        cy, cx = rng.uniform(lo, hi, 2)
        s = rng.uniform(2.0, 10.0)
        a = rng.uniform(0.01, 0.1)
        r = int(6 * s) + 1
        y0, y1 = max(0, int(cy) - r), min(n, int(cy) + r + 1)
        x0, x1 = max(0, int(cx) - r), min(n, int(cx) + r + 1)
        img[y0:y1, x0:x1] += a * np.exp(
            -((yy[y0:y1] - cy) ** 2 + (xx[:, x0:x1] - cx) ** 2) / (2 * s * s))
    return img


def cfg5(device="cuda", precision: str = "f32", n_chan: int = 10) -> Workload:
    """Differentiable forward model workload: cfg2-shaped tracks with 10 channels over
    1.0-1.5 GHz (1.01e7 visibilities), 2048^2, S=8, 128 w-planes, oversampling 8.
    ``vis`` holds noise only (sigma 0.01); callers add the model prediction."""
    wl = _track_workload("cfg5", 5, 2048, 1e-5, n_chan, 1.0e9, 1.5e9, 128, 8, None, 8,
                         precision, 0, device, noise=0.01)
    wl.name = "cfg5"
    return wl


def small_tracks(n: int = 128, cell: float = 1.6e-4, n_chan: int = 4, hours: float = 1.0,
                 dt_s: float = 60.0, n_w: int = 9, support: int = 8, spp=None,
                 oversample: int = 8, precision: str = "f32", n_src: int = 5,
                 radius_m: float = 600.0, seed: int = 7, device="cpu",
                 m_img: Optional[int] = None) -> Workload:
    """A reduced track workload (same generator as the large configs) sized for tests."""
    wl = _track_workload("small_tracks", seed, n, cell, n_chan, 1.0e9, 1.5e9, n_w, support,
                         spp, oversample, precision, n_src, device, hours=hours, dt_s=dt_s,
                         radius_m=radius_m, m_img=m_img)
    return wl
