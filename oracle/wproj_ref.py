"""Plain FP64 w-projection imaging, step by step -- TEST INFRASTRUCTURE ONLY.

Only tests, the smoke check and the benchmark's CPU-baseline leg use this
module; the product library never does.

The paper (Lao et al. 2019, Sections 1-2) applies w-projection -- convolve each
visibility with a w-dependent kernel onto one uv-plane, then a 2D inverse FFT --
and cites Cornwell, Golap & Bhatnagar (2008) for the method instead of writing
it out.  The steps below are the standard formulation with each free choice
fixed explicitly:

  O0  FoV = N * cell; grid cell X <-> u = (X - N/2)/FoV; pixel x <-> l = (x - N/2) cell;
      arrays are [y][x] row-major with y <-> v <-> m.
  O1  w-planes w_p = -w_max + p dw, dw = 2 w_max/(N_w - 1), plane of w =
      clamp(floor((w + w_max)/dw + 1/2)); a single plane sits at w = 0.
      Hermitian fold (w_mode "fold" or "fold_sqrt"): a visibility with w < 0 is
      gridded as conj(V) at (-u, -v, -w), which leaves Re of the image unchanged
      (the two are Hermitian mirrors), so planes only cover [0, w_max]:
      "fold": w_p = p dw, dw = w_max/(N_w - 1), plane = clamp(floor(|w|/dw + 1/2));
      "fold_sqrt": w_p = w_max (p/(N_w - 1))^2, planes evenly spaced in sqrt|w|,
      plane = clamp(floor(sqrt(|w|/w_max) (N_w - 1) + 1/2)).  Degridding a folded row
      returns conj of the value degridded at (-u, -v, -w), the real-linear adjoint.
      w-stacking hybrid (w_mode "stack", n_wlayers = L): the w range is cut into L layers
      of width D = 2 w_max/L centred at w_l = -w_max + (l + 1/2) D, layer of w =
      clamp(floor((w + w_max)/D)); each layer has its own grid, and a visibility is
      gridded onto its layer's grid with the w-projection kernel of its residual
      w - w_l, whose N_w planes are linear over [-D/2, D/2] (dw = D/(N_w - 1), plane =
      clamp(floor((w - w_l + D/2)/dw + 1/2))).  Grids are [n_images L][N][N], layer
      fastest.  The image sums the layers' centred inverse DFTs, each multiplied by
      exp(+2 pi i w_l (n - 1)), n = sqrt(1 - l^2 - m^2) at the pixel (0 where
      l^2 + m^2 >= 1), before the real part and the correction (O7); the adjoint
      (O8) multiplies the corrected image by the conjugate factor before each layer's
      forward DFT.  One layer is the linear layout exactly.
  O2  taper psi = normalised prolate spheroidal function, c = pi S/2 (pswf.py).
  O3  kernel table of plane p: the Fourier transform of psi(l) psi(m) times the
      w phase screen exp(+2 pi i w_p (sqrt(1-l^2-m^2) - 1)), sampled at m x m
      cell-centred image points and evaluated at uv offsets a/O cells,
      a in (-S_p O/2, S_p O/2]; each of the O^2 S_p x S_p sub-kernels is divided
      by its complex sum.
  O4  per visibility: g = u FoV + N/2, q = floor(g O + 1/2),
      x0 = floor((q - S_p O/2)/O) + 1, ou = x0 O - q + S_p O/2 - 1 (same on v);
      a footprint leaving the grid drops the visibility.
  O5  grid[y0+kv][x0+ku] += W V T_p[ov][ou][kv][ku];  sumW += W.
  O6  centred unnormalised inverse DFT of the grid.
  O7  image = Re(.) kappa(x) kappa(y) / sumW, kappa = 1/psi((x - N/2)/(N/2)) inside
      |nu| < 1 and 0 on the edge pixel.
  O8  model image -> grid: centred unnormalised forward DFT of kappa kappa I.
  O9  degrid: V = sum_taps conj(T) M;  chi^2 gradient = -2 Re(kappa kappa F+(grid(W r))).

Visibilities with weight 0 are skipped; negative or non-finite weights are
skipped and counted; non-finite uvw or off-grid footprints are dropped and
counted; |w| > w_max (with more than one plane) is clamped to the edge plane
and counted.
"""

from __future__ import annotations

import math

import numpy as np

from . import pswf

PRECISIONS = ("f64", "f32", "f32_f16table")
W_MODES = ("linear", "fold", "fold_sqrt", "stack")


class Plan:
    """Derived quantities of a parameter block (the C-ABI's wproj_params)."""

    def __init__(self, params: dict):
        self.n = int(params["n"])
        self.cell = float(params["cell_rad"])
        self.n_w = int(params["n_wplanes"])
        self.w_max = float(params["w_max"])
        self.support = int(params["support"])
        spp = params.get("support_per_plane")
        self.supports = [int(s) for s in spp] if spp is not None else [self.support] * self.n_w
        self.O = int(params["oversample"])
        self.m = int(params["kernel_image_size"])
        self.n_images = int(params.get("n_images", 1))
        wm = params.get("w_mode", "linear")
        self.w_mode = W_MODES[wm] if isinstance(wm, (int, np.integer)) and 0 <= wm < 4 else wm
        self.n_layers = int(params.get("n_wlayers", 1)) if self.w_mode == "stack" else 1
        self.validate()
        self.fov = float(self.n) * self.cell
        self.fold = self.w_mode in ("fold", "fold_sqrt")
        self.n_grids = self.n_images * self.n_layers
        if self.w_mode == "stack":
            self.layer_w = (2.0 * self.w_max) / float(self.n_layers)
            self.w_layers = np.array([-self.w_max + (l + 0.5) * self.layer_w for l in range(self.n_layers)])
            half = self.layer_w / 2.0
            self.dw = self.layer_w / float(self.n_w - 1) if self.n_w > 1 else 0.0
            self.w_planes = (np.array([-half + p * self.dw for p in range(self.n_w)]) if self.n_w > 1
                             else np.zeros(1))
        elif self.n_w == 1:
            self.dw = 0.0
            self.w_planes = np.zeros(1)
        elif self.w_mode == "linear":
            self.dw = (2.0 * self.w_max) / float(self.n_w - 1)
            self.w_planes = np.array([-self.w_max + p * self.dw for p in range(self.n_w)])
        elif self.w_mode == "fold":
            self.dw = self.w_max / float(self.n_w - 1)
            self.w_planes = np.array([p * self.dw for p in range(self.n_w)])
        else:
            self.dw = 0.0
            self.w_planes = np.array([self.w_max * (p / float(self.n_w - 1)) ** 2
                                      for p in range(self.n_w)])

    def validate(self):
        n, O = self.n, self.O
        ok = (
            2 <= n <= 32768 and n % 2 == 0
            and math.isfinite(self.cell) and self.cell > 0 and n * self.cell < 2.0
            and 1 <= self.n_w <= 4096
            and math.isfinite(self.w_max) and self.w_max >= 0
            and (self.n_w == 1 or self.w_max > 0)
            and 1 <= self.support <= 32
            and len(self.supports) == self.n_w
            and 1 <= O <= 256
            and 2 <= self.m <= 4096 and self.m % 2 == 0
            and self.n_images >= 1
            and self.w_mode in W_MODES
            and 1 <= self.n_layers <= 4096
            and (self.w_mode != "stack" or self.w_max > 0)
        )
        ok = ok and all(1 <= s <= 32 and s <= n and (s * O) % 2 == 0 for s in self.supports)
        if not ok:
            raise ValueError("invalid w-projection parameters")


# ---------------------------------------------------------------------------
# O1 / O4: w-plane and footprint of each visibility
# ---------------------------------------------------------------------------


def plane_index(plan: Plan, w: np.ndarray) -> np.ndarray:
    """O1: nearest plane, rounding half up, clamped to [0, N_w - 1].  With a Hermitian
    fold, w is the folded (non-negative) coordinate."""
    w = np.asarray(w, dtype=np.float64)
    if plan.n_w == 1:
        return np.zeros(w.shape, dtype=np.int64)
    if plan.w_mode == "linear":
        t = np.floor((w + plan.w_max) / plan.dw + 0.5)
    elif plan.w_mode == "stack":  # w is the residual w - w_l
        t = np.floor((w + plan.layer_w / 2.0) / plan.dw + 0.5)
    elif plan.w_mode == "fold":
        t = np.floor(w / plan.dw + 0.5)
    else:
        t = np.floor(np.sqrt(w / plan.w_max) * float(plan.n_w - 1) + 0.5)
    t = np.clip(np.nan_to_num(t, nan=0.0), 0, plan.n_w - 1)
    return t.astype(np.int64)


def layer_index(plan: Plan, w: np.ndarray) -> np.ndarray:
    """w-stacking: the layer of w, floor((w + w_max)/D) clamped to [0, L - 1]."""
    w = np.asarray(w, dtype=np.float64)
    if plan.n_layers == 1:
        return np.zeros(w.shape, dtype=np.int64)
    t = np.floor((w + plan.w_max) / plan.layer_w)
    t = np.clip(np.nan_to_num(t, nan=0.0), 0, plan.n_layers - 1)
    return t.astype(np.int64)


def axis_footprint(plan: Plan, coord: np.ndarray, supp: np.ndarray):
    """O4 on one axis: (first cell x0, oversample index ou, on-grid flag).

    g = coord FoV + N/2 (cells), q = floor(g O + 1/2) (1/O-cell lattice),
    x0 = floor((q - S O/2)/O) + 1, a0 = x0 O - q, ou = a0 + S O/2 - 1.
    The footprint is the S cells whose centres lie in (q/O - S/2, q/O + S/2].
    """
    O = plan.O
    g = coord * plan.fov + plan.n / 2.0
    qd = np.floor(g * O + 0.5)
    finite = np.isfinite(qd) & (np.abs(qd) < 1e15)
    q = np.where(finite, qd, 0.0).astype(np.int64)
    half = supp * O // 2
    x0 = (q - half) // O + 1  # numpy // on int64 is floor division
    ou = x0 * O - q + half - 1
    on = finite & (x0 >= 0) & (x0 + supp <= plan.n)
    return x0, ou, on


def snap(plan: Plan, uvw: np.ndarray, weight: np.ndarray):
    """Per-visibility geometry and validity.

    Returns dict with x0, y0, ou, ov, p (int64 arrays), valid (bool), fold (bool: the
    row was mirrored to (-u, -v, -w) and its visibility is conjugated), layer (int64:
    the w-stacking layer, 0 otherwise), and the counters [dropped (non-finite uvw or
    off-grid), w clamped, bad weight].
    """
    uvw = np.asarray(uvw, dtype=np.float64)
    wt = np.asarray(weight, dtype=np.float64)
    flagged = wt == 0.0
    bad_w = ~flagged & ~(np.isfinite(wt) & (wt > 0.0))
    consider = ~flagged & ~bad_w
    fin = np.isfinite(uvw).all(axis=1)
    fold = fin & (uvw[:, 2] < 0.0) if plan.fold else np.zeros(fin.shape, dtype=bool)
    sgn = np.where(fold, -1.0, 1.0)
    u = np.where(fin, uvw[:, 0] * sgn, 0.0)
    v = np.where(fin, uvw[:, 1] * sgn, 0.0)
    w = np.where(fin, uvw[:, 2] * sgn, 0.0)
    if plan.w_mode == "stack":
        layer = layer_index(plan, w)
        w = w - (-plan.w_max + (layer + 0.5) * plan.layer_w)  # residual from the layer centre
    else:
        layer = np.zeros(w.shape, dtype=np.int64)
    p = plane_index(plan, w)
    supp = np.asarray(plan.supports, dtype=np.int64)[p]
    x0, ou, onx = axis_footprint(plan, u, supp)
    y0, ov, ony = axis_footprint(plan, v, supp)
    valid = consider & fin & onx & ony
    dropped = consider & ~valid
    if plan.n_w > 1 or plan.n_layers > 1:
        clamped = valid & (np.abs(uvw[:, 2]) > plan.w_max)
    else:
        clamped = np.zeros_like(valid)
    counters = np.array([dropped.sum(), clamped.sum(), bad_w.sum()], dtype=np.int64)
    return dict(x0=x0, y0=y0, ou=ou, ov=ov, p=p, valid=valid, fold=fold & valid, layer=layer,
                counters=counters)


def degrid_valid(plan: Plan, uvw: np.ndarray):
    """Geometry for degridding: the same footprint rule, no weights involved."""
    g = snap(plan, uvw, np.ones(np.asarray(uvw).shape[0]))
    return g


# ---------------------------------------------------------------------------
# O2 / O3: taper and kernel tables
# ---------------------------------------------------------------------------


def image_samples(plan: Plan) -> np.ndarray:
    """nu_i = (2 i + 1 - m)/m: cell-centred, symmetric samples of [-1, 1]."""
    m = plan.m
    return (2.0 * np.arange(m) + 1.0 - m) / m


def screen(plan: Plan, p: int) -> np.ndarray:
    """s_p[j][i] = psi(nu_i) psi(nu_j) exp(+2 pi i w_p (sqrt(1 - l_i^2 - m_j^2) - 1)).

    j indexes m (y), i indexes l (x); samples with l^2 + m^2 >= 1 are zero.
    """
    nu = image_samples(plan)
    lmax = plan.fov / 2.0
    lv = nu * lmax
    ps = pswf.taper(plan.support, nu)
    r2 = lv[None, :] ** 2 + lv[:, None] ** 2
    inside = r2 < 1.0
    nterm = np.sqrt(np.where(inside, 1.0 - r2, 1.0)) - 1.0
    s = ps[None, :] * ps[:, None] * np.exp(2j * np.pi * plan.w_planes[p] * nterm)
    return np.where(inside, s, 0.0)


def dft_matrix(plan: Plan, supp: int) -> np.ndarray:
    """E[a, i] = exp(-2 pi i a (i + 1/2 - m/2) / (O m)) for a in (-S O/2, S O/2].

    Row r holds a = r + 1 - S O/2.  Since (i + 1/2 - m/2)/m = nu_i/2 = l_i/FoV, the
    phase equals -2 pi u l_i at the uv offset u = a/(O FoV), i.e. a/O cells.
    """
    O, m = plan.O, plan.m
    a = np.arange(supp * O) + 1 - supp * O // 2
    i = np.arange(m)
    return np.exp(-2j * np.pi * np.outer(a, i + 0.5 - m / 2.0) / (O * m))


def raw_table(plan: Plan, p: int) -> np.ndarray:
    """C_p[b][a] = sum_j sum_i s_p[j][i] E[b, j] E[a, i]  (= E s_p E^T), un-normalised."""
    E = dft_matrix(plan, plan.supports[p])
    return E @ screen(plan, p) @ E.T


def kernel_tables(plan: Plan):
    """Normalised sub-kernels, one array per plane, shape [O][O][S_p][S_p] ([ov][ou][kv][ku]).

    Tap (kv, ku) of sub-kernel (ov, ou) is C_p[ov + kv O][ou + ku O]: row index
    r = ou + ku O corresponds to a = a0(ou) + ku O with a0(ou) = ou + 1 - S O/2.
    Each sub-kernel is divided by the complex sum of its taps.
    """
    O = plan.O
    out = []
    for p in range(plan.n_w):
        S = plan.supports[p]
        C = raw_table(plan, p)
        t = C.reshape(S, O, S, O).transpose(1, 3, 0, 2)  # [ov][ou][kv][ku]
        t = t / t.sum(axis=(2, 3), keepdims=True)
        out.append(np.ascontiguousarray(t))
    return out


def flat_tables(tables):
    """Concatenate per-plane tables: (complex128 flat array, int64 tap offset per plane)."""
    offs = np.zeros(len(tables) + 1, dtype=np.int64)
    for p, t in enumerate(tables):
        offs[p + 1] = offs[p] + t.size
    return np.concatenate([t.ravel() for t in tables]), offs


def kappa(plan: Plan) -> np.ndarray:
    """O7: kappa(x) = 1/psi(nu_x), nu_x = (x - N/2)/(N/2), and 0 where |nu_x| >= 1."""
    n = plan.n
    nu = (np.arange(n) - n / 2.0) / (n / 2.0)
    ps = pswf.taper(plan.support, nu)
    out = np.zeros(n)
    inner = np.abs(nu) < 1.0
    out[inner] = 1.0 / ps[inner]
    return out


# ---------------------------------------------------------------------------
# O5: gridding
# ---------------------------------------------------------------------------


def _image_ranges(plan: Plan, nvis: int, image_offsets):
    if image_offsets is None:
        return [(0, nvis)]
    off = np.asarray(image_offsets, dtype=np.int64)
    return [(int(off[i]), int(off[i + 1])) for i in range(plan.n_images)]


def grid(plan: Plan, tables, uvw, vis, weight, image_offsets=None):
    """O5: returns (grid complex128 [n_images L][N][N], sumW [n_images], counters[3]);
    L = 1 except with w-stacking, where row j goes to grid img L + layer_j."""
    uvw = np.asarray(uvw, dtype=np.float64)
    vis = np.asarray(vis, dtype=np.complex128)
    weight = np.asarray(weight, dtype=np.float64)
    n = plan.n
    G = np.zeros((plan.n_grids, n, n), dtype=np.complex128)
    sumw = np.zeros(plan.n_images)
    counters = np.zeros(3, dtype=np.int64)
    for img, (s, e) in enumerate(_image_ranges(plan, uvw.shape[0], image_offsets)):
        geo = snap(plan, uvw[s:e], weight[s:e])
        counters += geo["counters"]
        val = geo["valid"]
        wv = weight[s:e] * np.where(geo["fold"], np.conj(vis[s:e]), vis[s:e])
        sumw[img] = weight[s:e][val].sum()
        for p in np.unique(geo["p"][val]):
            sel = val & (geo["p"] == p)
            T = tables[p]
            S = T.shape[-1]
            x0, y0 = geo["x0"][sel], geo["y0"][sel]
            ou, ov = geo["ou"][sel], geo["ov"][sel]
            gi = img * plan.n_layers + geo["layer"][sel]
            a = wv[sel]
            for kv in range(S):
                for ku in range(S):
                    np.add.at(G, (gi, y0 + kv, x0 + ku), a * T[ov, ou, kv, ku])
    return G, sumw, counters


# ---------------------------------------------------------------------------
# O6 / O7 / O8: transforms and correction
# ---------------------------------------------------------------------------


def grid_cells(plan: Plan, tables, uvw, vis, weight):
    """O5 for one image, kept sparse: the touched cells as (flat index y N + x, value).

    Same contributions as grid() (W V T_p[ov][ou][kv][ku] at cell (y0 + kv, x0 + ku)),
    summed per cell; for grids too large to hold densely on the host.
    Returns (cells int64 sorted, values complex128, sumW, counters[3]).
    """
    if plan.n_layers != 1:
        raise ValueError("grid_cells covers one grid per image (no w-stacking layers)")
    uvw = np.asarray(uvw, dtype=np.float64)
    geo = snap(plan, uvw, weight)
    vis = np.asarray(vis, dtype=np.complex128)
    wv = np.asarray(weight, dtype=np.float64) * np.where(geo["fold"], np.conj(vis), vis)
    val = geo["valid"]
    idx, con = [], []
    for p in np.unique(geo["p"][val]):
        sel = val & (geo["p"] == p)
        T = tables[p]
        S = T.shape[-1]
        x0, y0 = geo["x0"][sel], geo["y0"][sel]
        ou, ov = geo["ou"][sel], geo["ov"][sel]
        a = wv[sel]
        for kv in range(S):
            for ku in range(S):
                idx.append((y0 + kv) * plan.n + (x0 + ku))
                con.append(a * T[ov, ou, kv, ku])
    if not idx:
        return (np.zeros(0, np.int64), np.zeros(0, np.complex128),
                float(np.asarray(weight)[val].sum()), geo["counters"])
    idx = np.concatenate(idx)
    con = np.concatenate(con)
    cells, inv = np.unique(idx, return_inverse=True)
    vals = np.zeros(cells.shape[0], dtype=np.complex128)
    np.add.at(vals, inv, con)
    return cells, vals, float(np.asarray(weight, dtype=np.float64)[val].sum()), geo["counters"]


def image_pixels(plan: Plan, cells, vals, sumw, ys, xs):
    """O6 + O7 at chosen pixels, from a sparse grid: kappa(x) kappa(y) Re(sum over cells of
    G[Y][X] exp(+2 pi i ((X - N/2)(x - N/2) + (Y - N/2)(y - N/2))/N)) / sumW."""
    n = plan.n
    k = kappa(plan)
    Y = (np.asarray(cells) // n - n // 2).astype(np.float64)
    X = (np.asarray(cells) % n - n // 2).astype(np.float64)
    out = np.empty(len(ys))
    for i, (y, x) in enumerate(zip(ys, xs)):
        ph = 2.0 * np.pi * (X * (x - n // 2) + Y * (y - n // 2)) / n
        out[i] = np.sum(vals * np.exp(1j * ph)).real * k[x] * k[y] / sumw
    return out


def centred_idft(grid2d: np.ndarray) -> np.ndarray:
    """O6: out[y][x] = sum_{Y,X} G[Y][X] exp(+2 pi i ((X-N/2)(x-N/2) + (Y-N/2)(y-N/2))/N)."""
    n = grid2d.shape[-1]
    return np.fft.fftshift(np.fft.ifft2(np.fft.ifftshift(grid2d, axes=(-2, -1))), axes=(-2, -1)) * (n * n)


def centred_dft(img: np.ndarray) -> np.ndarray:
    """O8's transform: out[Y][X] = sum_{y,x} I[y][x] exp(-2 pi i ((X-N/2)(x-N/2) + (Y-N/2)(y-N/2))/N)."""
    return np.fft.fftshift(np.fft.fft2(np.fft.ifftshift(img, axes=(-2, -1))), axes=(-2, -1))


def layer_phase(plan: Plan, layer: int) -> np.ndarray:
    """w-stacking: exp(+2 pi i w_l (sqrt(1 - l^2 - m^2) - 1)) at every pixel [y][x],
    l = (x - N/2) cell, m = (y - N/2) cell; 0 where l^2 + m^2 >= 1."""
    n = plan.n
    lv = (np.arange(n) - n / 2.0) * plan.cell
    r2 = lv[None, :] ** 2 + lv[:, None] ** 2
    inside = r2 < 1.0
    nterm = np.sqrt(np.where(inside, 1.0 - r2, 1.0)) - 1.0
    return np.where(inside, np.exp(2j * np.pi * plan.w_layers[layer] * nterm), 0.0)


def grid_to_image(plan: Plan, G: np.ndarray, sumw=None) -> np.ndarray:
    """O6 + O7: real image kappa(x) kappa(y) Re(IDFT(G)) / sumW (sumW omitted if None).
    With w-stacking, Re of the sum over layers of IDFT(G_l) times the layer's phase."""
    k = kappa(plan)
    if plan.w_mode == "stack":
        L = plan.n_layers
        G = np.asarray(G).reshape(-1, L, plan.n, plan.n)
        acc = np.zeros((G.shape[0], plan.n, plan.n), dtype=np.complex128)
        for l in range(L):
            acc += centred_idft(G[:, l]) * layer_phase(plan, l)
        img = acc.real * (k[None, :] * k[:, None])
    else:
        img = centred_idft(G).real * (k[None, :] * k[:, None])
    if sumw is not None:
        img = img / np.asarray(sumw, dtype=np.float64).reshape(-1, 1, 1)
    return img


def image_to_grid(plan: Plan, img: np.ndarray) -> np.ndarray:
    """O8: M = DFT(kappa kappa I), complex128, same leading shape as img.  With w-stacking,
    layer l's grid is DFT(kappa kappa I conj(phase_l)): [n_images L][N][N]."""
    k = kappa(plan)
    corr = np.asarray(img, dtype=np.float64) * (k[None, :] * k[:, None])
    if plan.w_mode != "stack":
        return centred_dft(corr)
    corr = corr.reshape(-1, plan.n, plan.n)
    out = np.empty((corr.shape[0], plan.n_layers, plan.n, plan.n), dtype=np.complex128)
    for l in range(plan.n_layers):
        out[:, l] = centred_dft(corr * np.conj(layer_phase(plan, l)))
    return out.reshape(-1, plan.n, plan.n)


# ---------------------------------------------------------------------------
# O9: degridding and the chi^2 gradient
# ---------------------------------------------------------------------------


def degrid(plan: Plan, tables, uvw, M, image_offsets=None):
    """V_j = sum_{kv,ku} conj(T_p[ov][ou][kv][ku]) M[y0+kv][x0+ku]; 0 for dropped rows."""
    uvw = np.asarray(uvw, dtype=np.float64)
    M = np.asarray(M, dtype=np.complex128).reshape(plan.n_grids, plan.n, plan.n)
    out = np.zeros(uvw.shape[0], dtype=np.complex128)
    for img, (s, e) in enumerate(_image_ranges(plan, uvw.shape[0], image_offsets)):
        geo = degrid_valid(plan, uvw[s:e])
        val = geo["valid"]
        acc = np.zeros(e - s, dtype=np.complex128)
        for p in np.unique(geo["p"][val]):
            sel = val & (geo["p"] == p)
            T = tables[p]
            S = T.shape[-1]
            x0, y0 = geo["x0"][sel], geo["y0"][sel]
            ou, ov = geo["ou"][sel], geo["ov"][sel]
            gi = img * plan.n_layers + geo["layer"][sel]
            v = np.zeros(sel.sum(), dtype=np.complex128)
            for kv in range(S):
                for ku in range(S):
                    v += np.conj(T[ov, ou, kv, ku]) * M[gi, y0 + kv, x0 + ku]
            acc[sel] = v
        # a folded row was degridded at (-u, -v, -w): its value is the conjugate
        out[s:e] = np.where(geo["fold"], np.conj(acc), acc)
    return out


def predict(plan: Plan, tables, uvw, img, image_offsets=None):
    """Forward model A(I) = degrid(image_to_grid(I))."""
    return degrid(plan, tables, uvw, image_to_grid(plan, img), image_offsets)


def chi2(plan: Plan, tables, uvw, vis_obs, weight, img, image_offsets=None) -> float:
    r = np.asarray(vis_obs) - predict(plan, tables, uvw, img, image_offsets)
    return float(np.sum(np.asarray(weight) * np.abs(r) ** 2))


def chi2_grad(plan: Plan, tables, uvw, vis_obs, weight, img, image_offsets=None):
    """O9: d chi^2 / dI = -2 Re(kappa kappa IDFT(grid of W r)), r = V_obs - A(I)."""
    r = np.asarray(vis_obs) - predict(plan, tables, uvw, img, image_offsets)
    G, _, _ = grid(plan, tables, uvw, r, weight, image_offsets)
    return -2.0 * grid_to_image(plan, G, None)
