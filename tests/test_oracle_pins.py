"""Pins of the FP64 oracle against facts it does not compute itself.

Each test checks the oracle against an independent statement: a library
routine for a special case, a brute-force sum, an exact identity of the
method, a convergence law, or hand-derived worked values.  A dropped term, a
wrong sign or index, or a transposed operand in the oracle fails at least one.
"""

import math
import os

import numpy as np
import pytest
import scipy.special as sps

import synth
from oracle import cref, eq56, pswf
from oracle import wproj_ref as R

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _direct_dft_image(plan, uvw, vis, wt, valid):
    """Brute-force dirty image with the w term:
    I(x,y) = sum_j W_j Re[V_j exp(+2 pi i (u l + v m + w (n - 1)))] / sum_j W_j."""
    n = plan.n
    x = (np.arange(n) - n / 2.0) * plan.cell
    L = x[None, :]
    M = x[:, None]
    Nn = np.sqrt(1.0 - L * L - M * M) - 1.0
    u, V, W = uvw[valid], vis[valid], wt[valid]
    out = np.zeros((n, n))
    for j in range(u.shape[0]):
        out += W[j] * np.real(V[j] * np.exp(2j * np.pi * (u[j, 0] * L + u[j, 1] * M + u[j, 2] * Nn)))
    return out / W.sum()


def _wproj_image(wl):
    plan = R.Plan(wl.params)
    tabs = R.kernel_tables(plan)
    G, sw, _ = R.grid(plan, tabs, wl.uvw, wl.vis, wl.weight)
    return plan, R.grid_to_image(plan, G, sw)[0]


# --------------------------------------------------------------------------- taper


@pytest.mark.parametrize("S", [4, 7, 8, 9, 16])
def test_taper_matches_scipy_prolate(S):
    c = math.pi * S / 2.0
    x = np.linspace(-0.995, 0.995, 57)
    ref = np.array([sps.pro_ang1(0, 0, c, xx)[0] for xx in x]) / sps.pro_ang1(0, 0, c, 0.0)[0]
    assert np.abs(pswf.taper(S, x) - ref).max() < 1e-8


def test_taper_support_and_eigen_relation():
    # Outside [-1, 1] the taper is zero; psi_0 is the eigenfunction of the
    # band-limited Fourier transform: int_{-1}^{1} exp(i c x t) psi(t) dt = lam psi(x).
    S = 8
    c = math.pi * S / 2
    assert pswf.taper(S, [1.5, -2.0]).tolist() == [0.0, 0.0]
    t, wq = np.polynomial.legendre.leggauss(200)
    pt = pswf.taper(S, t)
    lam = np.sum(wq * pt)  # x = 0
    for x in (0.3, 0.7, 0.95):
        lhs = np.sum(wq * np.exp(1j * c * x * t) * pt)
        assert abs(lhs - lam * pswf.taper(S, [x])[0]) < 1e-12 * abs(lam)


# --------------------------------------------------------------------------- indexing


def test_worked_index_examples():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "index_examples.txt"))
            if l.strip() and not l.startswith("#")]
    for S, g, q, x0, last, off0, off1, ou in rows:
        S, q, x0, last, ou = int(S), int(q), int(x0), int(last), int(ou)
        g, off0, off1 = float(g), float(off0), float(off1)
        plan = R.Plan(dict(n=64, cell_rad=1e-3, n_wplanes=1, w_max=0.0, support=S,
                           oversample=8, kernel_image_size=32))
        coord = (g - plan.n / 2.0) / plan.fov
        a, o, on = R.axis_footprint(plan, np.array([coord]), np.array([S]))
        assert on[0] and a[0] == x0 and o[0] == ou
        assert x0 + S - 1 == last
        assert x0 - q / 8.0 == off0 and last - q / 8.0 == off1


def test_footprint_brute_force():
    # Enumerate the cells whose centres lie in (q/O - S/2, q/O + S/2] directly.
    rng = np.random.default_rng(0)
    for S in (3, 4, 7, 8, 9, 12):
        for O in (1, 2, 4, 8):
            if (S * O) % 2:
                continue
            plan = R.Plan(dict(n=64, cell_rad=1e-3, n_wplanes=1, w_max=0.0, support=S,
                               oversample=O, kernel_image_size=32))
            g = rng.uniform(-4.0, 68.0, 300)
            coord = (g - 32.0) / plan.fov
            x0, ou, on = R.axis_footprint(plan, coord, np.full(g.shape, S))
            for k in range(g.size):
                gg = coord[k] * plan.fov + 32.0
                q = math.floor(gg * O + 0.5)
                cells = [X for X in range(-40, 120) if q / O - S / 2 < X <= q / O + S / 2]
                assert len(cells) == S
                assert x0[k] == cells[0]
                a = cells[0] * O - q  # first tap offset in 1/O cells
                assert ou[k] == a + S * O // 2 - 1 and 0 <= ou[k] < O
                assert on[k] == (cells[0] >= 0 and cells[-1] <= 63)


def test_plane_assignment_and_counters():
    plan = R.Plan(dict(n=64, cell_rad=1e-3, n_wplanes=5, w_max=100.0, support=4,
                       oversample=4, kernel_image_size=16))
    # planes at -100, -50, 0, 50, 100; ties round up
    w = np.array([-100.0, -76.0, -75.0, -25.0, 0.0, 24.9, 25.0, 100.0, 130.0, -400.0])
    assert R.plane_index(plan, w).tolist() == [0, 0, 1, 2, 2, 2, 3, 4, 4, 0]
    uvw = np.zeros((7, 3))
    uvw[1, 0] = np.nan  # dropped
    uvw[2, 0] = 1e9  # off grid
    uvw[3, 2] = 150.0  # clamped
    wt = np.array([1.0, 1.0, 1.0, 1.0, 0.0, -1.0, np.nan])
    g = R.snap(plan, uvw, wt)
    assert g["valid"].tolist() == [True, False, False, True, False, False, False]
    assert g["counters"].tolist() == [2, 1, 2]


def test_params_validation():
    good = dict(n=64, cell_rad=1e-3, n_wplanes=3, w_max=10.0, support=7, oversample=8,
                kernel_image_size=32)
    R.Plan(good)
    for bad in (dict(n=63), dict(n=0), dict(cell_rad=-1.0), dict(cell_rad=0.1),
                dict(n_wplanes=0), dict(w_max=-1.0), dict(oversample=0),
                dict(support=7, oversample=1), dict(kernel_image_size=31),
                dict(support_per_plane=[7, 7]), dict(n_wplanes=3, w_max=0.0)):
        with pytest.raises(ValueError):
            R.Plan({**good, **bad})


# --------------------------------------------------------------------------- tables


def test_subkernel_sums_and_conjugate_planes():
    wl = synth.cfg1w()
    plan = R.Plan(wl.params)
    tabs = R.kernel_tables(plan)
    for t in tabs:
        assert np.abs(t.sum(axis=(2, 3)) - 1.0).max() < 1e-13
    # symmetric planes: w_p = -w_{N_w-1-p}, so the tables are complex conjugates
    for p in range(plan.n_w):
        q = plan.n_w - 1 - p
        assert np.abs(tabs[p] - np.conj(tabs[q])).max() < 1e-12


def test_raw_table_mirror_symmetries():
    wl = synth.cfg1w()
    plan = R.Plan(wl.params)
    for p in (0, 5, 16):
        C = R.raw_table(plan, p)  # [b][a], row r <-> a = r + 1 - S O/2
        # a -> -a maps row r to row S O - 2 - r (a = S O/2 has no mirror: drop the last row)
        inner = C[:-1, :-1]
        assert np.abs(C - C.T).max() < 1e-12 * np.abs(C).max()
        assert np.abs(inner - inner[::-1, :]).max() < 1e-12 * np.abs(C).max()


@pytest.mark.parametrize("m_img,tol", [(16, 2e-5), (32, 5e-6), (64, 1.5e-6), (128, 4e-7)])
def test_w0_table_is_separable_prolate(m_img, tol):
    # With w = 0 the screen is psi(l) psi(m): the table is real, even and rank one,
    # and by the finite-Fourier eigen-relation c(a)/c(0) -> psi(2a/(S O)) as m grows
    # (midpoint rule, error ~ m^-2).
    S, O = 8, 8
    plan = R.Plan(dict(n=64, cell_rad=1e-3, n_wplanes=1, w_max=0.0, support=S, oversample=O,
                       kernel_image_size=m_img))
    C = R.raw_table(plan, 0)
    assert np.abs(C.imag).max() < 1e-12 * np.abs(C).max()
    sv = np.linalg.svd(C.real, compute_uv=False)
    assert sv[1] / sv[0] < 1e-13
    mid = S * O // 2 - 1  # row of a = 0
    c1 = C.real[mid]
    a = np.arange(S * O) + 1 - S * O // 2
    ref = pswf.taper(S, 2.0 * a / (S * O))
    assert np.abs(c1 / c1[mid] - ref).max() < tol


def test_w0_gridding_equals_separable_gridder():
    # Plain separable gridder from 1D tables c(a) = sum_i psi(nu_i) E[a,i] built here.
    rng = np.random.default_rng(3)
    n, S, O, m = 64, 7, 8, 32
    plan = R.Plan(dict(n=n, cell_rad=1e-3, n_wplanes=1, w_max=0.0, support=S, oversample=O,
                       kernel_image_size=m))
    tabs = R.kernel_tables(plan)
    nv = 300
    uvw = np.zeros((nv, 3))
    uvw[:, 0] = rng.uniform(-20, 20, nv) / plan.fov
    uvw[:, 1] = rng.uniform(-20, 20, nv) / plan.fov
    vis = rng.standard_normal(nv) + 1j * rng.standard_normal(nv)
    wt = rng.uniform(0.5, 2.0, nv)
    G, _, _ = R.grid(plan, tabs, uvw, vis, wt)
    nu = (2.0 * np.arange(m) + 1.0 - m) / m
    ps = pswf.taper(S, nu)
    ref = np.zeros((n, n), dtype=complex)
    for j in range(nv):
        cell = []
        for ax in (0, 1):
            g = uvw[j, ax] * plan.fov + n / 2.0
            q = math.floor(g * O + 0.5)
            first = min(X for X in range(-2, n + 3) if q / O - S / 2 < X)
            offs = [(first + k) * O - q for k in range(S)]  # offsets in 1/O cells
            c = np.array([np.sum(ps * np.exp(-1j * np.pi * a * nu / O)) for a in offs])
            cell.append((first, c / c.sum()))
        (x0, cx), (y0, cy) = cell
        ref[y0:y0 + S, x0:x0 + S] += wt[j] * vis[j] * np.outer(cy, cx)
    assert np.abs(G[0] - ref).max() < 1e-12 * np.abs(ref).max()


# --------------------------------------------------------------------------- imaging


def test_unit_visibilities_image_to_exact_one_at_centre():
    wl = synth.cfg1()
    plan = R.Plan(wl.params)
    tabs = R.kernel_tables(plan)
    ones = np.ones(wl.nvis, dtype=complex)
    G, sw, _ = R.grid(plan, tabs, wl.uvw, ones, wl.weight)
    img = R.grid_to_image(plan, G, sw)[0]
    c = plan.n // 2
    assert abs(img[c, c] - 1.0) < 1e-12
    assert img.max() <= img[c, c] + 1e-12


def test_degrid_unit_delta_gives_unit_visibilities():
    wl = synth.cfg1w()
    plan = R.Plan(wl.params)
    tabs = R.kernel_tables(plan)
    delta = np.zeros((plan.n, plan.n))
    delta[plan.n // 2, plan.n // 2] = 1.0
    V = R.predict(plan, tabs, wl.uvw, delta)
    assert np.abs(V - 1.0).max() < 1e-13


def _inner_err(img, ref):
    n = img.shape[0]
    q = n // 4
    s = (slice(q, n - q), slice(q, n - q))
    return np.abs(img - ref)[s].max() / np.abs(ref).max()


def test_direct_dft_w_dominated_convergence():
    # The w-dominated tiny field: w-projection must beat ignoring w by a wide margin
    # and its error must fall as the plane count and oversampling grow.
    errs = {}
    for key, kw in {"w_ignored": dict(n_w=1), "nw33_o8": dict(n_w=33, oversample=8),
                    "nw33_o32": dict(n_w=33, oversample=32),
                    "nw65_o32": dict(n_w=65, oversample=32)}.items():
        wl = synth.cfg1w(**kw)
        plan, img = _wproj_image(wl)
        geo = R.snap(plan, wl.uvw, wl.weight)
        ref = _direct_dft_image(plan, wl.uvw, wl.vis, wl.weight, geo["valid"])
        errs[key] = _inner_err(img, ref)
    assert errs["w_ignored"] > 5e-2
    assert errs["nw33_o8"] < 6e-3
    assert errs["nw33_o32"] < errs["nw33_o8"]
    assert errs["nw65_o32"] < errs["nw33_o32"]


def test_direct_dft_cfg1_oversampling_law():
    # cfg1's w term is small (w FoV^2 ~ 0.08 cells), so the remaining error is the
    # nearest-sample snapping on the 1/O lattice: first order in 1/O.
    wl = synth.cfg1()
    errs = []
    for O in (8, 32, 64):
        sub = synth.Workload("s", {**wl.params, "oversample": O, "kernel_image_size": 32},
                             wl.uvw[:4000], wl.vis[:4000], wl.weight[:4000])
        plan, img = _wproj_image(sub)
        geo = R.snap(plan, sub.uvw, sub.weight)
        errs.append(_inner_err(img, _direct_dft_image(plan, sub.uvw, sub.vis, sub.weight,
                                                      geo["valid"])))
    assert errs[0] < 1e-2
    assert errs[1] < errs[0] / 3.0
    assert errs[2] < errs[1] / 1.6


def test_adjoint_identity_core_and_corrected():
    wl = synth.cfg1w()
    plan = R.Plan(wl.params)
    tabs = R.kernel_tables(plan)
    rng = np.random.default_rng(5)
    nv, n = wl.nvis, plan.n
    x = rng.standard_normal(nv) + 1j * rng.standard_normal(nv)
    y = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    W = rng.uniform(0.5, 2.0, nv)
    # core operator: G0 x = IDFT(grid(W x)), G0^H y = W degrid(DFT(y))
    Gx = R.centred_idft(R.grid(plan, tabs, wl.uvw, x, W)[0][0])
    GHy = W * R.degrid(plan, tabs, wl.uvw, R.centred_dft(y))
    lhs = np.vdot(Gx, y)
    rhs = np.vdot(x, GHy)
    assert abs(lhs - rhs) < 1e-13 * abs(lhs)
    # with the kappa correction and the real part (the imaging/prediction pair)
    yr = rng.standard_normal((n, n))
    img = R.grid_to_image(plan, R.grid(plan, tabs, wl.uvw, x, W)[0], None)[0]
    back = W * R.predict(plan, tabs, wl.uvw, yr)
    lhs = np.sum(img * yr)
    rhs = np.real(np.vdot(x, back))
    assert abs(lhs - rhs) < 1e-10 * np.linalg.norm(yr) * np.linalg.norm(img)


def test_linearity_permutation_chunking():
    wl = synth.cfg1()
    plan = R.Plan(wl.params)
    tabs = R.kernel_tables(plan)
    uvw, vis, wt = wl.uvw[:3000], wl.vis[:3000], wl.weight[:3000]
    G = R.grid(plan, tabs, uvw, vis, wt)[0]
    G2 = R.grid(plan, tabs, uvw, 2.0 * vis - 1j * vis, wt)[0]
    assert np.abs(G2 - (2.0 - 1j) * G).max() < 1e-13 * np.abs(G).max()
    perm = np.random.default_rng(1).permutation(3000)
    Gp = R.grid(plan, tabs, uvw[perm], vis[perm], wt[perm])[0]
    assert np.abs(Gp - G).max() < 1e-13 * np.abs(G).max()
    Ga = R.grid(plan, tabs, uvw[:1234], vis[:1234], wt[:1234])[0]
    Gb = R.grid(plan, tabs, uvw[1234:], vis[1234:], wt[1234:])[0]
    assert np.abs(Ga + Gb - G).max() < 1e-13 * np.abs(G).max()


def test_hermitian_consistency():
    # Gridding conj(V) at -uvw mirrors the grid through the centre and conjugates it,
    # so the real image is unchanged.  Positions are kept off the rounding ties where
    # the half-open footprint rule breaks the mirror symmetry.
    rng = np.random.default_rng(9)
    wl = synth.cfg1w()
    plan = R.Plan(wl.params)
    tabs = R.kernel_tables(plan)
    O = plan.O
    uvw = wl.uvw.copy()
    for ax in (0, 1):
        g = uvw[:, ax] * plan.fov + plan.n / 2
        frac = g * O - np.floor(g * O)
        uvw = uvw[np.abs(frac - 0.5) > 0.05]
    geo = R.snap(plan, uvw, np.ones(len(uvw)))
    keep = geo["valid"] & (geo["ou"] != O - 1) & (geo["ov"] != O - 1)
    uvw = uvw[keep]
    vis = rng.standard_normal(len(uvw)) + 1j * rng.standard_normal(len(uvw))
    wt = np.ones(len(uvw))
    G, sw, _ = R.grid(plan, tabs, uvw, vis, wt)
    Gm, swm, _ = R.grid(plan, tabs, -uvw, np.conj(vis), wt)
    n = plan.n
    # cell X <-> N - X
    mirror = np.conj(Gm[0][::-1, ::-1])
    assert np.abs(mirror[:n - 1, :n - 1] - G[0][1:, 1:]).max() < 1e-12 * np.abs(G).max()
    a = R.grid_to_image(plan, G, sw)[0]
    b = R.grid_to_image(plan, Gm, swm)[0]
    # the edge correction kappa^2 amplifies rounding by ~1e3 at the border: inner half
    assert _inner_err(b, a) < 1e-12


def test_chi2_gradient_finite_differences():
    wl = synth.cfg1w(n_vis=400)
    plan = R.Plan({**wl.params, "n": 32, "cell_rad": 2e-3})
    tabs = R.kernel_tables(plan)
    rng = np.random.default_rng(2)
    keep = R.snap(plan, wl.uvw, wl.weight)["valid"]
    uvw, vobs = wl.uvw[keep], wl.vis[keep]
    W = rng.uniform(0.5, 2.0, uvw.shape[0])
    img = rng.standard_normal((plan.n, plan.n)) * 0.01
    g = R.chi2_grad(plan, tabs, uvw, vobs, W, img)[0]
    for _ in range(20):
        y, x = rng.integers(1, plan.n, 2)
        h = 1e-4 * max(1.0, abs(img[y, x]))
        e = np.zeros_like(img)
        e[y, x] = h
        fd = (R.chi2(plan, tabs, uvw, vobs, W, img + e) - R.chi2(plan, tabs, uvw, vobs, W, img - e)) / (2 * h)
        assert abs(fd - g[y, x]) < 1e-6 * max(1.0, np.abs(g).max())


# --------------------------------------------------------------------------- C oracle


@pytest.mark.parametrize("nthreads", [1, 4])
def test_c_oracle_matches_numpy_oracle(nthreads):
    wl = synth.small_tracks(n=128, n_w=9, support=8, spp=None)
    uvw = wl.uvw.numpy()
    vis = wl.vis.numpy()
    wt = np.random.default_rng(4).uniform(0.0, 2.0, wl.nvis)
    wt[::7] = 0.0
    wt[3] = -1.0
    uvw[5, 1] = np.inf
    plan = R.Plan(wl.params)
    tabs = R.kernel_tables(plan)
    G, sw, cnt = R.grid(plan, tabs, uvw, vis, wt)
    Gc, swc, cntc = cref.grid(plan, tabs, uvw, vis, wt, nthreads=nthreads)
    assert np.abs(Gc - G).max() <= 1e-12 * np.abs(G).max()
    assert abs(swc[0] - sw[0]) <= 1e-12 * sw[0]
    assert cntc.tolist() == cnt.tolist()
    M = np.random.default_rng(6).standard_normal((1, plan.n, plan.n)) + 0j
    assert np.abs(cref.degrid(plan, tabs, uvw, M, nthreads=nthreads)
                  - R.degrid(plan, tabs, uvw, M)).max() < 1e-12 * np.abs(M).max()


def test_c_oracle_multi_image_and_variable_support():
    wl = synth.cfg1w(n_w=9, s_max=12)
    plan0 = R.Plan(wl.params)
    offs = np.array([0, 700, 700, 2000])
    plan = R.Plan({**wl.params, "n_images": 3})
    tabs = R.kernel_tables(plan0)
    G, sw, cnt = R.grid(plan, tabs, wl.uvw, wl.vis, wl.weight, offs)
    Gc, swc, cntc = cref.grid(plan, tabs, wl.uvw, wl.vis, wl.weight, offs, nthreads=3)
    assert np.abs(Gc - G).max() <= 1e-12 * np.abs(G).max()
    assert np.allclose(swc, sw, rtol=0, atol=1e-9) and cntc.tolist() == cnt.tolist()
    assert np.abs(G[1]).max() == 0.0


# --------------------------------------------------------------------------- Eq. 5 / Eq. 6


def test_eq5_bijection_small_and_vla():
    a1, a2 = np.triu_indices(3)
    assert eq56.baseline_index(a1, a2, 3).tolist() == [0, 1, 2, 3, 4, 5]
    a1, a2 = np.triu_indices(27)
    idx = eq56.baseline_index(a1, a2, 27)
    assert sorted(idx.tolist()) == list(range(27 * 28 // 2))
    # symmetric in the antenna order
    assert (eq56.baseline_index(a2, a1, 27) == idx).all()


def test_eq6_scan_and_regroup_match_brute_force():
    rng = np.random.default_rng(8)
    b = rng.integers(0, 40, 2000)
    c = eq56.counts(b, 40)
    assert c.tolist() == [int((b == k).sum()) for k in range(40)]
    s = eq56.start_index(c)
    assert s.tolist() == [int(c[:k].sum()) for k in range(40)]
    perm = eq56.regroup_order(b, 40)
    assert (perm == np.argsort(b, kind="stable")).all()


def test_channel_major_order_matches_lexicographic_sort():
    """The channel-major visibility order is the sort of (baseline, channel, time) with
    time the row's original position: checked against numpy's lexsort on a small case,
    with empty baselines and an uneven row count per baseline."""
    rng = np.random.default_rng(9)
    n_b, n_chan = 12, 5
    b = rng.integers(0, n_b, 300)
    b[b == 3] = 4  # baseline 3 has no rows
    perm = eq56.regroup_order(b, n_b)
    got = eq56.channel_major_order(perm, b, n_b, n_chan)
    rows = np.repeat(np.arange(len(b)), n_chan)
    chans = np.tile(np.arange(n_chan), len(b))
    want = np.lexsort((rows, chans, b[rows]))  # last key is the primary one
    assert got.tolist() == want.tolist()
    assert sorted(got.tolist()) == list(range(len(b) * n_chan))


# --------------------------------------------------------------------------- sparse forms
def test_sparse_grid_and_pixel_image_match_dense_forms():
    """grid_cells (the touched cells only, for grids too large for the host) holds exactly
    the dense grid's non-zero cells; image_pixels (a direct sum per pixel) matches the
    FFT-based image on the inner half (the edge kappa^2 ~1e7 amplifies FFT rounding)."""
    wl = synth.cfg1()
    plan = R.Plan(wl.params)
    tabs = R.kernel_tables(plan)
    uvw, vis, wt = (np.asarray(a) for a in (wl.uvw, wl.vis, wl.weight))
    G, sw, c = R.grid(plan, tabs, uvw, vis, wt)
    cells, vals, sw2, c2 = R.grid_cells(plan, tabs, uvw, vis, wt)
    dense = np.zeros(plan.n * plan.n, dtype=np.complex128)
    dense[cells] = vals
    assert np.array_equal(dense, G[0].ravel())
    assert np.count_nonzero(G[0]) == np.count_nonzero(vals)
    assert sw2 == sw[0] and c2.tolist() == c.tolist()
    img = R.grid_to_image(plan, G, sw)[0]
    rng = np.random.default_rng(0)
    n = plan.n
    ys = rng.integers(n // 4, 3 * n // 4, 40)
    xs = rng.integers(n // 4, 3 * n // 4, 40)
    pix = R.image_pixels(plan, cells, vals, sw2, ys, xs)
    assert np.abs(pix - img[ys, xs]).max() <= 1e-14 * np.abs(img).max()


# --------------------------------------------------------------------------- Hermitian fold


def _fold_plan(mode, n_w=5, w_max=100.0):
    return R.Plan(dict(n=64, cell_rad=1e-3, n_wplanes=n_w, w_max=w_max, support=4, oversample=4,
                       kernel_image_size=16, w_mode=mode))


def test_fold_plane_worked_examples():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "fold_planes.txt"))
            if l.strip() and not l.startswith("#")]
    w = np.array([float(r[0]) for r in rows])
    uvw = np.stack([np.full(len(w), 3.0), np.full(len(w), -2.0), w], axis=1)
    for col, mode in ((2, "fold"), (3, "fold_sqrt")):
        plan = _fold_plan(mode)
        g = R.snap(plan, uvw, np.ones(len(w)))
        assert g["p"].tolist() == [int(r[col]) for r in rows], mode
        assert g["fold"].tolist() == [r[1] == "1" for r in rows], mode
        assert g["counters"][1] == sum(abs(x) > 100.0 for x in w)
    assert np.allclose(_fold_plan("fold_sqrt").w_planes, [0.0, 6.25, 25.0, 56.25, 100.0], rtol=0, atol=0)
    assert np.allclose(_fold_plan("fold").w_planes, [0.0, 25.0, 50.0, 75.0, 100.0], rtol=0, atol=0)


@pytest.mark.parametrize("mode", ["fold", "fold_sqrt"])
def test_fold_plane_brute_force(mode):
    # nearest plane by enumeration: |w| against every plane, distance measured in w
    # (fold) or in sqrt|w| (fold_sqrt); random w has no ties
    plan = _fold_plan(mode, n_w=23, w_max=750.0)
    w = np.random.default_rng(3).uniform(-800.0, 800.0, 5000)
    a = np.minimum(np.abs(w), plan.w_max)
    if mode == "fold":
        d = np.abs(a[:, None] - plan.w_planes[None, :])
    else:
        d = np.abs(np.sqrt(a)[:, None] - np.sqrt(plan.w_planes)[None, :])
    uvw = np.stack([np.zeros_like(w), np.zeros_like(w), w], axis=1)
    assert R.snap(plan, uvw, np.ones(len(w)))["p"].tolist() == np.argmin(d, axis=1).tolist()


def _tie_free(plan, uvw):
    # drop rows whose snapping is within 5 % of a rounding tie, or whose sub-kernel is the
    # last one (the half-open table range has no mirror for it), on either side of the
    # mirror: the mirrored footprint rule is then exactly the mirror of the footprint
    O = plan.O
    for ax in (0, 1):
        g = uvw[:, ax] * plan.fov + plan.n / 2
        frac = g * O - np.floor(g * O)
        uvw = uvw[np.abs(frac - 0.5) > 0.05]
    for s in (1.0, -1.0):
        geo = R.snap(plan, s * uvw, np.ones(len(uvw)))
        uvw = uvw[geo["valid"] & (geo["ou"] != O - 1) & (geo["ov"] != O - 1)]
    return uvw


def test_fold_equals_linear_planes_of_the_same_spacing():
    # "fold" with N planes over [0, w_max] has the spacing of the linear rule with 2N - 1
    # planes over [-w_max, w_max], whose upper N planes sit at the same w.  Rows with
    # w >= 0 use the same plane and taps in both; rows with w < 0 are gridded mirrored
    # and conjugated, which changes the grid but not Re of the image.  So the two images
    # agree to rounding on rows away from the snapping ties.
    wl = synth.cfg1w(n_w=9, s_max=7)
    rng = np.random.default_rng(12)
    base = dict(wl.params)
    base.pop("support_per_plane")
    lin = R.Plan({**base, "n_wplanes": 17, "support": 7, "w_mode": "linear"})
    fold = R.Plan({**base, "n_wplanes": 9, "support": 7, "w_mode": "fold"})
    assert np.abs(lin.w_planes[8:] - fold.w_planes).max() < 1e-12
    uvw = _tie_free(lin, wl.uvw)
    # keep |w| off the plane-assignment ties of both rules
    t = np.abs(uvw[:, 2]) / fold.dw
    uvw = uvw[np.abs(t - np.floor(t) - 0.5) > 0.02]
    assert (uvw[:, 2] < 0).sum() > 300 and (uvw[:, 2] > 0).sum() > 300
    vis = rng.standard_normal(len(uvw)) + 1j * rng.standard_normal(len(uvw))
    wt = rng.uniform(0.5, 2.0, len(uvw))
    G1, s1, _ = R.grid(lin, R.kernel_tables(lin), uvw, vis, wt)
    G2, s2, _ = R.grid(fold, R.kernel_tables(fold), uvw, vis, wt)
    a = R.grid_to_image(lin, G1, s1)[0]
    b = R.grid_to_image(fold, G2, s2)[0]
    assert _inner_err(b, a) < 1e-11
    # and degridding: a folded row's prediction equals the unfolded one (real image)
    img = rng.standard_normal((lin.n, lin.n))
    p1 = R.predict(lin, R.kernel_tables(lin), uvw, img)
    p2 = R.predict(fold, R.kernel_tables(fold), uvw, img)
    assert np.abs(p2 - p1).max() < 1e-11 * np.abs(p1).max()


@pytest.mark.parametrize("mode", ["fold", "fold_sqrt"])
def test_fold_direct_dft(mode):
    # the w-dominated tiny field imaged with folded planes over [0, 1000] lambda, supports
    # growing with w_p from 7 to 12: close to the direct DFT with the w term, and the
    # error falls as the plane count grows (oversampling 32, so that plane spacing rather
    # than the snapping to the 1/O lattice dominates)
    wl = synth.cfg1w(n_w=33, oversample=32)
    errs = []
    for n_w in (5, 9, 17):
        params = {**wl.params, "n_wplanes": n_w, "w_mode": mode}
        plan0 = R.Plan({**params, "support_per_plane": None})
        params["support_per_plane"] = [7 + int(math.floor(5 * w / 1000.0 + 0.5)) for w in plan0.w_planes]
        sub = synth.Workload("f", params, wl.uvw, wl.vis, wl.weight)
        plan, img = _wproj_image(sub)
        geo = R.snap(plan, wl.uvw, wl.weight)
        assert geo["fold"].sum() > 500
        errs.append(_inner_err(img, _direct_dft_image(plan, wl.uvw, wl.vis, wl.weight, geo["valid"])))
    print(f"fold {mode}: inner-half error vs the direct DFT {errs}")
    assert errs[2] < 6e-3
    assert errs[1] < errs[0] and errs[2] < errs[1]


@pytest.mark.parametrize("mode", ["fold", "fold_sqrt"])
def test_fold_adjoint_identity(mode):
    # the folded pair is real-linear (conjugation): <Re IDFT(grid W x), y> = Re <x, W A(y)>
    wl = synth.cfg1w(n_w=17)
    params = {**wl.params, "w_mode": mode, "n_wplanes": 9, "support_per_plane": None, "support": 7}
    plan = R.Plan(params)
    tabs = R.kernel_tables(plan)
    rng = np.random.default_rng(15)
    x = rng.standard_normal(wl.nvis) + 1j * rng.standard_normal(wl.nvis)
    W = rng.uniform(0.5, 2.0, wl.nvis)
    y = rng.standard_normal((plan.n, plan.n))
    img = R.grid_to_image(plan, R.grid(plan, tabs, wl.uvw, x, W)[0], None)[0]
    back = W * R.predict(plan, tabs, wl.uvw, y)
    lhs = np.sum(img * y)
    rhs = np.real(np.vdot(x, back))
    assert abs(lhs - rhs) < 1e-10 * np.linalg.norm(y) * np.linalg.norm(img)


@pytest.mark.parametrize("mode", ["fold", "fold_sqrt"])
def test_c_oracle_matches_numpy_oracle_folded(mode):
    wl = synth.small_tracks(n=128, n_w=5, support=8, spp=None)
    uvw = wl.uvw.numpy().copy()
    uvw[::3, 2] *= -1.0  # plenty of w < 0 rows
    vis = wl.vis.numpy()
    wt = np.random.default_rng(4).uniform(0.0, 2.0, wl.nvis)
    plan = R.Plan({**wl.params, "w_mode": mode})
    tabs = R.kernel_tables(plan)
    G, sw, cnt = R.grid(plan, tabs, uvw, vis, wt)
    Gc, swc, cntc = cref.grid(plan, tabs, uvw, vis, wt, nthreads=4)
    assert np.abs(Gc - G).max() <= 1e-12 * np.abs(G).max()
    assert cntc.tolist() == cnt.tolist()
    M = np.random.default_rng(6).standard_normal((1, plan.n, plan.n)) + 1j
    assert np.abs(cref.degrid(plan, tabs, uvw, M, nthreads=4)
                  - R.degrid(plan, tabs, uvw, M)).max() < 1e-12 * np.abs(M).max()


# --------------------------------------------------------------------------- w-stacking


def _stack_plan(L, n_w=5, w_max=8.0, **kw):
    base = dict(n=64, cell_rad=1e-3, n_wplanes=n_w, w_max=w_max, support=7, oversample=8,
                kernel_image_size=32, w_mode="stack", n_wlayers=L)
    base.update(kw)
    return R.Plan(base)


def test_stack_layer_worked_examples():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "stack_layers.txt"))
            if l.strip() and not l.startswith("#")]
    w = np.array([float(r[0]) for r in rows])
    plan = _stack_plan(4)
    assert plan.w_layers.tolist() == [-6.0, -2.0, 2.0, 6.0]
    assert plan.w_planes.tolist() == [-2.0, -1.0, 0.0, 1.0, 2.0]
    uvw = np.stack([np.full(len(w), 3.0), np.full(len(w), -2.0), w], axis=1)
    g = R.snap(plan, uvw, np.ones(len(w)))
    assert g["layer"].tolist() == [int(r[1]) for r in rows]
    assert g["p"].tolist() == [int(r[2]) for r in rows]
    assert g["counters"][1] == sum(int(r[3]) for r in rows)


def test_stack_layer_and_plane_brute_force():
    # nearest layer centre and nearest residual plane by enumeration (random w: no ties)
    plan = _stack_plan(7, n_w=6, w_max=650.0)
    w = np.random.default_rng(21).uniform(-640.0, 640.0, 4000)
    lay = np.argmin(np.abs(w[:, None] - plan.w_layers[None, :]), axis=1)
    res = w - plan.w_layers[lay]
    pl = np.argmin(np.abs(res[:, None] - plan.w_planes[None, :]), axis=1)
    g = R.snap(plan, np.stack([np.zeros_like(w), np.zeros_like(w), w], axis=1), np.ones(len(w)))
    assert g["layer"].tolist() == lay.tolist()
    assert g["p"].tolist() == pl.tolist()


def test_stack_one_layer_is_the_linear_layout():
    # one layer of width 2 w_max centred at 0 with N_w residual planes is the linear layout
    # of N_w planes over [-w_max, w_max], operation for operation: identical grids
    wl = synth.cfg1w(n_w=9, s_max=7)
    base = {**wl.params, "support_per_plane": None, "support": 7}
    lin = R.Plan({**base, "w_mode": "linear"})
    st = R.Plan({**base, "w_mode": "stack", "n_wlayers": 1})
    assert np.array_equal(lin.w_planes, st.w_planes)
    G1, s1, c1 = R.grid(lin, R.kernel_tables(lin), wl.uvw, wl.vis, wl.weight)
    G2, s2, c2 = R.grid(st, R.kernel_tables(st), wl.uvw, wl.vis, wl.weight)
    assert np.array_equal(G1, G2) and np.array_equal(s1, s2) and c1.tolist() == c2.tolist()
    assert np.array_equal(R.grid_to_image(lin, G1, s1), R.grid_to_image(st, G2, s2))


def test_stack_direct_dft_falls_with_layers():
    # the w-dominated tiny field (w FoV^2 up to ~4 cells), three residual planes per layer,
    # support 7, oversampling 32: the error against the direct DFT with the w term falls
    # as the layers multiply, to the level of 33-plane w-projection
    wl = synth.cfg1w(n_w=33, oversample=32)
    errs = []
    for L in (1, 4, 16):
        params = {**wl.params, "n_wplanes": 3, "w_mode": "stack", "n_wlayers": L,
                  "support_per_plane": None, "support": 7}
        sub = synth.Workload("s", params, wl.uvw, wl.vis, wl.weight)
        plan, img = _wproj_image(sub)
        geo = R.snap(plan, wl.uvw, wl.weight)
        errs.append(_inner_err(img, _direct_dft_image(plan, wl.uvw, wl.vis, wl.weight, geo["valid"])))
    print(f"stack: inner-half error vs the direct DFT for 1, 4, 16 layers: {errs}")
    assert errs[1] < errs[0] / 2 and errs[2] < errs[1]
    assert errs[2] < 6e-3


def test_stack_adjoint_identity():
    # imaging and prediction with layers: <Re sum_l IDFT(grid_l W x) phase_l kappa kappa, y>
    # = Re <x, W A(y)>
    wl = synth.cfg1w(n_w=17)
    params = {**wl.params, "w_mode": "stack", "n_wlayers": 5, "n_wplanes": 4,
              "support_per_plane": None, "support": 7}
    plan = R.Plan(params)
    tabs = R.kernel_tables(plan)
    rng = np.random.default_rng(25)
    x = rng.standard_normal(wl.nvis) + 1j * rng.standard_normal(wl.nvis)
    W = rng.uniform(0.5, 2.0, wl.nvis)
    y = rng.standard_normal((plan.n, plan.n))
    img = R.grid_to_image(plan, R.grid(plan, tabs, wl.uvw, x, W)[0], None)[0]
    back = W * R.predict(plan, tabs, wl.uvw, y)
    lhs = np.sum(img * y)
    rhs = np.real(np.vdot(x, back))
    assert abs(lhs - rhs) < 1e-10 * np.linalg.norm(y) * np.linalg.norm(img)


@pytest.mark.parametrize("nthreads", [1, 4])
def test_c_oracle_matches_numpy_oracle_stacked(nthreads):
    wl = synth.small_tracks(n=128, n_w=5, support=8, spp=None)
    uvw = wl.uvw.numpy()
    vis = wl.vis.numpy()
    wt = np.random.default_rng(8).uniform(0.0, 2.0, wl.nvis)
    offs = np.array([0, wl.nvis // 3, wl.nvis // 3, wl.nvis])
    plan = R.Plan({**wl.params, "w_mode": "stack", "n_wlayers": 6, "n_images": 3})
    tabs = R.kernel_tables(plan)
    G, sw, cnt = R.grid(plan, tabs, uvw, vis, wt, offs)
    assert G.shape[0] == 18 and len({int(i) for i in np.nonzero(np.abs(G).sum(axis=(1, 2)))[0]}) > 6
    Gc, swc, cntc = cref.grid(plan, tabs, uvw, vis, wt, offs, nthreads=nthreads)
    assert np.abs(Gc - G).max() <= 1e-12 * np.abs(G).max()
    assert np.allclose(swc, sw, rtol=1e-13, atol=0) and cntc.tolist() == cnt.tolist()
    M = np.random.default_rng(6).standard_normal((18, plan.n, plan.n)) + 1j
    assert np.abs(cref.degrid(plan, tabs, uvw, M, offs, nthreads=nthreads)
                  - R.degrid(plan, tabs, uvw, M, offs)).max() < 1e-12 * np.abs(M).max()
