"""Rows regrouped by baseline on the device (Section 2.2, Eqs. 5 and 6) against the
oracle (oracle/eq56.py): the permutation, Eq. 6's start offsets and the counts C must
match exactly.  Row gathers against torch indexing.

Workloads: the 8 h, 27-antenna track of the 2048^2 benchmark (2880 x 351 rows in time
order, the layout a measurement set stores), shuffled rows with autocorrelations and
swapped antenna order, 255 antennas (the largest supported), a row count that makes
the device use blocks larger than its minimum, and the degenerate cases (no rows, one
row, one antenna, invalid antenna IDs)."""

import numpy as np
import pytest
import torch

import paper_1905_03213_amd as W
import synth
from oracle import eq56

pytestmark = pytest.mark.gpu


def _expected(a1, a2, n_ant):
    """Oracle regroup, with rows carrying an invalid antenna ID numbered n_b (last)."""
    a1 = np.asarray(a1, dtype=np.int64)
    a2 = np.asarray(a2, dtype=np.int64)
    n_b = n_ant * (n_ant + 1) // 2
    ok = (a1 >= 0) & (a2 >= 0) & (a1 < n_ant) & (a2 < n_ant)
    b = np.full(a1.shape[0], n_b, dtype=np.int64)
    b[ok] = eq56.baseline_index(a1[ok], a2[ok], n_ant)
    c = eq56.counts(b, n_b + 1)
    return eq56.regroup_order(b, n_b + 1), eq56.start_index(c), c


def _check(a1, a2, n_ant):
    t1 = torch.as_tensor(np.asarray(a1, dtype=np.int32), device="cuda")
    t2 = torch.as_tensor(np.asarray(a2, dtype=np.int32), device="cuda")
    perm, start, counts = W.regroup_rows(t1, t2, n_ant)
    torch.cuda.synchronize()
    p_ref, s_ref, c_ref = _expected(a1, a2, n_ant)
    assert np.array_equal(perm.cpu().numpy(), p_ref)
    assert np.array_equal(start.cpu().numpy(), s_ref)
    assert np.array_equal(counts.cpu().numpy(), c_ref)
    return perm


def _track_rows(hours=8.0, dt_s=10.0):
    _, a1, a2 = synth.array_tracks(np.random.default_rng(2), hours=hours, dt_s=dt_s)
    n_t = int(round(hours * 3600 / dt_s))
    return np.tile(a1, n_t), np.tile(a2, n_t), n_t, len(a1)


def test_regroup_benchmark_track():
    a1, a2, n_t, n_bl = _track_rows()
    assert a1.shape[0] == 2880 * 351
    perm = _check(a1, a2, 27).cpu().numpy()
    # every baseline's rows are its n_t timestamps in time order
    assert np.array_equal(perm[:n_t] % n_bl, np.zeros(n_t) + perm[0] % n_bl)
    assert (np.diff(perm[:n_t]) == n_bl).all()


@pytest.mark.parametrize("n_rows,n_ant,seed", [(100_003, 27, 0), (50_000, 255, 1), (7, 3, 2),
                                               (2048, 27, 3), (2049, 27, 4)])
def test_regroup_shuffled_rows(n_rows, n_ant, seed):
    rng = np.random.default_rng(seed)
    a1 = rng.integers(0, n_ant, n_rows)
    a2 = rng.integers(0, n_ant, n_rows)  # autocorrelations and either antenna order
    _check(a1, a2, n_ant)


def test_regroup_large_blocks():
    # 255 antennas and 5e6 rows: more than 2^26 per-block counts at 2048 rows per block,
    # so the device enlarges its blocks
    rng = np.random.default_rng(5)
    n_rows, n_ant = 5_000_000, 255
    a1 = rng.integers(0, n_ant, n_rows)
    a2 = rng.integers(0, n_ant, n_rows)
    _check(a1, a2, n_ant)


def test_regroup_degenerate():
    _check([], [], 27)
    _check([3], [1], 27)
    _check([0, 0, 0], [0, 0, 0], 1)  # one antenna: only its autocorrelation
    # invalid IDs go last, in row order, and are counted in counts[n_b]
    a1 = [2, -1, 0, 27, 1, 2, 5]
    a2 = [1, 3, 0, 0, 1, 30, 4]
    perm = _check(a1, a2, 27).cpu().numpy()
    assert perm[-3:].tolist() == [1, 3, 5]


def test_gather_rows_matches_indexing():
    a1, a2, n_t, n_bl = _track_rows(hours=1.0)
    t1 = torch.as_tensor(a1.astype(np.int32), device="cuda")
    t2 = torch.as_tensor(a2.astype(np.int32), device="cuda")
    perm, _, _ = W.regroup_rows(t1, t2, 27)
    n_rows = a1.shape[0]
    g = torch.Generator(device="cpu").manual_seed(0)
    uvw = torch.randn((n_rows, 16, 3), dtype=torch.float64, generator=g).cuda()   # 16 channels
    vis = torch.randn((n_rows, 16), dtype=torch.complex64, generator=g).cuda()
    assert torch.equal(W.gather_rows(perm, uvw), uvw[perm])
    assert torch.equal(W.gather_rows(perm, vis), vis[perm])
    wt3 = torch.randn((n_rows, 3), dtype=torch.float32, generator=g).cuda()  # 12-byte rows
    assert torch.equal(W.gather_rows(perm, wt3), wt3[perm])
    # out-of-range entries leave their rows untouched and are counted
    bad_perm = perm.clone()
    bad_perm[5] = -1
    bad_perm[7] = n_rows
    out = torch.zeros_like(vis)
    bad = torch.zeros(1, dtype=torch.int64, device="cuda")
    W.gather_rows(bad_perm, vis, out=out, bad=bad)
    ref = vis[perm.clamp(0, n_rows - 1)]
    ref[5] = 0
    ref[7] = 0
    assert torch.equal(out, ref) and int(bad.item()) == 2
