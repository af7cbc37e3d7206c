"""Baseline index and per-baseline start offsets (paper Section 2.2, Eqs. 5 and 6).

Test infrastructure only (see the oracle package docstring).

The paper's GPU path needs rows grouped by baseline and then ordered by time.
A measurement set stores only the two antenna IDs of each row, so a baseline
number is derived from them (Eq. 5), rows per baseline are counted into an
array C, and an exclusive prefix sum of C gives each baseline's first row in
the regrouped order (Eq. 6).  Antenna IDs are 0-based here; with that reading
Eq. 5 maps every pair a1 <= a2 (autocorrelations included) one-to-one onto
0 .. N_ant (N_ant + 1)/2 - 1.
"""

import numpy as np


def baseline_index(ant1, ant2, n_ant: int):
    """Eq. 5: I_B = (-S^2 + 2 S N_ant + S)/2 + |I_ant1 - I_ant2|, S = min(I_ant1, I_ant2)."""
    a1 = np.asarray(ant1, dtype=np.int64)
    a2 = np.asarray(ant2, dtype=np.int64)
    s = np.minimum(a1, a2)
    return (-s * s + 2 * s * n_ant + s) // 2 + np.abs(a1 - a2)


def counts(bidx, n_baselines: int):
    """The array C: number of rows (timestamps) carrying each baseline number."""
    c = np.zeros(n_baselines, dtype=np.int64)
    for b in np.asarray(bidx, dtype=np.int64):
        c[b] += 1
    return c


def start_index(c):
    """Eq. 6: B_start[0] = 0 and B_start[i] = sum_{k < i} C[k] (exclusive prefix sum)."""
    c = np.asarray(c, dtype=np.int64)
    out = np.zeros(c.shape[0], dtype=np.int64)
    run = 0
    for i in range(c.shape[0]):
        out[i] = run
        run += c[i]
    return out


def regroup_order(bidx, n_baselines: int):
    """Row permutation that groups rows by baseline, keeping time order inside a group.

    Row j goes to position B_start[I_B(j)] + (number of earlier rows with the
    same baseline); returns perm with regrouped[k] = rows[perm[k]].
    """
    b = np.asarray(bidx, dtype=np.int64)
    start = start_index(counts(b, n_baselines))
    fill = start.copy()
    perm = np.empty(b.shape[0], dtype=np.int64)
    for j in range(b.shape[0]):
        perm[fill[b[j]]] = j
        fill[b[j]] += 1
    return perm


def channel_major_order(row_perm, bidx, n_baselines: int, n_chan: int):
    """Visibility order after the regroup, channel by channel: the paper's CUDA gridder
    walks one baseline's timestamps in sequence (Section 2.2); with n_chan channels per
    row that is, for each baseline in turn and each channel c, the baseline's rows in
    time order.  Visibility (row j, channel c) has source index j n_chan + c; returns the
    source index of every position of that order."""
    row_perm = np.asarray(row_perm, dtype=np.int64)
    b = np.asarray(bidx, dtype=np.int64)
    c = counts(b, n_baselines)
    start = start_index(c)
    out = []
    for bl in range(n_baselines):
        rows = row_perm[start[bl]:start[bl] + c[bl]]  # this baseline's rows, in time order
        for ch in range(n_chan):
            out.extend((rows * n_chan + ch).tolist())
    return np.asarray(out, dtype=np.int64)
