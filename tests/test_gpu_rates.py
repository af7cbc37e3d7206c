"""The device rate measurements that bench.py divides by: LDS streaming
(wproj_measure_lds) and L1-resident vector-memory loads (wproj_measure_vmem) return
finite rates within physical bounds, and a longer run moves proportionally more data in
proportionally more time."""

import math

import pytest

import paper_1905_03213_amd as W

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_lds_rate(mode):
    bps, ms = W.measure_lds(mode, rounds=1024)
    assert math.isfinite(bps) and 1e12 < bps < 1e15 and ms > 0.0


@pytest.mark.parametrize("width", [4, 8, 16])
def test_vmem_rate(width):
    bps, ms = W.measure_vmem(width, rounds=1024)
    assert math.isfinite(bps) and 1e11 < bps < 1e15 and ms > 0.0
    bps4, ms4 = W.measure_vmem(width, rounds=4096)
    assert ms4 > 2.0 * ms  # four times the loads take clearly longer
    assert 0.5 < bps4 / bps < 2.0
