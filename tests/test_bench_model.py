"""The algorithmic op model bench.py prices the INT32 roofline with.

Plane counts must hold every c value the kernels can meet (two's complement:
B planes hold [-2^(B-1), 2^(B-1) - 1]); plane caps never price more than the
uncapped form; and the per-evaluation figures quoted for the workloads follow
from the model.
"""
import pytest

import bench


def fits(lo, hi, B):
    return -(1 << (B - 1)) <= lo and hi <= (1 << (B - 1)) - 1


@pytest.mark.parametrize("nw", [1, 2, 3, 4, 5, 6])
def test_skew_planes_hold_every_c(nw):
    # skew space: even lag k = 2t + 2 has |C_k| <= L - k (odd), c = (C - 1) / 2
    for L in range(3, min(64 * nw + 1, 383) + 1, 2):
        if bench.lag_words(L) != nw:
            continue
        for t in range((L - 1) // 2):
            n = L - (2 * t + 2)
            assert fits((-n - 1) // 2, (n - 1) // 2, bench.planes_of(nw, t // 32)), (L, t)


@pytest.mark.parametrize("nw", [1, 2, 3, 4, 5, 6])
def test_full_planes_hold_every_c(nw):
    # whole space: lag k has |C_k| <= n = L - k with the parity of n, c = (C - p) / 2
    for L in range(3, 193):
        if (L - 1 + 31) // 32 != nw:
            continue
        for k in range(1, L):
            n, p = L - k, (L - k) % 2
            assert fits((-n - p) // 2, (n - p) // 2, bench.full_planes_of(nw, (k - 1) // 32)), (L, k)


@pytest.mark.parametrize("L", [27, 101, 151, 223, 301, 383])
def test_skew_caps_never_price_above_uncapped(L):
    full = bench.ops_per_scan(L, 0)
    assert bench.ops_per_scan(L, 4) <= bench.ops_per_scan(L, 5) <= bench.ops_per_scan(L, 6) <= full


@pytest.mark.parametrize("L", [3, 64, 65, 128, 129, 192])
def test_full_caps_never_price_above_uncapped(L):
    full = bench.full_ops_per_scan(L, 0)
    assert bench.full_ops_per_scan(L, 4) <= bench.full_ops_per_scan(L, 5) <= full


def test_quoted_per_evaluation_figures():
    D = 76
    assert [round(bench.ops_per_scan(151, c) / D, 1) for c in (4, 5, 6, 0)] == [29.0, 35.7, 42.4, 52.5]
    assert [round(bench.full_ops_per_scan(128, c) / 128, 1) for c in (0, 5, 4)] == [84.9, 62.2, 52.3]


def test_pair_count_matches_lag_ranges():
    # each candidate is priced per lag word its forward or backward range touches
    L, nw = 128, 4
    pl = [bench.full_planes_of(nw, w) for w in range(nw)]
    words = 0
    for i in range(1, L + 1):
        fw = len({(k - 1) // 32 for k in range(1, L - i + 1)})
        bw = len({(k - 1) // 32 for k in range(1, i)})
        q = len({(k - 1) // 32 for k in range(1, min(L - i, i - 1) + 1)})
        words += 2 * (sum(pl[:fw]) + fw + sum(pl[:bw]) + bw + q)
    assert words == bench.full_ops_per_scan(L, 0)
