"""Pins for the oracle's pattern order (Algorithm 2 Steps 4-5; the ML
ordering statement of Section II): every pattern, in ascending
(cost sum, colex) order, checked against a brute-force sort."""
import itertools
import math

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st


def brute_order(costs):
    n = len(costs)
    keys = []
    for mask in range(1 << n):
        c = sum(costs[r] for r in range(n) if (mask >> r) & 1)
        keys.append((c, mask))
    keys.sort()
    return keys


@pytest.mark.parametrize("n,hi,seed", [(1, 5, 0), (4, 3, 1), (8, 4, 2), (10, 50, 3),
                                       (12, 4096, 4), (12, 2, 5), (6, 1, 6)])
def test_enumeration_equals_brute_force_sort(orc, n, hi, seed):
    rng = np.random.default_rng(seed)
    costs = np.sort(rng.integers(0, hi + 1, n)).astype(np.uint32)
    masks, sums = orc.enumerate_teps(costs, 1 << n)
    got = [(int(s), int(m)) for s, m in zip(sums, masks[:, 0])]
    assert got == brute_order([int(c) for c in costs])


def test_enumeration_exhausts_and_stops(orc):
    costs = np.array([1, 2, 3], np.uint32)
    masks, sums = orc.enumerate_teps(costs, 100)
    assert len(masks) == 8


def test_enumeration_wide_masks(orc):
    """Ranks beyond 64 use further mask words; all-equal costs order by
    size then colex."""
    n = 130
    costs = np.full(n, 7, np.uint32)
    masks, sums = orc.enumerate_teps(costs, 1 + n + 20)
    assert masks.shape[1] == 3
    assert sums[0] == 0 and not masks[0].any()
    for r in range(n):                       # singletons in rank order
        bits = [(w, b) for w in range(3) for b in range(64) if (int(masks[1 + r, w]) >> b) & 1]
        assert bits == [(r // 64, r % 64)]
    pairs = list(itertools.combinations(range(n), 2))
    pairs.sort(key=lambda p: (p[1], p[0]))   # colex
    for k in range(20):
        bits = [w * 64 + b for w in range(3) for b in range(64)
                if (int(masks[1 + n + k, w]) >> b) & 1]
        assert tuple(bits) == pairs[k]


@settings(max_examples=40, deadline=None)
@given(st.lists(st.integers(0, 40), min_size=1, max_size=11))
def test_order_properties(orc, costs_list):
    costs = np.sort(np.array(costs_list, np.uint32))
    n = len(costs)
    masks, sums = orc.enumerate_teps(costs, 1 << n)
    assert len(masks) == 1 << n                                  # 2^n patterns
    assert len({int(m) for m in masks[:, 0]}) == 1 << n
    assert np.all(np.diff(sums.astype(np.int64)) >= 0)           # non-increasing likelihood
    for q, m in enumerate(masks[:, 0], start=1):                 # |T| <= floor(log2 q)
        assert bin(int(m)).count("1") <= int(math.floor(math.log2(q)))
    for s, m in zip(sums, masks[:, 0]):
        assert int(s) == sum(int(costs[r]) for r in range(n) if (int(m) >> r) & 1)


def test_unsorted_costs_rejected(orc):
    with pytest.raises(ValueError):
        orc.enumerate_teps(np.array([3, 1], np.uint32), 4)
