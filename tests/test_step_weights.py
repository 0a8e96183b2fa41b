"""The per-query work unit of the roofline: w, the columns the successor-tree
step from a pattern's parent XORs in (the order of Algorithm 2 Step 4 under
the (cost, colex) reading)."""
import json
import os

import numpy as np

from golden.make_step_weights import OUT, step_weights


def successor_tree_w(n):
    """w of every subset of n ranks, by walking the successor tree."""
    w = {0: 0}
    stack = [0]
    while stack:
        t = stack.pop()
        j = t.bit_length() - 1            # largest rank, -1 for the root
        if j + 1 >= n:
            continue
        a = t | (1 << (j + 1))            # T + {j+1}: one new column
        w[a] = 1
        stack.append(a)
        if j >= 0:
            b = (t & ~(1 << j)) | (1 << (j + 1))   # T - {j} + {j+1}: two columns
            w[b] = 2
            stack.append(b)
    return w


def test_step_weights_match_the_successor_tree():
    for n in (1, 2, 5, 9):
        ref = successor_tree_w(n)
        assert len(ref) == 2 ** n            # every subset has exactly one parent
        masks = np.array(sorted(ref), dtype=np.uint64)
        assert list(step_weights(masks)) == [ref[int(m)] for m in masks]


def test_step_weights_near_powers_of_two():
    masks = np.array([(1 << 63), (1 << 63) | (1 << 62), (1 << 53) - 1, 1 << 53,
                      (1 << 60) - 1, (1 << 60) + 1], dtype=np.uint64)
    assert list(step_weights(masks)) == [2, 1, 1, 2, 1, 2]


def test_stored_mean_w_is_consistent():
    rec = json.load(open(OUT))
    assert 1.0 <= rec["mean_w"] <= 2.0
    assert abs(rec["lane_ops_per_query"] - (rec["mean_w"] + 1) * ((rec["rows"] + 31) // 32)) < 1e-9
    assert rec["queries"] > 0


def test_wide_masks_match_the_successor_tree():
    """step_weights_wide (masks of any width) equals the tree walk on every
    subset of 10 ranks, and decides across 64-bit word boundaries."""
    from golden.make_step_weights import step_weights_wide
    n = 10
    tree = successor_tree_w(n)
    masks = np.array(sorted(tree), dtype=np.uint64)[:, None]
    got = step_weights_wide(masks)
    assert [int(x) for x in got] == [tree[int(m)] for m in masks[:, 0]]
    two = np.zeros((4, 2), np.uint64)
    two[0, 1] = 1 << 6                      # rank 70 alone: type two
    two[1, 1] = (1 << 6) | (1 << 5)         # ranks 69 and 70: type one
    two[2, 1] = 1                           # rank 64, rank 63 absent: type two
    two[2, 0] = 1 << 5
    two[3, 1] = 1                           # ranks 63 and 64 across the word boundary: one
    two[3, 0] = 1 << 63
    assert list(step_weights_wide(two)) == [2, 1, 2, 1]


def test_stored_uneven_bucket_weights_are_consistent():
    from golden.make_step_weights import OUT_UNEVEN
    rec = json.load(open(OUT_UNEVEN))
    assert rec["workload"] == "uneven_mix" and len(rec["buckets"]) == 12
    for key, b in rec["buckets"].items():
        N, M = (int(x) for x in key.split(","))
        assert b["rows"] == N // 2 and 0 <= b["mean_w"] <= 2 and b["queries"] >= b["codewords"]
        assert abs(b["lane_ops_per_query"] - (b["mean_w"] + 1) * ((N // 2 + 31) // 32)) < 1e-9
