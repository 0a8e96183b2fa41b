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
