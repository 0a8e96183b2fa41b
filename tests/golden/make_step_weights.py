"""Write step_weights_polar128_16qam.json: the mean number of columns w
that the successor-tree step from a pattern's parent XORs in, over the
patterns a decode queries (the first q in (cost, colex) order), for the first
256 codewords of the polar128_16qam workload; and
step_weights_uneven_mix.json: the same per (N, M) bucket of the uneven_mix
workload, over its first UNEVEN_PER_BUCKET codewords of each bucket.

In the successor tree (root: the empty pattern; from T with largest rank j,
the children T + {j+1} and T - {j} + {j+1}), a pattern whose largest rank r
has r - 1 in it (or r = 0) is a type-one child (w = 1); otherwise it is a
type-two child (w = 2); the empty pattern has w = 0.  The incremental
syndrome of a query costs (w + 1) * ceil(rows / 32) 32-bit operations: w
column XORs and one zero test.

Uses only the oracle and the workload generator:
    python tests/golden/make_step_weights.py
"""
from __future__ import annotations

import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

OUT = os.path.join(HERE, "step_weights_polar128_16qam.json")
OUT_UNEVEN = os.path.join(HERE, "step_weights_uneven_mix.json")
WORDS = 256
UNEVEN_PER_BUCKET = 8


def step_weights(masks: np.ndarray) -> np.ndarray:
    """w per pattern (masks: uint64, at most 64 ranks)."""
    m = np.asarray(masks, dtype=np.uint64)
    w = np.zeros(m.size, np.int64)
    nz = m != 0
    r = np.zeros(m.size, np.int64)
    r[nz] = np.floor(np.log2(m[nz].astype(np.float64))).astype(np.int64)
    # the float log2 may be off by one near powers of two: settle it exactly
    for _ in range(2):
        hi = nz & ((m >> r.astype(np.uint64)) == 0)
        r[hi] -= 1
        lo = nz & (r < 63) & ((m >> (r + 1).astype(np.uint64)) != 0)
        r[lo] += 1
    below = (m >> np.maximum(r - 1, 0).astype(np.uint64)) & np.uint64(1)
    w[nz] = np.where((r[nz] == 0) | (below[nz] == 1), 1, 2)
    return w


def step_weights_wide(masks: np.ndarray) -> np.ndarray:
    """w per pattern for masks of any width (uint64 [count, words], rank r
    is bit r % 64 of word r // 64)."""
    m = np.atleast_2d(np.asarray(masks, dtype=np.uint64))
    w = np.zeros(m.shape[0], np.int64)
    for i, row in enumerate(m):
        bits = 0
        for k, word in enumerate(row):
            bits |= int(word) << (64 * k)
        if bits == 0:
            continue
        r = bits.bit_length() - 1
        w[i] = 1 if r == 0 or (bits >> (r - 1)) & 1 else 2
    return w


def uneven_main():
    import oracle
    import workload as wl
    oracle.build(force=False)
    jobs = wl.config_jobs("uneven_mix", count=1024)
    picked: dict[tuple[int, int], list] = {}
    for j in jobs:
        lst = picked.setdefault((j.N, j.M), [])
        if len(lst) < UNEVEN_PER_BUCKET:
            lst.append(j)
    buckets = {}
    for (N, M), lst in sorted(picked.items()):
        code = wl.polar_code(N, N // 2)
        total_w = total_q = 0
        for j in lst:
            _, q, _ = oracle.decode(code.h_rows, j.N, j.rx, j.M, j.noise_var, j.cap)
            _, cost, pos = oracle.demap(j.N, j.M, j.rx)
            order = np.lexsort((pos, cost))
            masks, _ = oracle.enumerate_teps(cost[order], q)
            total_w += int(step_weights_wide(masks).sum())
            total_q += int(q)
        rows = N // 2
        mean_w = total_w / total_q
        buckets[f"{N},{M}"] = {"codewords": len(lst), "queries": total_q, "mean_w": mean_w,
                               "rows": rows,
                               "lane_ops_per_query": (mean_w + 1) * ((rows + 31) // 32)}
        print(N, M, buckets[f"{N},{M}"], flush=True)
    rec = {"workload": "uneven_mix", "per_bucket_codewords": UNEVEN_PER_BUCKET,
           "buckets": buckets}
    with open(OUT_UNEVEN, "w") as f:
        json.dump(rec, f, indent=1)
        f.write("\n")


def main():
    import oracle
    import workload as wl
    oracle.build(force=False)
    jobs = wl.config_jobs("polar128_16qam", count=WORDS)
    code = wl.polar_code(128, 64)
    total_w = 0
    total_q = 0
    for j in jobs:
        _, q, _ = oracle.decode(code.h_rows, j.N, j.rx, j.M, j.noise_var, j.cap)
        _, cost, pos = oracle.demap(j.N, j.M, j.rx)
        order = np.lexsort((pos, cost))
        masks, _ = oracle.enumerate_teps(cost[order], q)
        total_w += int(step_weights(masks[:, 0]).sum())
        total_q += int(q)
    rec = {"workload": "polar128_16qam", "codewords": WORDS, "queries": total_q,
           "mean_w": total_w / total_q, "rows": 64,
           "lane_ops_per_query": (total_w / total_q + 1) * 2}
    with open(OUT, "w") as f:
        json.dump(rec, f, indent=1)
        f.write("\n")
    print(json.dumps(rec))


if __name__ == "__main__":
    if len(sys.argv) > 1 and sys.argv[1] == "uneven":
        uneven_main()
    else:
        main()
