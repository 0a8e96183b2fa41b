"""Launch-shape autotuner for one (n, M) bucket.

Times candidate tunings (grand_tuning_set) on a sample batch of that bucket
(of the size the bucket's launches will have: the best workgroup size and
count depend on how many words a launch holds),
keeps only candidates whose outputs equal the first candidate's (a tuning
changes the launch shape, never a result; a candidate whose node store
overflows reports GRAND_ECAPACITY and is dropped), and installs the fastest.
Batches decoded afterwards use it for every launch of that bucket.  Mixed
batches whose buckets are each too small to fill the device run as one merged
launch with the wildcard (0, 0) entry; autotune_batch tunes that entry on a
sample of such a batch."""
from __future__ import annotations

import itertools

import numpy as np

from . import decoder


def default_candidates(n: int, M: int) -> list[dict]:
    """b in {8, 9, 10} x 6..8 workgroups of 256 threads per CU, and b = 9 x
    2..4 workgroups of 512 threads per CU (long words gain from more waves
    per word)."""
    base = decoder.get_tuning(n, M)
    out = []
    for low_bits, grid in itertools.product((8, 9, 10), (6, 7, 8)):
        out.append(dict(base, block=256, low_bits=low_bits, grid_per_cu=grid))
    for grid in (2, 3, 4):
        out.append(dict(base, block=512, low_bits=9, grid_per_cu=grid))
    return out


def _time_candidates(key, cands, make_plan, count, reps, stream):
    """Install each candidate for bucket `key`, time `reps` launches of the
    plan make_plan() builds, and keep those whose outputs equal the first
    valid candidate's.  The original tuning is restored."""
    import torch
    original = decoder.get_tuning(*key)
    ref = None
    table = []
    try:
        for c in cands:
            try:
                decoder.set_tuning(*key, **c)
            except Exception as e:   # an invalid tuning for this device
                table.append({"tuning": c, "ms": None, "rejected": str(e)})
                continue
            plan = make_plan()
            plan.launch(stream)
            torch.cuda.synchronize()
            times = []
            for _ in range(reps):
                a = torch.cuda.Event(enable_timing=True)
                b = torch.cuda.Event(enable_timing=True)
                a.record(stream)
                out = plan.launch(stream)
                b.record(stream)
                torch.cuda.synchronize()
                times.append(a.elapsed_time(b))
            res = [t.cpu().numpy().copy() for t in (out.codewords, out.queries, out.abandoned,
                                                     out.status)]
            if np.any(res[3][:count] != 0):
                table.append({"tuning": c, "ms": None, "rejected": "device status errors"})
                continue
            if ref is None:
                ref = res
            elif not all(np.array_equal(x[:count], y[:count]) for x, y in zip(res, ref)):
                table.append({"tuning": c, "ms": None, "rejected": "results differ"})
                continue
            table.append({"tuning": c, "ms": float(np.median(times))})
    finally:
        decoder.set_tuning(*key, **original)
    ok = [t for t in table if t["ms"] is not None]
    if not ok:
        raise RuntimeError("no candidate tuning decoded the sample")
    return min(ok, key=lambda t: t["ms"]), table


def autotune_batch(codes, code_index, M, cap, noise_var, rx_offset, rx, candidates=None,
                   reps: int = 3, stream=None) -> dict:
    """Tune the wildcard (0, 0) entry, which merged launches of mixed batches
    use, on a sample mixed batch (the same arguments as BatchPlan).  Installs
    and returns the fastest candidate whose outputs equal the others'."""
    import torch
    count = len(code_index)
    cands = candidates if candidates is not None else default_candidates(0, 0)
    if not cands:
        raise ValueError("no candidate tunings")
    stream = stream or torch.cuda.current_stream(rx.device)
    best, table = _time_candidates(
        (0, 0), cands,
        lambda: decoder.BatchPlan(codes, code_index, M, cap, noise_var, rx_offset, rx),
        count, reps, stream)
    decoder.set_tuning(0, 0, **best["tuning"])
    return {"n": 0, "M": 0, "best": best["tuning"], "ms": best["ms"], "table": table}


def autotune(code, M: int, rx, rx_offset, cap, noise_var, candidates=None, reps: int = 3,
             stream=None) -> dict:
    """rx: float32 device tensor holding the sample words at rx_offset (one
    per word, all of `code` and modulation M).  Returns the chosen tuning,
    its median launch time and every candidate's timing."""
    import torch
    n = code.n
    count = len(rx_offset)
    cands = candidates if candidates is not None else default_candidates(n, M)
    if not cands:
        raise ValueError("no candidate tunings")
    stream = stream or torch.cuda.current_stream(rx.device)
    best, table = _time_candidates(
        (n, M), cands,
        lambda: decoder.BatchPlan([code], np.zeros(count, np.uint32), [M] * count,
                                  np.asarray(cap, np.uint64), np.asarray(noise_var, np.float32),
                                  rx_offset, rx),
        count, reps, stream)
    decoder.set_tuning(n, M, **best["tuning"])
    return {"n": n, "M": M, "best": best["tuning"], "ms": best["ms"], "table": table}
