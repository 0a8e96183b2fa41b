"""grand_decode_batch_noalloc (no device allocation, static scratch array)
against grand_decode_batch on the same inputs: two calls in a row, the
second with a smaller batch of other shapes, then size limits."""
import ctypes

import numpy as np
import pytest

import workload as w
from helpers import make_plan, outputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch
    import paper_2405_01808_amd as g
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    g.init(0)
    return g


def run_both(gpu, jobs, label):
    import torch
    from paper_2405_01808_amd import _native as nat
    plan, _ = make_plan(gpu, jobs)
    plan.launch()
    torch.cuda.synchronize()
    ref = outputs(plan)
    for t in (plan.out.codewords, plan.out.queries, plan.out.abandoned, plan.out.status):
        t.fill_(-1 if t.dtype != torch.uint8 else 7)
    print(f"{label}: {len(jobs)} words through grand_decode_batch_noalloc", flush=True)
    rc = nat.lib().grand_decode_batch_noalloc(ctypes.byref(plan.desc), None)
    assert rc == nat.GRAND_OK, nat.lib().grand_last_error()
    torch.cuda.synchronize()
    got = outputs(plan)
    n = len(jobs)
    st = got[3][:n]
    assert np.all(st == 0), (label, np.unique(st))
    for k, name in enumerate(("queries", "abandoned", "status"), start=1):
        assert np.array_equal(got[k][:n], ref[k][:n]), (label, name)
    for i, j in enumerate(jobs):      # the used 64-bit words of each codeword
        nw = (j.N + 63) // 64
        assert np.array_equal(got[0][i, :nw], ref[0][i, :nw]), (label, "codeword", i)
    return ref


def test_noalloc_equals_batch_twice(gpu):
    big = w.config_jobs("polar128_16qam", count=4096)
    ref = run_both(gpu, big, "first call")
    assert 0 < ref[2][:len(big)].sum() < len(big)        # hits and abandons
    # the serving mix's shorter words (N <= 256, every M): other shapes
    small = [j for j in w.config_jobs("serving_mix", count=400, start=2000) if j.N <= 256]
    assert 100 < len(small) < len(big) and len({(j.N, j.M) for j in small}) > 8
    run_both(gpu, small, "second call, smaller")


def test_noalloc_rejects_sizes_beyond_its_limits(gpu):
    from paper_2405_01808_amd import _native as nat
    jobs = w.config_jobs("polar128_16qam", count=8)
    plan, _ = make_plan(gpu, jobs)
    L = nat.lib()
    d = plan.desc
    count = d.count
    d.count = nat.NOALLOC_MAX_WORDS + 1
    assert L.grand_decode_batch_noalloc(ctypes.byref(d), None) == nat.GRAND_EINVAL
    assert b"GRAND_NOALLOC_MAX_WORDS" in L.grand_last_error()
    d.count = count
    rxc = d.rx_count
    d.rx_count = rxc - 1
    assert L.grand_decode_batch_noalloc(ctypes.byref(d), None) == nat.GRAND_EINVAL
    d.rx_count = rxc
    assert L.grand_decode_batch_noalloc(ctypes.byref(d), None) == nat.GRAND_OK
