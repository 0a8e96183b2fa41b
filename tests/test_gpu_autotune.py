"""The launch-shape autotuner: picks the fastest valid candidate, rejects a
candidate whose node store overflows, and never changes a result."""
import numpy as np
import pytest

import workload as w

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch
    import paper_2405_01808_amd as g
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    g.init(0)
    return g


def test_autotune_installs_fastest_valid_candidate(gpu):
    import torch
    jobs = w.jobs_from_spec("tune", seed=31, count=1024, cap=1 << 12, Ns=(128,), Ms=(16,),
                            ebn0=("uniform", 3.0, 7.0))
    code = gpu.Code(128, w.polar_code(128, 64).h_rows)
    L2 = len(jobs[0].rx)
    rx = torch.from_numpy(np.concatenate([j.rx for j in jobs])).cuda()
    offs = np.arange(len(jobs), dtype=np.uint64) * L2
    caps = [j.cap for j in jobs]
    nvs = [j.noise_var for j in jobs]
    before = gpu.get_tuning(128, 16)

    def decode():
        plan = gpu.BatchPlan([code], np.zeros(len(jobs), np.uint32), [16] * len(jobs), caps, nvs,
                             offs, rx)
        out = plan.launch()
        torch.cuda.synchronize()
        return [t.cpu().numpy().copy() for t in (out.codewords, out.queries, out.abandoned,
                                                  out.status)]

    ref = decode()
    cands = [dict(before, low_bits=8), dict(before, low_bits=9), dict(before, grid_per_cu=6),
             dict(before, node_cap=64)]
    try:
        res = gpu.autotune(code, 16, rx, offs, caps, nvs, candidates=cands, reps=2)
        timed = [t for t in res["table"] if t["ms"] is not None]
        rejected = [t for t in res["table"] if t["ms"] is None]
        assert len(timed) >= 3
        assert any(t["tuning"]["node_cap"] == 64 for t in rejected)   # store overflow
        assert res["best"] in [t["tuning"] for t in timed]
        assert res["ms"] == min(t["ms"] for t in timed)
        assert gpu.get_tuning(128, 16) == res["best"]
        got = decode()
        for x, y in zip(got, ref):
            assert np.array_equal(x, y)
    finally:
        gpu.set_tuning(128, 16, **before)


def test_autotune_batch_tunes_the_merged_launch(gpu):
    """A mixed batch whose buckets are each too small to fill the device runs
    as one merged launch with the wildcard (0, 0) tuning: autotune_batch times
    candidates for that entry, installs the fastest, and results stay equal."""
    import torch
    from helpers import make_plan, outputs
    jobs = w.config_jobs("uneven_mix", count=600, cap=1 << 12)
    plan, order = make_plan(gpu, jobs)
    before = gpu.get_tuning(0, 0)

    def decode():
        p, _ = make_plan(gpu, jobs)
        p.launch()
        torch.cuda.synchronize()
        return outputs(p)

    ref = decode()
    cands = [dict(before, low_bits=8), dict(before, low_bits=9), dict(before, grid_per_cu=6),
             dict(before, node_cap=64)]
    try:
        res = gpu.autotune_batch(order, plan.code_index, plan.M, plan.cap, plan.noise_var,
                                 plan.rx_offset, plan.rx, candidates=cands, reps=2)
        timed = [t for t in res["table"] if t["ms"] is not None]
        assert len(timed) >= 3
        assert any(t["tuning"]["node_cap"] == 64 for t in [t for t in res["table"]
                                                             if t["ms"] is None])
        assert gpu.get_tuning(0, 0) == res["best"]
        got = decode()
        for x, y in zip(got[:4], ref[:4]):   # performed checks depend on the tuning
            assert np.array_equal(x, y)
    finally:
        gpu.set_tuning(0, 0, **before)
