"""Serving: continuous batching of a request stream through the native
server, against single decodes and the oracle."""
import time

import numpy as np
import pytest

import workload as w
from helpers import oracle_results

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch
    import paper_2405_01808_amd as g
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    g.init(0)
    return g


class Codes:
    def __init__(self, g):
        self.g = g
        self.by_key = {}
        self.order = []

    def index(self, N, K):
        if (N, K) not in self.by_key:
            self.by_key[(N, K)] = len(self.order)
            self.order.append(self.g.Code(N, w.polar_code(N, K).h_rows))
        return self.by_key[(N, K)]


def make_trace(g, jobs, rate, codes):
    idx = [codes.index(j.N, j.K) for j in jobs]
    arrivals = np.cumsum(np.random.default_rng(11).exponential(1.0 / rate, len(jobs)))
    return g.Trace(codes.order, idx, [j.M for j in jobs], [j.cap for j in jobs],
                   [j.noise_var for j in jobs], [j.rx for j in jobs], arrivals)


def test_mix_results_equal_single_decodes_and_oracle(gpu):
    jobs = w.config_jobs("serving_mix", count=600, cap=1 << 14)
    codes = Codes(gpu)
    trace = make_trace(gpu, jobs, 5e4, codes)
    srv = gpu.Server(max_inflight=256, lanes=4, max_batch=128, memory_budget=1 << 30)
    res, wall = trace.run_server(srv)
    print(f"served {len(jobs)} requests in {wall * 1e3:.1f} ms", flush=True)
    assert all(r.status == 0 for r in res)
    for i, (j, r) in enumerate(zip(jobs, res)):
        code = codes.order[codes.index(j.N, j.K)]
        cw, q, ab = gpu.decode(code, j.rx, j.M, j.noise_var, j.cap)
        nw = (j.N + 63) // 64
        assert (r.queries, r.abandoned) == (q, ab), i
        assert np.array_equal(r.codeword[:nw], cw), i
        assert r.complete_s >= r.submit_s >= r.arrival_s - 1e-6
    sample = list(range(0, 600, 15))
    ocw, oq, oab = oracle_results([jobs[i] for i in sample])
    for k, i in enumerate(sample):
        nw = (jobs[i].N + 63) // 64
        assert (res[i].queries, res[i].abandoned) == (int(oq[k]), int(oab[k])), i
        assert np.array_equal(res[i].codeword[:nw], ocw[k]), i


def test_admission_refusal_and_cancel_leave_no_state(gpu):
    codes = Codes(gpu)
    jobs = w.config_jobs("serving_mix", count=8, cap=1 << 10)
    need = max(gpu.request_bytes(j.N, j.M) for j in jobs)
    srv = gpu.Server(max_inflight=3, lanes=1, max_batch=8, memory_budget=3 * need)
    ids = []
    for j in jobs[:3]:
        ids.append(srv.submit(codes.order[codes.index(j.N, j.K)], j.rx, j.M, j.noise_var, j.cap))
    j = jobs[3]
    assert srv.try_submit(codes.order[codes.index(j.N, j.K)], j.rx, j.M, j.noise_var, j.cap) is None
    st = srv.stats()
    assert st["pending"] == 3 and st["memory_in_use"] > 0
    srv.cancel(ids[1])
    with pytest.raises(gpu.GrandError):
        srv.cancel(ids[1])
    assert srv.stats()["pending"] == 2
    got = []
    t0 = time.time()
    while len(got) < 2 and time.time() - t0 < 30:
        got += srv.poll()
    assert sorted(r.request_id for r in got) == sorted([ids[0], ids[2]])
    st = srv.stats()
    assert st == {"pending": 0, "running": 0, "memory_in_use": 0}
    # room again after draining
    assert srv.try_submit(codes.order[codes.index(j.N, j.K)], j.rx, j.M, j.noise_var, j.cap)
    t0 = time.time()
    got = []
    while not got and time.time() - t0 < 30:
        got = srv.poll()
    assert srv.stats()["memory_in_use"] == 0


def test_light_request_overtakes_heavy_one(gpu):
    """A request admitted while a long decode runs is launched on another
    lane and finishes first (batches overlap on the device)."""
    codes = Codes(gpu)
    heavy = w.jobs_from_spec("heavy", seed=3, count=1, cap=1 << 18, Ns=(1024,), Ms=(4,),
                             ebn0=("fixed", 1.0))[0]
    light = w.jobs_from_spec("light", seed=4, count=1, cap=1 << 18, Ns=(32,), Ms=(4,),
                             ebn0=("fixed", 12.0))[0]
    srv = gpu.Server(max_inflight=16, lanes=2, max_batch=8, memory_budget=1 << 30)
    hid = srv.submit(codes.order[codes.index(1024, 512)], heavy.rx, 4, heavy.noise_var, heavy.cap)
    srv.poll()                                  # heavy goes to lane 0
    lid = srv.submit(codes.order[codes.index(32, 16)], light.rx, 4, light.noise_var, light.cap)
    order = []
    t0 = time.time()
    while len(order) < 2 and time.time() - t0 < 60:
        order += [r.request_id for r in srv.poll()]
    assert order == [lid, hid]
