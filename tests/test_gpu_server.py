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


def assert_equal_single(gpu, codes, jobs, res):
    for i, (j, r) in enumerate(zip(jobs, res)):
        code = codes.order[codes.index(j.N, j.K)]
        cw, q, ab = gpu.decode(code, j.rx, j.M, j.noise_var, j.cap)
        nw = (j.N + 63) // 64
        assert r.status == 0, i
        assert (r.queries, r.abandoned) == (q, ab), i
        assert np.array_equal(r.codeword[:nw], cw), i
        assert r.complete_s >= r.submit_s >= r.arrival_s - 1e-6


def wait_results(srv, count, limit_s=60):
    got = []
    t0 = time.time()
    while len(got) < count and time.time() - t0 < limit_s:
        got += srv.poll()
    return got


PERSISTENT_OFF = pytest.mark.skip(
    reason="persistent serving mode is switched off: its first GPU run did not finish "
           "(killed for silence) and the cause is not established")


@pytest.mark.parametrize("persistent,wide", [(False, 0), (False, 2),
                                              pytest.param(True, 0, marks=PERSISTENT_OFF)],
                         ids=["lanes", "wide_lanes", "persistent"])
def test_mix_results_equal_single_decodes_and_oracle(gpu, persistent, wide):
    """wide_lanes = 2: long words (2L >= 512) go to two lanes of their own,
    one 1024-thread workgroup each; results are the same."""
    jobs = w.config_jobs("serving_mix", count=600, cap=1 << 14)
    codes = Codes(gpu)
    trace = make_trace(gpu, jobs, 5e4, codes)
    srv = gpu.Server(max_inflight=256, lanes=4 + wide, max_batch=128, memory_budget=1 << 30,
                     persistent=persistent, wide_lanes=wide)
    res, wall = trace.run_server(srv)
    srv.close()
    print(f"served {len(jobs)} requests in {wall * 1e3:.1f} ms", flush=True)
    assert_equal_single(gpu, codes, jobs, res)
    sample = list(range(0, 600, 15))
    ocw, oq, oab = oracle_results([jobs[i] for i in sample])
    for k, i in enumerate(sample):
        nw = (jobs[i].N + 63) // 64
        assert (res[i].queries, res[i].abandoned) == (int(oq[k]), int(oab[k])), i
        assert np.array_equal(res[i].codeword[:nw], ocw[k]), i


def test_serving_mix_at_full_cap_matches_oracle(gpu):
    """The serving mix at its own query cap (2^18): 400 requests of the
    Poisson stream served while others are in flight, every result equal to
    the oracle's and to a single grand_decode of the same request."""
    jobs = w.config_jobs("serving_mix", count=400, start=1000)
    assert all(j.cap == 1 << 18 for j in jobs)
    codes = Codes(gpu)
    trace = make_trace(gpu, jobs, 2e5, codes)
    srv = gpu.Server(max_inflight=1024, lanes=6, max_batch=64, memory_budget=4 << 30,
                     wide_lanes=2)
    res, wall = trace.run_server(srv)
    srv.close()
    print(f"served {len(jobs)} requests at cap 2^18 in {wall * 1e3:.1f} ms", flush=True)
    ocw, oq, oab = oracle_results(jobs)
    assert 0 < int(np.sum(oab)) < len(jobs)          # both hits and abandons
    for i, j in enumerate(jobs):
        nw = (j.N + 63) // 64
        assert res[i].status == 0, i
        assert (res[i].queries, res[i].abandoned) == (int(oq[i]), int(oab[i])), (i, j.N, j.M)
        assert np.array_equal(res[i].codeword[:nw], ocw[i]), i
    assert_equal_single(gpu, codes, jobs[::8], res[::8])


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


@PERSISTENT_OFF
def test_persistent_ring_wraps_with_out_of_order_completion(gpu):
    """Ring of 4 slots, 48 requests of mixed weight: slots are reused while
    earlier ones are still decoding, and publishing waits for the slot."""
    codes = Codes(gpu)
    jobs = w.config_jobs("serving_mix", count=48, cap=1 << 16)
    srv = gpu.Server(max_inflight=4, memory_budget=1 << 30, persistent=True)
    ids, res = {}, {}
    t0 = time.time()
    nxt = 0
    while len(res) < len(jobs) and time.time() - t0 < 60:
        while nxt < len(jobs):
            j = jobs[nxt]
            rid = srv.try_submit(codes.order[codes.index(j.N, j.K)], j.rx, j.M, j.noise_var,
                                 j.cap)
            if rid is None:
                break
            ids[rid] = nxt
            nxt += 1
        for r in srv.poll():
            res[ids[r.request_id]] = r
    assert srv.stats() == {"pending": 0, "running": 0, "memory_in_use": 0}
    srv.close()
    assert len(res) == len(jobs)
    assert_equal_single(gpu, codes, jobs, [res[i] for i in range(len(jobs))])


@PERSISTENT_OFF
def test_persistent_admission_and_cancel(gpu):
    """Persistent mode publishes a request at once: it is refused beyond the
    slot count and cannot be cancelled once submitted."""
    codes = Codes(gpu)
    jobs = w.config_jobs("serving_mix", count=4, cap=1 << 10)
    srv = gpu.Server(max_inflight=3, memory_budget=1 << 30, persistent=True)
    ids = [srv.submit(codes.order[codes.index(j.N, j.K)], j.rx, j.M, j.noise_var, j.cap)
           for j in jobs[:3]]
    j = jobs[3]
    assert srv.try_submit(codes.order[codes.index(j.N, j.K)], j.rx, j.M, j.noise_var, j.cap) is None
    with pytest.raises(gpu.GrandError):
        srv.cancel(ids[0])
    got = wait_results(srv, 3)
    assert sorted(r.request_id for r in got) == sorted(ids)
    assert srv.stats() == {"pending": 0, "running": 0, "memory_in_use": 0}
    srv.close()
    assert_equal_single(gpu, codes, jobs[:3], sorted(got, key=lambda r: r.request_id))


@PERSISTENT_OFF
def test_persistent_kernel_relaunches_after_idle_exit(gpu):
    """The resident kernel leaves after an idle period; later requests
    relaunch it and still decode correctly."""
    codes = Codes(gpu)
    jobs = w.config_jobs("serving_mix", count=6, cap=1 << 12)
    srv = gpu.Server(max_inflight=64, memory_budget=1 << 30, persistent=True)
    res = []
    for k in range(3):
        for j in jobs[2 * k:2 * k + 2]:
            srv.submit(codes.order[codes.index(j.N, j.K)], j.rx, j.M, j.noise_var, j.cap)
        got = wait_results(srv, 2)
        assert len(got) == 2
        res += sorted(got, key=lambda r: r.request_id)
        time.sleep(0.2)                        # longer than the idle limit
    srv.close()
    assert_equal_single(gpu, codes, jobs, res)


@PERSISTENT_OFF
def test_persistent_light_request_overtakes_heavy_one(gpu):
    codes = Codes(gpu)
    heavy = w.jobs_from_spec("heavy", seed=3, count=1, cap=1 << 18, Ns=(1024,), Ms=(4,),
                             ebn0=("fixed", 1.0))[0]
    light = w.jobs_from_spec("light", seed=4, count=1, cap=1 << 18, Ns=(32,), Ms=(4,),
                             ebn0=("fixed", 12.0))[0]
    srv = gpu.Server(max_inflight=16, memory_budget=1 << 30, persistent=True)
    hid = srv.submit(codes.order[codes.index(1024, 512)], heavy.rx, 4, heavy.noise_var, heavy.cap)
    lid = srv.submit(codes.order[codes.index(32, 16)], light.rx, 4, light.noise_var, light.cap)
    order = [r.request_id for r in wait_results(srv, 2)]
    srv.close()
    assert order == [lid, hid]


@PERSISTENT_OFF
def test_persistent_destroy_with_requests_in_flight(gpu):
    """Destroying the server stops the resident kernel even while requests
    are published and unfinished."""
    codes = Codes(gpu)
    jobs = w.jobs_from_spec("heavy", seed=5, count=8, cap=1 << 18, Ns=(1024,), Ms=(4,),
                            ebn0=("fixed", 1.0))
    srv = gpu.Server(max_inflight=64, memory_budget=1 << 30, persistent=True)
    for j in jobs:
        srv.submit(codes.order[codes.index(1024, 512)], j.rx, 4, j.noise_var, j.cap)
    t0 = time.time()
    srv.close()
    assert time.time() - t0 < 10
    # the device is usable afterwards
    j = jobs[0]
    cw, q, ab = gpu.decode(codes.order[codes.index(1024, 512)], j.rx, 4, j.noise_var, 1 << 10)
    assert q >= 1


def test_failed_launch_returns_requests_and_server_recovers(gpu):
    """A launch that fails (forced from the host with the test hook) returns
    its requests as GRAND_EDEVICE results; the server then serves normally."""
    from paper_2405_01808_amd import _native as nat
    codes = Codes(gpu)
    jobs = w.config_jobs("serving_mix", count=12, cap=1 << 10)
    srv = gpu.Server(max_inflight=64, lanes=1, max_batch=64, memory_budget=1 << 30)
    ids = [srv.submit(codes.order[codes.index(j.N, j.K)], j.rx, j.M, j.noise_var, j.cap)
           for j in jobs[:6]]
    nat.lib().grand_debug_fail_launches(1)
    try:
        with pytest.raises(gpu.GrandError):
            srv.poll()                  # this poll's launch fails
    finally:
        nat.lib().grand_debug_fail_launches(0)
    got = wait_results(srv, 6)
    assert sorted(r.request_id for r in got) == sorted(ids)
    assert all(r.status == nat.GRAND_EDEVICE for r in got)
    assert srv.stats() == {"pending": 0, "running": 0, "memory_in_use": 0}
    ids2 = [srv.submit(codes.order[codes.index(j.N, j.K)], j.rx, j.M, j.noise_var, j.cap)
            for j in jobs[6:]]
    got2 = sorted(wait_results(srv, 6), key=lambda r: r.request_id)
    srv.close()
    assert [r.request_id for r in got2] == sorted(ids2)
    assert_equal_single(gpu, codes, jobs[6:], got2)
