"""Back-to-back launches on one stream: the work counters are never reset,
each launch starts from the value the previous launches leave, so batches
of different sizes and bucket counts enqueued without synchronisation (and
a graph replay among them) must give the same results as alone."""
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


def test_queued_batches_equal_batches_alone(gpu):
    import torch
    specs = [("uneven_mix", 700, 1 << 10), ("polar32_qpsk", 3000, 1 << 8),
             ("polar128_16qam", 37, 1 << 12), ("uneven_mix", 1, 1 << 10),
             ("polar32_qpsk", 2049, 1 << 6)]
    plans = []
    for k, (name, count, cap) in enumerate(specs):
        jobs = w.config_jobs(name, count=count, cap=cap, start=100 * k)
        plans.append(make_plan(gpu, jobs)[0])
    # two buckets that each fill the device: launches on two counters
    big = w.jobs_from_spec("order2", seed=41, count=4400, cap=1 << 8, Ns=(32, 64), Ms=(4,),
                           ebn0=("uniform", 2.0, 6.0))
    plans.append(make_plan(gpu, big)[0])
    stream = torch.cuda.current_stream()
    alone = []
    for p in plans:
        p.launch(stream)
        torch.cuda.synchronize()
        alone.append(outputs(p))
    graph = gpu.BatchGraph(plans[0])
    for rnd in range(3):
        for p in plans:
            o = p.out
            for t in (o.codewords, o.queries, o.abandoned, o.checks):
                t.zero_()
        for p in plans:                 # no synchronisation in between
            p.launch(stream)
        graph.launch(stream)            # replays plans[0] into the same outputs
        for p in reversed(plans):
            p.launch(stream)
        torch.cuda.synchronize()
        for i, p in enumerate(plans):
            for x, y in zip(outputs(p), alone[i]):
                assert np.array_equal(x, y), (rnd, i)
    graph.close()
