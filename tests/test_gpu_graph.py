"""Batch graphs (grand_graph_*): replays of a captured batch equal the eager
batch path, across replays with other work and synchronisations between
them, and after the received values in the captured buffer change."""
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


def clear(plan):
    o = plan.out
    for t in (o.codewords, o.queries, o.abandoned, o.checks):
        t.zero_()
    o.status.fill_(123)


def assert_same(a, b, what):
    for x, y, name in zip(a, b, ("codewords", "queries", "abandoned", "status", "checks")):
        assert np.array_equal(x, y), f"{what}: {name} differ"


@pytest.mark.parametrize("case", ["merged", "per_bucket"])
def test_graph_replays_equal_eager_batch(gpu, case):
    import torch
    if case == "merged":      # small (n, M) buckets: one merged launch
        jobs = w.config_jobs("uneven_mix", count=1536, cap=1 << 12)
    else:                     # two buckets that each fill the device: two launches
        jobs = w.jobs_from_spec("graph2", seed=21, count=4400, cap=1 << 10, Ns=(32, 64),
                                Ms=(4,), ebn0=("uniform", 2.0, 6.0))
    plan, _ = make_plan(gpu, jobs)
    other, _ = make_plan(gpu, w.config_jobs("polar128_16qam", count=256, cap=1 << 12))
    stream = torch.cuda.current_stream()
    plan.launch(stream)
    torch.cuda.synchronize()
    ref = outputs(plan)
    assert np.all(ref[3][:len(jobs)] == 0)
    graph = gpu.BatchGraph(plan)
    for rep in range(3):
        clear(plan)
        graph.launch(stream)
        torch.cuda.synchronize()
        assert_same(outputs(plan), ref, f"replay {rep}")
        other.launch(stream)          # eager work between replays
        torch.cuda.synchronize()
    # new received values in the captured buffer: swap words of equal length
    rng = np.random.default_rng(5)
    by_len = {}
    for i, j in enumerate(jobs):
        by_len.setdefault(len(j.rx), []).append(i)
    perm = list(range(len(jobs)))
    for idx in by_len.values():
        sh = list(rng.permutation(idx))
        for a, b in zip(idx, sh):
            perm[a] = b
    new_jobs = [jobs[perm[i]] for i in range(len(jobs))]
    plan.rx.copy_(torch.from_numpy(np.concatenate([j.rx for j in new_jobs])).cuda())
    clear(plan)
    graph.launch(stream)
    torch.cuda.synchronize()
    got = outputs(plan)
    clear(plan)
    plan.launch(stream)
    torch.cuda.synchronize()
    assert_same(got, outputs(plan), "after new rx")
    assert not np.array_equal(got[1], ref[1])    # the inputs really changed
    graph.close()
