"""A stream's device job tables are reused by a batch whose tables are
identical to the last upload.  These tests change one thing at a time
between calls on one stream (the words' M, their caps, the received values
behind an unchanged table, a single decode in between) and check every call
against the oracle, bit-exact."""
import copy

import numpy as np
import pytest

import workload as w
from helpers import GpuCodes, assert_parity, gpu_batch, oracle_results

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def gpu():
    import torch
    import paper_2405_01808_amd as g
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    g.init(0)
    return g


def test_tables_follow_metadata_changes(gpu):
    codes = GpuCodes()
    a = w.jobs_from_spec("resA", seed=21, count=40, cap=3000, Ns=(64,), Ms=(16,),
                         ebn0=("uniform", 2.0, 9.0))
    b = w.jobs_from_spec("resB", seed=22, count=40, cap=3000, Ns=(64,), Ms=(64,),
                         ebn0=("uniform", 4.0, 12.0))
    c = copy.deepcopy(a)                 # same words, other caps: only the caps differ
    for i, j in enumerate(c):
        j.cap = 50 + 37 * i
    orc = {"a": oracle_results(a), "b": oracle_results(b), "c": oracle_results(c)}
    sets = {"a": a, "b": b, "c": c}
    code = gpu.Code(64, w.polar_code(64, 32).h_rows)
    for step, name in enumerate(["a", "a", "b", "c", "a", "single", "a", "c", "c"]):
        say(f"call {step}: {name}")
        if name == "single":
            j = b[3]
            cw, q, ab = gpu.decode(code, j.rx, j.M, j.noise_var, j.cap)
            assert (q, ab) == (int(orc["b"][1][3]), int(orc["b"][2][3]))
            assert np.array_equal(cw, orc["b"][0][3])
            continue
        assert_parity(sets[name], gpu_batch(sets[name], codes), orc[name], label=f"{step}:{name}")


def test_new_received_values_behind_an_unchanged_table(gpu):
    """The table holds offsets, not values: overwriting the received values
    in place and launching the same plan again decodes the new values."""
    import torch
    first = w.jobs_from_spec("rxA", seed=31, count=48, cap=4000, Ns=(128,), Ms=(16,),
                             ebn0=("uniform", 3.0, 7.0))
    second = w.jobs_from_spec("rxB", seed=32, count=48, cap=4000, Ns=(128,), Ms=(16,),
                              ebn0=("uniform", 3.0, 7.0))
    for j, k in zip(first, second):      # identical tables, other received values
        k.noise_var = j.noise_var
    codes = GpuCodes()
    idx = np.array([codes.index(j.N, j.K) for j in first], np.uint32)
    L2 = len(first[0].rx)
    offs = np.arange(len(first), dtype=np.uint64) * L2
    rx = torch.from_numpy(np.concatenate([j.rx for j in first])).cuda()
    plan = gpu.BatchPlan(codes.order, idx, [j.M for j in first], [j.cap for j in first],
                         [j.noise_var for j in first], offs, rx)

    def run():
        out = plan.launch(None)
        torch.cuda.synchronize()
        return (out.codewords.cpu().numpy().view(np.uint64),
                out.queries.cpu().numpy().view(np.uint64), out.abandoned.cpu().numpy(),
                out.status.cpu().numpy(), out.checks.cpu().numpy().view(np.uint64))

    for name, jobs in [("first", first), ("first again", first), ("second", second)]:
        say(name)
        rx.copy_(torch.from_numpy(np.concatenate([j.rx for j in jobs])))
        torch.cuda.synchronize()
        assert_parity(jobs, run(), oracle_results(jobs), label=name)


def test_longer_batch_with_the_same_leading_words(gpu):
    """A batch whose first words match the last upload but which has more
    words uploads again; then the shorter batch again."""
    codes = GpuCodes()
    full = w.jobs_from_spec("prefix", seed=41, count=56, cap=3000, Ns=(64,), Ms=(16,),
                            ebn0=("uniform", 2.0, 9.0))
    short = full[:40]
    orc_full, orc_short = oracle_results(full), oracle_results(short)
    for name, jobs, orc in [("short", short, orc_short), ("full", full, orc_full),
                            ("short again", short, orc_short)]:
        say(name)
        assert_parity(jobs, gpu_batch(jobs, codes), orc, label=name)
