"""Full-size workloads on the GPU: every codeword is checked for properties
that hold at any size, and a seeded sample is compared bit-exactly with the
oracle (which cannot decode the whole workload in test time)."""
import time

import numpy as np
import pytest

import workload as w
from helpers import GpuCodes, assert_parity, gpu_batch, oracle_results
import oracle

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


def check_properties(jobs, res):
    """Zero syndrome for accepted words, the hard word on abandonment,
    1 <= q <= cap, checks >= q, no device errors."""
    gcw, gq, gab, gst, gchk = res
    n = len(jobs)
    assert np.all(gst[:n] == 0), np.unique(gst)
    q = gq[:n].astype(np.int64)
    caps = np.array([j.cap for j in jobs], np.int64)
    assert np.all((q >= 1) & (q <= caps))
    acc = gab[:n] == 0
    assert np.all(gchk[:n][acc].astype(np.int64) >= q[acc])
    by_n = {}
    for i, j in enumerate(jobs):
        by_n.setdefault((j.N, j.K), []).append(i)
    for (N, K), idx in by_n.items():
        idx = np.array(idx)
        bits = w.unpack_bits(gcw[idx, : (N + 63) // 64], N).astype(np.int64)
        syn = bits @ w.polar_code(N, K).h_dense.T.astype(np.int64) % 2
        ok = acc[idx]
        assert not syn[ok].any(), "accepted word with a nonzero syndrome"
        for k in idx[~ok]:
            yhat, _, _ = oracle.demap(N, jobs[k].M, jobs[k].rx)
            assert int(gq[k]) == jobs[k].cap
            assert np.array_equal(w.unpack_bits(gcw[k, : (N + 63) // 64], N), yhat)


def run_config(name, sample, seed):
    jobs = w.config_jobs(name)
    t0 = time.perf_counter()
    res = gpu_batch(jobs)
    say(f"{name}: {len(jobs)} words on the GPU in {time.perf_counter() - t0:.3f}s "
        f"(incl. staging), mean q {res[1][:len(jobs)].astype(float).mean():.0f}, "
        f"abandoned {res[2][:len(jobs)].mean():.3f}")
    check_properties(jobs, res)
    idx = np.sort(np.random.default_rng(seed).choice(len(jobs), size=sample, replace=False))
    sub = [jobs[i] for i in idx]
    o = oracle_results(sub)
    assert_parity(sub, tuple(x[idx] for x in res), o, label=name)


def test_polar128_16qam_full(gpu):
    run_config("polar128_16qam", sample=512, seed=1)


def test_uneven_mix_full(gpu):
    run_config("uneven_mix", sample=192, seed=2)


def test_polar1024_256qam_full(gpu):
    run_config("polar1024_256qam", sample=16, seed=3)


def test_polar1024_256qam_hits_match_oracle(gpu):
    """The long-codeword config's words (N = 1024, 256-QAM, cap 2^20) at
    Eb/N0 where the search finds codewords (15-19 dB; at the config's own
    10-14 dB every word abandons): hits deep in the order and abandons, bit
    exact with the oracle."""
    jobs = w.jobs_from_spec("polar1024_256qam_hi", seed=40, count=32, cap=1 << 20, Ns=(1024,),
                            Ms=(256,), ebn0=("uniform", 15.0, 19.0))
    res = gpu_batch(jobs)
    check_properties(jobs, res)
    o = oracle_results(jobs)
    ab = np.asarray(o[2])
    q = np.asarray(o[1])
    assert ab.sum() > 0 and (ab == 0).sum() > 0
    assert np.any((ab == 0) & (q > 1000))
    assert_parity(jobs, res, o, label="polar1024_256qam at 15-19 dB")
