"""Algorithm 2's symbol cut-off on the GPU (grand_decode_batch with
cutoff_symbols, grand_decode_ex) against the oracle's cut-off mode, bit for
bit: decoded word, query count and abandon flag.  The cases cover every
configuration's shapes, 64-QAM words whose last symbol carries pad bits, the
largest symbol count (N = 1024 QPSK, 512 symbols), S = 1, S = Section IV's 8,
and S at or beyond the symbol count (the full pattern space)."""
import numpy as np
import pytest

import workload as w
from helpers import GpuCodes, assert_parity, gpu_batch, h_rows, oracle_results

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch
    import paper_2405_01808_amd as g
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    g.init(0)
    return g


def workload_cases():
    return [
        ("polar32_qpsk", w.config_jobs("polar32_qpsk", count=300), (1, 3, 8)),
        ("polar128_16qam", w.config_jobs("polar128_16qam", count=256), (2, 8)),
        ("uneven_mix", w.config_jobs("uneven_mix", count=400, cap=1 << 16), (4, 8)),
        ("polar1024_256qam", w.config_jobs("polar1024_256qam", count=48), (8,)),
        ("serving_mix", w.config_jobs("serving_mix", count=300, cap=1 << 16), (8,)),
        ("qam64_pad", w.jobs_from_spec("qam64_pad", 10, 120, 1 << 16, (32, 64, 128), (64,),
                                       ("uniform", 0.0, 8.0)), (1, 2, 6)),
        ("qpsk1024", w.jobs_from_spec("qpsk1024", 9, 24, 1 << 16, (1024,), (4,),
                                      ("uniform", 2.0, 8.0)), (8,)),
    ]


@pytest.mark.parametrize("case", range(7))
def test_cutoff_batch_matches_oracle(gpu, case):
    name, jobs, cuts = workload_cases()[case]
    for S in cuts:
        print(f"cutoff batch {name}: {len(jobs)} words, S = {S}", flush=True)
        orc = oracle_results(jobs, cutoff=S)
        res = gpu_batch(jobs, cutoff=S)
        assert_parity(jobs, res, orc, label=f"{name} S={S}")
        # the kept flips bound the search: q <= 4^S
        assert int(res[1].max()) <= 4 ** S


def test_cutoff_at_or_beyond_symbol_count_is_the_full_search(gpu):
    jobs = w.config_jobs("polar32_qpsk", count=200)
    L = w.symbols_per_codeword(32, 4)
    codes = GpuCodes()
    full = gpu_batch(jobs, codes)
    for S in (L, L + 1, 1 << 30):
        cut = gpu_batch(jobs, codes, cutoff=S)
        for a, b in zip(full, cut):
            assert np.array_equal(a, b), S
    assert_parity(jobs, full, oracle_results(jobs))


def test_decode_ex_single_words_match_oracle(gpu):
    import oracle
    for name, count in (("polar32_qpsk", 12), ("polar128_16qam", 8), ("uneven_mix", 12)):
        for j in w.config_jobs(name, count=count, cap=1 << 16):
            code = gpu.Code(j.N, h_rows(j.N, j.K))
            for S in (1, 8):
                print(f"decode_ex {name} N={j.N} M={j.M} S={S}", flush=True)
                cw, q, ab = gpu.decode(code, j.rx, j.M, j.noise_var, j.cap, cutoff=S)
                ocw, oq, oab = oracle.decode_ex(h_rows(j.N, j.K), j.N, j.rx, j.M, j.noise_var,
                                                j.cap, S)
                assert (q, ab) == (oq, oab)
                assert np.array_equal(cw, ocw)
