"""The measured bitwise peak (grand_probe_xor_rate) that the decode kernel's
roofline is checked against: positive, and within a plausible range of the
chip's unit-count figure (256 CUs x 128 lanes/clk x 2.4 GHz, the per-lane
rate behind the fp32 vector peak)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

DATASHEET = 256 * 128 * 2.4e9


def test_xor_rate_probe_is_plausible():
    import torch
    import paper_2405_01808_amd as g
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    g.init(0)
    rate, sec = g.probe_xor_rate(1 << 12)
    print(f"xor lane-ops/s {rate:.4g} ({rate / DATASHEET:.3f} of 78.6 T), {sec * 1e3:.3f} ms")
    assert sec > 0
    assert 0.3 * DATASHEET < rate < 1.1 * DATASHEET


@pytest.mark.parametrize("N,words", [(16, 64), (8, 8)])
def test_dense_pmult_baseline_counts_every_codeword(N, words):
    """With 65536 patterns over N <= 16 positions, the patterns cover every
    N-bit vector 65536 / 2^N times, so the zero syndromes of each word are
    exactly (65536 / 2^N) x 2^K: the baseline really forms H (yhat + e)."""
    import torch
    import workload as w
    import paper_2405_01808_amd as g
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    g.init(0)
    code = g.Code(N, w.polar_code(N, N // 2).h_rows)
    rate, zeros = g.probe_dense_pmult(code, words, 65536)
    print(f"dense pMult N={N}: {rate:.4g} checks/s, {zeros} zero syndromes")
    assert rate > 0
    assert zeros == words * (65536 >> N) * (1 << (N // 2))


@pytest.mark.parametrize("cfg,N,K,count", [("polar128_16qam", 128, 64, 48),
                                           ("polar1024_256qam", 1024, 512, 8)])
def test_pmult_matches_oracle_algorithm1(cfg, N, K, count):
    """grand_pmult (one full Algorithm 1 product per vector) against the
    oracle's Algorithm 1, element by element, on workload vectors yhat + e:
    the hard decisions of the config's received words, each with its first 24
    test error patterns in decoding order (items ranked by (cost, position))."""
    import torch
    import workload as w
    import oracle
    import paper_2405_01808_amd as g
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    g.init(0)
    cw = w.polar_code(N, K)
    code = g.Code(N, cw.h_rows)
    vecs = []
    for j in w.config_jobs(cfg, count=count):
        yhat, cost, pos = oracle.demap(N, j.M, j.rx)
        rank = np.lexsort((pos, cost))
        masks, _ = oracle.enumerate_teps(cost[rank], 24)
        for m in masks:
            e = np.zeros(N, np.uint8)
            for r in range(len(rank)):
                if (int(m[r // 64]) >> (r % 64)) & 1:
                    e[pos[rank[r]]] ^= 1
            vecs.append(yhat ^ e)
    vecs = np.array(vecs, np.uint8)
    x = torch.from_numpy(w.pack_bits(vecs).view(np.int64)).cuda()
    syn = g.pmult(code, x).cpu().numpy().view(np.uint64)
    got = w.unpack_bits(syn, N - K)
    for i, v in enumerate(vecs):
        r, _, _, _ = oracle.pmult(cw.h_dense, v)
        assert np.array_equal(got[i], r), (cfg, i)
    # the vectors include codewords' neighbourhoods: some syndromes are zero
    # only if a pattern hits; at least the syndromes are not all equal
    assert len({bytes(s) for s in got}) > len(vecs) // 2
