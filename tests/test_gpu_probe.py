"""The measured bitwise peak (grand_probe_xor_rate) that the decode kernel's
roofline is checked against: positive, and within a plausible range of the
chip's unit-count figure (256 CUs x 128 lanes/clk x 2.4 GHz, the per-lane
rate behind the fp32 vector peak)."""
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
