"""Pins for the oracle's demapper (Algorithm 2 Step 1; Definitions 3.1, 3.2).

The checks use plain geometry computed here by exhaustive search over the
constellation, and the workload's own modulator (a separate implementation
of the Gray labelling), never the oracle's formulas."""
import json
import math
import os

import numpy as np
import pytest

import workload as w

ONE = 4096
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
MS = [4, 16, 64, 256, 1024, 4096]


def quantize(x):
    return np.rint(np.float64(np.float32(x)) * ONE).astype(np.int64)   # half to even


def geometry(xq, levels):
    """Brute force on one axis: nearest amplitude (ties to the upper one), the
    nearest other amplitude (ties to the upper one) and the penalty
    ((x - t)^2 - (x - s)^2) / (4 ONE) in units of 1/ONE."""
    amps = np.arange(-(levels - 1), levels, 2)
    d = (xq - amps * ONE) ** 2
    order = sorted(range(len(amps)), key=lambda k: (d[k], -amps[k]))
    s, t = amps[order[0]], amps[order[1]]
    num = int((xq - t * ONE) ** 2 - (xq - s * ONE) ** 2)
    assert num % (4 * ONE) == 0
    return int(s), int(t), num // (4 * ONE)


def axis_samples(levels, rng, k=300):
    edge = levels + 2.0
    xs = list(rng.uniform(-edge, edge, k))
    # decision boundaries, centres, and points beyond the outermost levels
    xs += [float(b) for b in range(-(levels - 2), levels - 1, 2)]
    xs += [float(a) for a in range(-(levels - 1), levels, 2)]
    xs += [levels + 5.25, -(levels + 7.5), 0.0, 1.0 / ONE, -1.0 / ONE, 0.5 / ONE]
    return np.array(xs, dtype=np.float32)


@pytest.mark.parametrize("M", MS)
def test_hard_decision_cost_and_neighbour_match_geometry(orc, M):
    m = w.bits_per_axis(M)
    levels = 1 << m
    rng = np.random.default_rng(M)
    xs = axis_samples(levels, rng)
    N = 1 << math.ceil(math.log2(2 * m))   # symbol 0 is tested, the rest is filler
    L = w.symbols_per_codeword(N, M)
    for a, b in zip(xs, xs[::-1]):
        rx = np.full(2 * L, 0.5, np.float32)
        rx[0], rx[1] = a, b
        yhat, cost, pos = orc.demap(N, M, rx)
        mine = [i for i in range(len(pos)) if pos[i] < 2 * m]
        assert len(mine) == 2     # Corollary 3.1: exactly 2 flips -> 4 candidates
        for axis, x in enumerate((a, b)):
            s, t, pen = geometry(quantize(x), levels)
            # hard decision: the modulator maps the returned bits to s
            sym = w.modulate(yhat.astype(np.int64), M).reshape(-1)
            assert sym[axis] == s
            # the item of this axis flips the bit that moves s to t
            k = [i for i in mine if (pos[i] >= m) == bool(axis)]
            assert len(k) == 1
            flipped = yhat.copy()
            flipped[pos[k[0]]] ^= 1
            sym2 = w.modulate(flipped.astype(np.int64), M).reshape(-1)
            assert sym2[axis] == t and sym2[1 - axis] == sym[1 - axis]
            # cost = (|r - t|^2 - |r - s|^2) / 4 in units of 1/ONE
            assert cost[k[0]] == min(pen, 32767)


@pytest.mark.parametrize("M", [4, 16, 64, 256])
def test_definition_3_1_interior_formula(orc, M):
    """Where the neighbour lies on the received value's side, the cost is
    Definition 3.1's d = 1 - |A - a| (to the 1/4096 grid)."""
    m = w.bits_per_axis(M)
    levels = 1 << m
    rng = np.random.default_rng(11)
    N = 1 << math.ceil(math.log2(2 * m))
    L = w.symbols_per_codeword(N, M)
    for x in rng.uniform(-(levels - 1), levels - 1, 200).astype(np.float32):
        rx = np.full(2 * L, 0.5, np.float32)
        rx[0] = x
        yhat, cost, pos = orc.demap(N, M, rx)
        A = w.modulate(yhat.astype(np.int64), M).reshape(-1)[0]
        on_side = abs(A + 2 * np.sign(x - A)) <= levels - 1 and x != A
        if on_side:
            ci = [c for c, p in zip(cost, pos) if p < m][0]
            assert abs(ci / ONE - (1 - abs(A - float(x)))) <= 0.5 / ONE + 1e-12


@pytest.mark.parametrize("M", MS)
@pytest.mark.parametrize("N", [32, 64, 128, 1024])
def test_noise_free_roundtrip(orc, M, N):
    """Lattice points demap to the transmitted bits, and every flip costs
    exactly one unit (d = 1)."""
    rng = np.random.default_rng(N + M)
    bits = rng.integers(0, 2, N, dtype=np.uint8)
    rx = w.modulate(bits, M).astype(np.float32).reshape(-1)
    yhat, cost, pos = orc.demap(N, M, rx)
    assert np.array_equal(yhat, bits)
    L = w.symbols_per_codeword(N, M)
    m = w.bits_per_axis(M)
    if 2 * m * L == N:
        assert len(cost) == 2 * L
    else:
        assert 2 * (L - 1) <= len(cost) <= 2 * L
    assert np.all(cost == ONE)
    assert np.all(pos < N)
    assert len(set(pos.tolist())) == len(pos)


def test_worked_example_symbol_counts(orc):
    g = json.load(open(os.path.join(GOLDEN, "symbols_64qam_n32.json")))
    for case in g["cases"]:
        N, M = case["N"], case["M"]
        L = w.symbols_per_codeword(N, M)
        assert L == case["L"]
        assert L * int(math.log2(M)) == case["bits"]
        rx = np.zeros(2 * L, np.float32) + 0.3
        yhat, cost, pos = orc.demap(N, M, rx)
        # Pad bits are not part of the codeword and carry no flips.
        assert np.all(pos < N) and len(yhat) == N


@pytest.mark.parametrize("M,L", [(4, 8), (16, 4), (16, 8), (256, 4)])
def test_corollary_pattern_space_is_4_to_the_L(orc, M, L):
    """Corollary 3.1: 4 candidates per symbol, so the pattern space has
    exactly 4^L members (no pad bits when 2m divides N)."""
    m = w.bits_per_axis(M)
    N = 2 * m * L
    assert N & (N - 1) == 0
    rng = np.random.default_rng(5)
    rx = rng.normal(0, 2, 2 * L).astype(np.float32)
    _, cost, _ = orc.demap(N, M, rx)
    assert len(cost) == 2 * L
    masks, costs = orc.enumerate_teps(np.sort(cost), 4 ** L + 10)
    assert len(masks) == 4 ** L
    assert len({int(x) for x in masks[:, 0]}) == 4 ** L


def test_padding_drops_pad_flips(orc):
    # N = 32, 64-QAM: 6 symbols of 6 bits; the last symbol has 4 pad bits.
    rng = np.random.default_rng(9)
    seen_pad = False
    for _ in range(200):
        rx = rng.uniform(-8, 8, 12).astype(np.float32)
        yhat, cost, pos = orc.demap(32, 64, rx)
        assert np.all(pos < 32)
        if len(pos) < 12:
            seen_pad = True
    assert seen_pad


def test_invalid_inputs_rejected(orc):
    with pytest.raises(ValueError):
        orc.demap(32, 8, np.zeros(32, np.float32))
    with pytest.raises(ValueError):
        orc.demap(32, 4, np.array([np.nan] + [0.0] * 31, np.float32))
    with pytest.raises(ValueError):
        orc.demap(32, 4, np.array([40000.0] + [0.0] * 31, np.float32))
    with pytest.raises(ValueError):
        orc.demap(48, 4, np.zeros(48, np.float32))
