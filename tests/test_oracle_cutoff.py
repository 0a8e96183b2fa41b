"""Pins for Algorithm 2's symbol cut-off (Steps 1-3) in the oracle.

Step 1 ranks each symbol by L(r, s) of Definition 3.1: the distance from the
received point to the corner that its decision cell shares with its three
near-neighbour candidates.  Here that corner is found from plain geometry
(the midpoints between each axis's nearest and second-nearest amplitudes),
independently of the decoder's formulas.  Steps 2-3 keep the S symbols with
the smallest L (ties by index), and Step 4 tests all combinations of their
candidates; the expected decode is a brute-force search over every codeword
of a small code that differs from the hard decision only on those symbols."""
import itertools

import numpy as np
import pytest

import workload as w
from test_oracle_decode import axis_table, quantize

ONE = 4096
BIG_CAP = 1 << 40


def geometry(rx, M):
    """Hard and second-nearest amplitude per (symbol, axis) and the squared
    distance (in units of 1/ONE^2) from the quantised point to the corner."""
    m = w.bits_per_axis(M)
    levels = 1 << m
    amps = np.arange(-(levels - 1), levels, 2)
    xq = quantize(rx).reshape(-1, 2)
    L = xq.shape[0]
    hard = np.zeros((L, 2), np.int64)
    nbr = np.zeros((L, 2), np.int64)
    for i in range(L):
        for a in range(2):
            d = (xq[i, a] - amps * ONE) ** 2
            order = sorted(range(len(amps)), key=lambda k: (d[k], -amps[k]))
            hard[i, a], nbr[i, a] = amps[order[0]], amps[order[1]]
    corner2 = (hard + nbr) * (ONE // 2)        # corner coordinates times ONE
    dist2 = ((xq - corner2) ** 2).sum(axis=1)
    return xq, hard, nbr, dist2


def expected_selection(rx, M, S):
    _, _, _, dist2 = geometry(rx, M)
    order = sorted(range(len(dist2)), key=lambda i: (int(dist2[i]), i))
    sel = np.zeros(len(dist2), bool)
    sel[order[:min(S, len(dist2))]] = True
    return sel


def brute_cutoff(code, rx, M, cap, sel):
    N = code.N
    m = w.bits_per_axis(M)
    L = w.symbols_per_codeword(N, M)
    assert 2 * m * L == N, "brute force assumes no pad bits"
    xq, hard, nbr, _ = geometry(rx, M)
    tab = axis_table(M)
    items = []
    for i in range(L):
        if not sel[i]:
            continue
        for a in range(2):
            hb, nb = tab[int(hard[i, a])], tab[int(nbr[i, a])]
            diff = [k for k in range(m) if hb[k] != nb[k]]
            pos = 2 * m * i + m * a + diff[0]
            num = (xq[i, a] - nbr[i, a] * ONE) ** 2 - (xq[i, a] - hard[i, a] * ONE) ** 2
            items.append((int(num // (4 * ONE)), pos, i, a))
    ranked = sorted(items, key=lambda t: (t[0], t[1]))
    rank_of = {(t[2], t[3]): r for r, t in enumerate(ranked)}
    n = len(ranked)
    yhat = np.array([b for i in range(L) for a in range(2) for b in tab[int(hard[i, a])]],
                    np.uint8)
    best = None
    for u in itertools.product([0, 1], repeat=code.K):
        c = code.encode(np.array(u, np.uint8))
        pts = w.modulate(c, M).reshape(L, 2)
        if not np.all((pts == hard) | ((pts == nbr) & sel[:, None])):
            continue
        dist = int(((xq - pts * ONE) ** 2).sum())
        mask = sum(1 << rank_of[(i, a)] for i in range(L) for a in range(2)
                   if pts[i, a] != hard[i, a])
        if best is None or (dist, mask) < best[0]:
            best = ((dist, mask), c)
    costs = [t[0] for t in ranked]
    if best is None:
        return yhat, min(cap, 1 << n), 1
    (dist, mask), c = best
    cstar = sum(costs[r] for r in range(n) if (mask >> r) & 1)
    below = sum(1 for T in range(1 << n)
                if (sum(costs[r] for r in range(n) if (T >> r) & 1), T) < (cstar, mask))
    q = below + 1
    if q > cap:
        return yhat, cap, 1
    return c, q, 0


def noisy_rx(code, M, rng, lo=-1.0, hi=8.0):
    u = rng.integers(0, 2, code.K, dtype=np.uint8)
    c = code.encode(u)
    s2 = w.noise_variance(M, rng.uniform(lo, hi))
    rx = w.awgn(w.modulate(c, M).astype(np.float64), s2, rng).reshape(-1)
    return np.clip(rx, -(2 ** int(np.log2(M))), 2 ** int(np.log2(M))), s2


@pytest.mark.parametrize("N,M", [(16, 4), (32, 16), (64, 64), (128, 256), (1024, 4)])
def test_selection_is_the_least_reliable_symbols_by_corner_distance(orc, N, M):
    code = w.polar_code(N, N // 2)
    rng = np.random.default_rng(31 * N + M)
    for trial in range(10):
        rx, _ = noisy_rx(code, M, rng)
        for S in (1, 3, 8, 10 ** 6):
            got = orc.select_symbols(N, M, rx, S)
            assert np.array_equal(got, expected_selection(rx, M, S)), (trial, S)


def test_selection_ties_go_to_lower_symbol_indices(orc):
    # every symbol on a lattice point (the same L), except two nudged toward a
    # corner: those two come first, then the lowest indices
    N, M = 16, 16
    L = w.symbols_per_codeword(N, M)
    rx = np.full(2 * L, 1.0, np.float32)
    rx[2 * 2], rx[2 * 2 + 1] = 1.9, 1.8      # symbol 2, near the corner (2, 2)
    rx[2 * 3], rx[2 * 3 + 1] = -0.2, 0.15    # symbol 3, near the corner (0, 0)
    assert list(np.flatnonzero(orc.select_symbols(N, M, rx, 1))) == [2]
    assert list(np.flatnonzero(orc.select_symbols(N, M, rx, 2))) == [2, 3]
    assert list(np.flatnonzero(orc.select_symbols(N, M, rx, 3))) == [0, 2, 3]


def test_cutoff_covering_every_symbol_is_the_full_decode(orc):
    for name in ("polar32_qpsk", "polar128_16qam"):
        for j in w.config_jobs(name, count=6):
            L = w.symbols_per_codeword(j.N, j.M)
            H = w.polar_code(j.N, j.K).h_rows
            full = orc.decode(H, j.N, j.rx, j.M, j.noise_var, j.cap)
            for S in (L, L + 5):
                cut = orc.decode_ex(H, j.N, j.rx, j.M, j.noise_var, j.cap, S)
                assert cut[1:] == full[1:] and np.array_equal(cut[0], full[0])


@pytest.mark.parametrize("N,M,S", [(16, 4, 1), (16, 4, 2), (16, 4, 3), (16, 4, 5),
                                   (16, 16, 1), (16, 16, 2), (16, 16, 3), (8, 4, 2)])
def test_cutoff_decode_matches_brute_force(orc, N, M, S):
    code = w.polar_code(N, N // 2)
    rng = np.random.default_rng(7 * N + 13 * M + S)
    hits = 0
    for trial in range(20):
        rx, s2 = noisy_rx(code, M, rng)
        sel = expected_selection(rx, M, S)
        exp_c, exp_q, exp_ab = brute_cutoff(code, rx, M, BIG_CAP, sel)
        cw, q, ab = orc.decode_ex(code.h_rows, N, rx, M, s2, BIG_CAP, S)
        assert (q, ab) == (exp_q, exp_ab), (trial, q, ab, exp_q, exp_ab)
        assert np.array_equal(w.unpack_bits(cw, N), exp_c)
        hits += 1 - exp_ab
    assert hits > 0


def test_cutoff_tests_exactly_4_to_the_S_patterns(orc):
    """With no zero syndrome among the candidates, the search abandons after
    all 4^S combinations (Proposition 3.1's 4^S instances)."""
    code = w.polar_code(128, 64)
    rng = np.random.default_rng(5)
    seen = 0
    for trial in range(40):
        rx, s2 = noisy_rx(code, 16, rng, 0.0, 1.0)
        for S in (2, 4, 6):
            cw, q, ab = orc.decode_ex(code.h_rows, 128, rx, 16, s2, BIG_CAP, S)
            if ab:
                assert q == 4 ** S
                seen += 1
            else:
                assert 1 <= q <= 4 ** S
    assert seen > 0
