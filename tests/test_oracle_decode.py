"""Pins for the oracle's decode (Algorithm 2 with the ML statement of
Section II): brute force over every codeword of small codes.

The expected result is computed here from plain geometry: the squared
Euclidean distance from the quantised received point to each candidate
codeword's constellation points (exact integers), the near-neighbour
candidates of Definition 3.2 taken as "each axis at its nearest or its
second-nearest amplitude", and the rank of a pattern counted over all
2^n subsets.  For QPSK every codeword is such a candidate, so the check is
full maximum-likelihood decoding."""
import itertools

import numpy as np
import pytest

import workload as w

ONE = 4096
BIG_CAP = 1 << 40


def quantize(x):
    return np.rint(np.float64(np.asarray(x, np.float32)) * ONE).astype(np.int64)


def axis_table(M):
    """Amplitude -> m label bits (MSB first) of one axis, from the modulator."""
    m = w.bits_per_axis(M)
    tab = {}
    for label in range(1 << m):
        bits = [(label >> (m - 1 - k)) & 1 for k in range(m)]
        amp = int(w.modulate(np.array(bits + [0] * m), M).reshape(-1)[0])
        tab[amp] = bits
    return tab


def brute_decode(code, rx, M, cap):
    N = code.N
    m = w.bits_per_axis(M)
    L = w.symbols_per_codeword(N, M)
    assert 2 * m * L == N, "brute force assumes no pad bits"
    levels = 1 << m
    amps = np.arange(-(levels - 1), levels, 2)
    xq = quantize(rx).reshape(L, 2)
    tab = axis_table(M)
    hard = np.zeros((L, 2), np.int64)
    nbr = np.zeros((L, 2), np.int64)
    for i in range(L):
        for a in range(2):
            d = (xq[i, a] - amps * ONE) ** 2
            order = sorted(range(len(amps)), key=lambda k: (d[k], -amps[k]))
            hard[i, a], nbr[i, a] = amps[order[0]], amps[order[1]]
    # items: the bit that separates the hard and neighbour labels, and the
    # penalty (|r - t|^2 - |r - s|^2) / (4 ONE)
    items = []
    for i in range(L):
        for a in range(2):
            hb, nb = tab[int(hard[i, a])], tab[int(nbr[i, a])]
            diff = [k for k in range(m) if hb[k] != nb[k]]
            assert len(diff) == 1
            pos = 2 * m * i + m * a + diff[0]
            num = (xq[i, a] - nbr[i, a] * ONE) ** 2 - (xq[i, a] - hard[i, a] * ONE) ** 2
            assert num % (4 * ONE) == 0 and num // (4 * ONE) <= 32767
            items.append((int(num // (4 * ONE)), pos, i, a))
    ranked = sorted(items, key=lambda t: (t[0], t[1]))
    rank_of = {(t[2], t[3]): r for r, t in enumerate(ranked)}
    n = len(ranked)
    yhat = np.array([b for i in range(L) for a in range(2) for b in tab[int(hard[i, a])]],
                    np.uint8)
    # candidate codewords: every axis at its hard or neighbour amplitude
    best = None
    for u in itertools.product([0, 1], repeat=code.K):
        c = code.encode(np.array(u, np.uint8))
        pts = w.modulate(c, M).reshape(L, 2)
        if not np.all((pts == hard) | (pts == nbr)):
            continue
        dist = int(((xq - pts * ONE) ** 2).sum())
        mask = sum(1 << rank_of[(i, a)] for i in range(L) for a in range(2)
                   if pts[i, a] != hard[i, a])
        key = (dist, mask)
        if best is None or key < best[0]:
            best = (key, c)
    total = 1 << n
    costs = [t[0] for t in ranked]
    if best is None:
        q = min(cap, total)
        return yhat, q, 1
    (dist, mask), c = best
    cstar = sum(costs[r] for r in range(n) if (mask >> r) & 1)
    assert dist - int(((xq - hard * ONE) ** 2).sum()) == 4 * ONE * cstar
    below = 0
    for T in range(total):
        cT = sum(costs[r] for r in range(n) if (T >> r) & 1)
        if (cT, T) < (cstar, mask):
            below += 1
    q = below + 1
    if q > cap:
        return yhat, cap, 1
    return c, q, 0


CASES = [(4, 4), (8, 4), (16, 4), (4, 16), (8, 16), (16, 16), (8, 256), (16, 256)]


@pytest.mark.parametrize("N,M", CASES)
def test_decode_matches_brute_force(orc, N, M):
    code = w.polar_code(N, N // 2)
    rng = np.random.default_rng(1000 * N + M)
    mismatches = 0
    for trial in range(25):
        u = rng.integers(0, 2, N // 2, dtype=np.uint8)
        c = code.encode(u)
        ebn0 = rng.uniform(-1, 8)
        s2 = w.noise_variance(M, ebn0)
        rx = w.awgn(w.modulate(c, M).astype(np.float64), s2, rng).reshape(-1)
        rx = np.clip(rx, -(2 ** int(np.log2(M))), 2 ** int(np.log2(M)))  # stay unsaturated
        exp_c, exp_q, exp_ab = brute_decode(code, rx, M, BIG_CAP)
        cw, q, ab = orc.decode(code.h_rows, N, rx, M, s2, BIG_CAP)
        got_c = w.unpack_bits(cw, N)
        assert (q, ab) == (exp_q, exp_ab), (trial, q, ab, exp_q, exp_ab)
        assert np.array_equal(got_c, exp_c)
        # a cap just below the rank abandons with the hard word, at the rank succeeds
        if not exp_ab and exp_q > 1:
            cw2, q2, ab2 = orc.decode(code.h_rows, N, rx, M, s2, exp_q - 1)
            yh, _, _ = brute_decode(code, rx, M, exp_q - 1)
            assert (q2, ab2) == (exp_q - 1, 1)
            assert np.array_equal(w.unpack_bits(cw2, N), yh)
            cw3, q3, ab3 = orc.decode(code.h_rows, N, rx, M, s2, exp_q)
            assert (q3, ab3) == (exp_q, 0)
        mismatches += int(not np.array_equal(got_c, c))
    assert mismatches < 25


def test_qpsk_is_full_ml(orc):
    """For QPSK every codeword is a candidate: the uncapped decode is the ML
    codeword over the whole codebook."""
    code = w.polar_code(16, 8)
    rng = np.random.default_rng(77)
    allc = np.array([code.encode(np.array(u, np.uint8))
                     for u in itertools.product([0, 1], repeat=8)])
    pts = w.modulate(allc, 4).reshape(len(allc), -1)
    for _ in range(60):
        c = allc[rng.integers(0, len(allc))]
        rx = w.awgn(w.modulate(c, 4).astype(np.float64), w.noise_variance(4, 0.0), rng).reshape(-1)
        xq = quantize(rx)
        d = ((xq[None, :] - pts * ONE) ** 2).sum(axis=1)
        cw, q, ab = orc.decode(code.h_rows, 16, rx, 4, 1.0, BIG_CAP)
        assert ab == 0
        got = w.unpack_bits(cw, 16)
        k = [i for i in range(len(allc)) if np.array_equal(allc[i], got)]
        assert len(k) == 1 and d[k[0]] == d.min()


def test_noise_free_decodes_in_one_query(orc):
    for N, M in [(32, 4), (128, 16), (1024, 256), (64, 64)]:
        code = w.polar_code(N, N // 2)
        c = code.encode(np.random.default_rng(N).integers(0, 2, N // 2, dtype=np.uint8))
        rx = w.modulate(c, M).astype(np.float32).reshape(-1)
        cw, q, ab = orc.decode(code.h_rows, N, rx, M, 0.1, 10)
        assert (q, ab) == (1, 0)
        assert np.array_equal(w.unpack_bits(cw, N), c)


def gf2_rref(A):
    A = (np.array(A, dtype=np.uint8) & 1).copy()
    r = 0
    for c in range(A.shape[1]):
        piv = [i for i in range(r, A.shape[0]) if A[i, c]]
        if not piv:
            continue
        A[[r, piv[0]]] = A[[piv[0], r]]
        for i in range(A.shape[0]):
            if i != r and A[i, c]:
                A[i] ^= A[r]
        r += 1
        if r == A.shape[0]:
            break
    return A


def test_basis_and_noise_variance_invariance(orc):
    """Any basis of the null space, and any noise variance, give the same
    decode (H x = 0 iff (T H) x = 0; sigma^2 scales all penalties alike)."""
    jobs = w.jobs_from_spec("inv", seed=5, count=30, cap=4096, Ns=(64,), Ms=(16,),
                            ebn0=("uniform", 3.0, 8.0))
    code = w.polar_code(64, 32)
    H2 = w.pack_bits(gf2_rref(code.h_dense))
    rng = np.random.default_rng(1)
    T = np.eye(32, dtype=np.uint8)
    for _ in range(100):
        i, j = rng.integers(0, 32, 2)
        if i != j:
            T[i] ^= T[j]
    H3 = w.pack_bits((T.astype(np.int64) @ code.h_dense % 2).astype(np.uint8))
    for jb in jobs:
        a = orc.decode(code.h_rows, 64, jb.rx, 16, jb.noise_var, jb.cap)
        b = orc.decode(H2, 64, jb.rx, 16, jb.noise_var, jb.cap)
        c = orc.decode(H3, 64, jb.rx, 16, jb.noise_var * 7.5, jb.cap)
        assert np.array_equal(a[0], b[0]) and a[1:] == b[1:]
        assert np.array_equal(a[0], c[0]) and a[1:] == c[1:]


def test_exhaustion_returns_two_to_the_n(orc):
    """With 16-QAM some hard words have no candidate codeword; the search
    then ends after all 2^n patterns with the abandon flag."""
    code = w.polar_code(4, 2)
    rng = np.random.default_rng(2)
    seen = False
    for _ in range(400):
        rx = rng.uniform(-4, 4, 2).astype(np.float32)
        exp = brute_decode(code, rx, 16, BIG_CAP)
        cw, q, ab = orc.decode(code.h_rows, 4, rx, 16, 1.0, BIG_CAP)
        assert (q, ab) == (exp[1], exp[2])
        if ab:
            assert q == 4
            seen = True
    assert seen


def test_decode_argument_errors(orc):
    code = w.polar_code(32, 16)
    rx = np.zeros(32, np.float32)
    with pytest.raises(ValueError):
        orc.decode(code.h_rows, 32, rx, 4, 1.0, 0)            # cap 0
    with pytest.raises(ValueError):
        orc.decode(code.h_rows, 32, rx, 4, -1.0, 10)          # noise variance
    with pytest.raises(ValueError):
        orc.decode(code.h_rows, 32, rx, 4, float("inf"), 10)
    with pytest.raises(ValueError):
        orc.decode(code.h_rows, 32, rx, 8, 1.0, 10)           # M
    bad = rx.copy()
    bad[3] = np.inf
    with pytest.raises(ValueError):
        orc.decode(code.h_rows, 32, bad, 4, 1.0, 10)
