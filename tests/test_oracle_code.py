"""Pins for the code construction (Definition "Polar codes", Section II) and
for the oracle's Algorithm 1 (Theorem 3.1, Table II)."""
import json
import math
import os

import numpy as np
import pytest

import workload as w
from workload.polar import parity_check_dense

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def kron_power(n):
    F = np.array([[1, 0], [1, 1]], dtype=np.int64)
    G = np.array([[1]], dtype=np.int64)
    for _ in range(n):
        G = np.kron(G, F)
    return G


def gf2_rank(A):
    A = (np.array(A, dtype=np.uint8) & 1).copy()
    r = 0
    rows, cols = A.shape
    for c in range(cols):
        piv = [i for i in range(r, rows) if A[i, c]]
        if not piv:
            continue
        A[[r, piv[0]]] = A[[piv[0], r]]
        for i in range(rows):
            if i != r and A[i, c]:
                A[i] ^= A[r]
        r += 1
        if r == rows:
            break
    return r


def gf2_rref(A):
    """Gauss-Jordan over GF(2), pivot columns taken left to right."""
    A = (np.array(A, dtype=np.uint8) & 1).copy()
    r = 0
    rows, cols = A.shape
    for c in range(cols):
        piv = [i for i in range(r, rows) if A[i, c]]
        if not piv:
            continue
        A[[r, piv[0]]] = A[[piv[0], r]]
        for i in range(rows):
            if i != r and A[i, c]:
                A[i] ^= A[r]
        r += 1
        if r == rows:
            break
    return A[:r]


@pytest.mark.parametrize("n", range(1, 11))
def test_generator_is_kronecker_power_and_involution(n):
    N = 1 << n
    G = kron_power(n)
    i, j = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    assert np.array_equal(G, ((i & j) == j).astype(np.int64))
    if N <= 256:
        assert np.array_equal((G @ G) % 2, np.eye(N, dtype=np.int64))


@pytest.mark.parametrize("N", [4, 8, 16, 32, 64, 128, 256, 512, 1024])
def test_parity_check_annihilates_generator(N):
    K = N // 2
    code = w.polar_code(N, K)
    G = kron_power(int(math.log2(N)))
    GI = G[code.info]
    H = code.h_dense.astype(np.int64)
    assert H.shape == (N - K, N)
    assert not ((GI @ H.T) % 2).any()           # G_I H^T = 0
    if N <= 256:
        assert gf2_rank(H) == N - K             # H spans the whole null space
    # Row for frozen index f has weight 2^(n - wt(f)).
    n = int(math.log2(N))
    for f, row in zip(code.frozen, code.h_dense):
        assert int(row.sum()) == 1 << (n - bin(f).count("1"))


@pytest.mark.parametrize("N", [8, 32, 128, 1024])
def test_encoder_matches_dense_product(N):
    code = w.polar_code(N, N // 2)
    rng = np.random.default_rng(7)
    G = kron_power(int(math.log2(N)))
    for _ in range(4):
        u = rng.integers(0, 2, N // 2, dtype=np.uint8)
        full = np.zeros(N, np.int64)
        full[code.info] = u
        assert np.array_equal(code.encode(u), (full @ G) % 2)
        assert not (code.h_dense.astype(np.int64) @ code.encode(u) % 2).any()


def test_frozen_set_is_least_reliable_by_pw():
    # Independent check of the PW ordering: compare weights as exact
    # elements of Q(2^(1/4)) via high-precision decimals.
    from decimal import Decimal, getcontext
    getcontext().prec = 60
    beta = Decimal(2) ** (Decimal(1) / Decimal(4))
    for N in (16, 32, 64, 128):
        pw = [sum(beta ** j for j in range(11) if (i >> j) & 1) for i in range(N)]
        expect = sorted(sorted(range(N), key=lambda i: pw[i])[: N // 2])
        assert w.frozen_set(N, N // 2) == expect


def test_pmult_equals_dense_product(orc):
    rng = np.random.default_rng(3)
    for N in (8, 32, 128, 512):
        code = w.polar_code(N, N // 2)
        for _ in range(5):
            c = rng.integers(0, 2, N, dtype=np.uint8)
            r, steps, ands, xors = orc.pmult(code.h_dense, c)
            assert np.array_equal(r, (code.h_dense.astype(np.int64) @ c) % 2)
            wts = code.h_dense.sum(axis=1)
            # Theorem 3.1: 1 + max ceil(log2 W_H(i)) steps, W_H ANDs,
            # sum ceil(log2 W_H(i)) XOR levels.
            assert steps == 1 + max(math.ceil(math.log2(x)) for x in wts)
            assert ands == wts.sum()
            assert xors == sum(math.ceil(math.log2(x)) for x in wts)


def test_table2_column_n128_reproduced(orc):
    """Table II at N = 128 (where the PW and 3GPP frozen sets coincide)."""
    g = json.load(open(os.path.join(GOLDEN, "table2_summary.json")))
    col = g["N"].index(128)
    code = w.polar_code(128, 64)
    H = gf2_rref(code.h_dense)
    assert H.shape == (64, 128)
    # Same row space as the frozen-column basis.
    assert gf2_rank(np.vstack([H, code.h_dense])) == 64
    c = np.zeros(128, np.uint8)
    _, steps, ands, xors = orc.pmult(H, c)
    assert ands == g["and_gates_WH"][col]
    assert round(100.0 * ands / (64 * 128), 2) == g["sparsity_pct"][col]
    assert int(H.sum(axis=1).max()) == g["max_row_weight"][col]
    assert xors == g["xor_gates"][col]
    assert steps == g["pmult_cycles"][col]
    # Observation after Fig. 3: the first row is the heaviest.
    assert int(H[0].sum()) == int(H.sum(axis=1).max())


def test_table2_internal_consistency():
    """Table II's rows follow from each other as Theorem 3.1 says."""
    g = json.load(open(os.path.join(GOLDEN, "table2_summary.json")))
    for N, wh, sp, mx, cyc in zip(g["N"], g["and_gates_WH"], g["sparsity_pct"],
                                  g["max_row_weight"], g["pmult_cycles"]):
        assert round(100.0 * wh / ((N // 2) * N), 2) == sp
        assert 1 + math.ceil(math.log2(mx)) == cyc


def test_plausibility_arithmetic():
    g = json.load(open(os.path.join(GOLDEN, "plausibility_n7.json")))
    assert 4 ** g["S"] == g["instances"]
    assert round(g["and_per_instance"] * g["instances"] / 1e6, 1) == g["and_total_millions"]
    assert round(g["xor_per_instance"] * g["instances"] / 1e6, 1) == g["xor_total_millions"]


def test_packing_roundtrip():
    rng = np.random.default_rng(0)
    for n in (2, 63, 64, 65, 1024):
        b = rng.integers(0, 2, n, dtype=np.uint8)
        assert np.array_equal(w.unpack_bits(w.pack_bits(b), n), b)
