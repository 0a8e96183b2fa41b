"""Polar code construction used to make decoder inputs.

This module builds the parity-check matrix H that the decoder receives as an
input, and encodes information words into codewords.  It holds no decoding
arithmetic: demapping, test-error-pattern ordering and syndrome checking live
in the oracle and in the HIP library, which both take H as an argument.

Conventions (Definition "Polar codes", Section II):
  * G_N = F^{(x) n} with F = [[1, 0], [1, 1]] and no bit reversal, so
    G_N[i][j] = 1 exactly when the bits of j are a subset of the bits of i.
  * c = u . G_N with the frozen positions of u set to 0.
  * H is (N-K) x N with G_I . H^T = 0.  Row r is column f_r of G_N, f_r being
    the r-th frozen index in ascending order, i.e. H[r][j] = 1 iff
    (j & f_r) == f_r.  Because G_N is its own inverse over GF(2), u = c . G_N,
    so row r states u_{f_r} = 0.
  * The frozen set is the N-K indices with the smallest polarization weight
    PW(i) = sum_j bit_j(i) * 2^(j/4); the paper uses the 3GPP reliability
    sequence (Section III), which is not available here.
"""
from __future__ import annotations

import numpy as np

BETA = 2.0 ** 0.25


def polarization_weight(i: int) -> float:
    """PW(i) = sum over set bits j of i of beta^j, beta = 2^(1/4)."""
    w = 0.0
    j = 0
    while i:
        if i & 1:
            w += BETA ** j
        i >>= 1
        j += 1
    return w


def frozen_set(N: int, K: int) -> list[int]:
    """The N-K least reliable indices by polarization weight, ascending."""
    if N < 2 or N & (N - 1):
        raise ValueError("N must be a power of two >= 2")
    if not 0 < K < N:
        raise ValueError("need 0 < K < N")
    order = sorted(range(N), key=lambda i: (polarization_weight(i), i))
    return sorted(order[: N - K])


def info_set(N: int, frozen: list[int]) -> list[int]:
    fz = set(frozen)
    return [i for i in range(N) if i not in fz]


def words_per_row(N: int) -> int:
    return (N + 63) // 64


def pack_bits(bits: np.ndarray) -> np.ndarray:
    """Pack a 0/1 vector (last axis) into little-endian uint64 words:
    bit j goes to word j // 64, bit j % 64."""
    bits = np.asarray(bits, dtype=np.uint8)
    n = bits.shape[-1]
    nw = (n + 63) // 64
    pad = nw * 64 - n
    if pad:
        bits = np.concatenate([bits, np.zeros(bits.shape[:-1] + (pad,), np.uint8)], axis=-1)
    b = bits.reshape(bits.shape[:-1] + (nw, 64)).astype(np.uint64)
    shifts = np.arange(64, dtype=np.uint64)
    return (b << shifts).sum(axis=-1, dtype=np.uint64)


def unpack_bits(words: np.ndarray, n: int) -> np.ndarray:
    words = np.asarray(words, dtype=np.uint64)
    shifts = np.arange(64, dtype=np.uint64)
    b = ((words[..., :, None] >> shifts) & np.uint64(1)).astype(np.uint8)
    return b.reshape(words.shape[:-1] + (-1,))[..., :n]


def parity_check_dense(N: int, frozen: list[int]) -> np.ndarray:
    """H as a dense (N-K) x N uint8 matrix: H[r][j] = 1 iff (j & f_r) == f_r."""
    j = np.arange(N)
    return np.stack([((j & f) == f).astype(np.uint8) for f in frozen])


def parity_check_rows(N: int, frozen: list[int]) -> np.ndarray:
    """H bit-packed by rows: (N-K) x ceil(N/64) uint64."""
    return pack_bits(parity_check_dense(N, frozen))


def encode(u_info: np.ndarray, N: int, info: list[int]) -> np.ndarray:
    """c = u . G_N over GF(2), u_I = u_info (ascending index order), u_F = 0.

    c_j = XOR of u_i over all i whose bits contain the bits of j, computed with
    the in-place superset-sum butterfly (one stage per bit)."""
    x = np.zeros(u_info.shape[:-1] + (N,), np.uint8)
    x[..., info] = u_info
    s = 1
    while s < N:
        idx = np.arange(N)
        lo = idx[(idx & s) == 0]
        x[..., lo] ^= x[..., lo | s]
        s <<= 1
    return x


def rref_basis(h_dense: np.ndarray) -> np.ndarray:
    """Another basis of the same null space: the reduced row echelon form of
    H over GF(2) (pivot columns from the left), the basis whose density
    Section III's Table II reports.  An input for the decoder like H itself:
    any basis gives the same decodes."""
    A = (np.array(h_dense, dtype=np.uint8) & 1).copy()
    r = 0
    for c in range(A.shape[1]):
        piv = np.nonzero(A[r:, c])[0]
        if piv.size == 0:
            continue
        p = r + int(piv[0])
        if p != r:
            A[[r, p]] = A[[p, r]]
        rows = np.nonzero(A[:, c])[0]
        rows = rows[rows != r]
        A[rows] ^= A[r]
        r += 1
        if r == A.shape[0]:
            break
    return A


class PolarCode:
    """(N, K) polar code with the PW frozen set, plus its packed H."""

    def __init__(self, N: int, K: int):
        self.N = N
        self.K = K
        self.rows = N - K
        self.frozen = frozen_set(N, K)
        self.info = info_set(N, self.frozen)
        self.h_dense = parity_check_dense(N, self.frozen)
        self.h_rows = pack_bits(self.h_dense)

    def encode(self, u_info: np.ndarray) -> np.ndarray:
        return encode(u_info, self.N, self.info)


_CODE_CACHE: dict[tuple[int, int], PolarCode] = {}


def polar_code(N: int, K: int) -> PolarCode:
    key = (N, K)
    if key not in _CODE_CACHE:
        _CODE_CACHE[key] = PolarCode(N, K)
    return _CODE_CACHE[key]
