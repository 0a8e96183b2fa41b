"""Gray square M-QAM modulation and AWGN, used to make decoder inputs.

Definition "M-QAM" (Section II, Eq. 1-2): M = 2^(2m) points whose two
quadrature amplitudes are odd multiples of d, d = sqrt(3 m E_b / (M - 1)).
Received values are handed to the decoder divided by d, i.e. in units of the
odd-integer lattice {+-1, +-3, ...}.

Labelling (the paper's Fig. 1 is not reproduced in the text, so this is the
convention both decoders are written against): each axis carries m bits of
a binary-reflected Gray code, level index 0 being the most negative
amplitude; a symbol's 2m bits are the in-phase label (MSB first) followed by
the quadrature label.  A codeword of N bits fills L = ceil(N / 2m) symbols
(Algorithm 2, input); missing bits of the last symbol are sent as 0.

Noise: E_b is the energy per coded bit of Eq. 2, so in lattice units
E_b = (M - 1) / (3 m) and the per-dimension variance at Eb/N0 (dB) is
sigma^2 = (M - 1) / (6 m 10^(EbN0/10)).
"""
from __future__ import annotations

import math

import numpy as np


def bits_per_axis(M: int) -> int:
    m = int(round(math.log2(M))) // 2
    if M < 4 or (1 << (2 * m)) != M:
        raise ValueError("M must be 4^m, m >= 1")
    return m


def symbols_per_codeword(N: int, M: int) -> int:
    m = bits_per_axis(M)
    return -(-N // (2 * m))


def gray_to_index(g: np.ndarray) -> np.ndarray:
    """Inverse binary-reflected Gray code: index = g ^ g>>1 ^ g>>2 ^ ..."""
    g = np.asarray(g, dtype=np.int64)
    idx = g.copy()
    shift = g >> 1
    while np.any(shift):
        idx ^= shift
        shift >>= 1
    return idx


def modulate(bits: np.ndarray, M: int) -> np.ndarray:
    """Map codeword bits (..., N) to lattice points (..., L, 2) (odd integers)."""
    m = bits_per_axis(M)
    bits = np.asarray(bits, dtype=np.int64)
    N = bits.shape[-1]
    L = symbols_per_codeword(N, M)
    pad = 2 * m * L - N
    if pad:
        bits = np.concatenate([bits, np.zeros(bits.shape[:-1] + (pad,), np.int64)], axis=-1)
    b = bits.reshape(bits.shape[:-1] + (L, 2, m))
    weights = 1 << np.arange(m - 1, -1, -1)          # MSB first
    labels = (b * weights).sum(axis=-1)               # (..., L, 2)
    idx = gray_to_index(labels)
    return 2 * idx - ((1 << m) - 1)


def noise_variance(M: int, ebn0_db: float) -> float:
    m = bits_per_axis(M)
    return (M - 1) / (6.0 * m * 10.0 ** (ebn0_db / 10.0))


def awgn(points: np.ndarray, sigma2: float, rng: np.random.Generator) -> np.ndarray:
    """Add N(0, sigma2) per real dimension; return float32 received values."""
    noise = rng.normal(0.0, math.sqrt(sigma2), size=points.shape)
    return (points + noise).astype(np.float32)
