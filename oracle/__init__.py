"""ctypes binding of the plain C oracle (grand_oracle.c).

TEST INFRASTRUCTURE: imported only by tests/, by __graft_entry__.smoke() and
by bench.py's CPU-baseline leg.  The product package never imports it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import time

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "grand_oracle.c")
_LIB = os.path.join(_HERE, "libgrand_oracle.so")

ORC_OK, ORC_EINVAL, ORC_ENOMEM = 0, -1, -2


def build(force: bool = True) -> str:
    """Compile the oracle with gcc -O2 (no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fPIC", "-shared",
                               "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm", "-lpthread"])
        os.replace(tmp, _LIB)
    return _LIB


class OrcJob(ctypes.Structure):
    _fields_ = [("N", ctypes.c_uint32), ("rows", ctypes.c_uint32), ("M", ctypes.c_uint32),
                ("cutoff", ctypes.c_uint32),
                ("h_rows", ctypes.c_void_p), ("rx", ctypes.c_void_p),
                ("noise_var", ctypes.c_double), ("cap", ctypes.c_uint64),
                ("codeword_out", ctypes.c_void_p), ("q_out", ctypes.c_void_p),
                ("abandoned_out", ctypes.c_void_p),
                ("status", ctypes.c_int32), ("pad1", ctypes.c_int32),
                ("seconds", ctypes.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = ctypes.CDLL(_LIB)
        vp, u32, u64 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64
        L.orc_demap.argtypes = [u32, u32, vp, vp, vp, vp, vp]
        L.orc_demap.restype = ctypes.c_int
        L.orc_pmult.argtypes = [u32, u32, vp, vp, vp, vp, vp, vp]
        L.orc_pmult.restype = ctypes.c_int
        L.orc_enumerate.argtypes = [u32, vp, u64, vp, vp]
        L.orc_enumerate.restype = ctypes.c_int64
        L.orc_decode.argtypes = [u32, u32, vp, vp, u32, ctypes.c_double, u64, vp, vp, vp]
        L.orc_decode.restype = ctypes.c_int
        L.orc_decode_ex.argtypes = [u32, u32, vp, vp, u32, ctypes.c_double, u64, u32, vp, vp, vp]
        L.orc_decode_ex.restype = ctypes.c_int
        L.orc_select_symbols.argtypes = [u32, u32, vp, u32, vp, vp]
        L.orc_select_symbols.restype = ctypes.c_int
        L.orc_decode_many.argtypes = [ctypes.POINTER(OrcJob), u32, u32]
        L.orc_decode_many.restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def demap(N: int, M: int, rx: np.ndarray):
    """Returns (yhat bits uint8[N], item costs, item positions) in natural order."""
    rx = np.ascontiguousarray(rx, dtype=np.float32)
    yhat = np.zeros(N, np.uint8)
    cap = rx.size
    cost = np.zeros(cap, np.uint32)
    pos = np.zeros(cap, np.uint32)
    n = ctypes.c_uint32(0)
    rc = lib().orc_demap(N, M, _ptr(rx), _ptr(yhat), _ptr(cost), _ptr(pos), ctypes.byref(n))
    if rc != ORC_OK:
        raise ValueError(f"orc_demap failed: {rc}")
    return yhat, cost[: n.value].copy(), pos[: n.value].copy()


def pmult(H: np.ndarray, c: np.ndarray):
    """Algorithm 1 on dense 0/1 arrays: returns (r, steps, and_gates, xor_gates)."""
    H = np.ascontiguousarray(H, dtype=np.uint8)
    c = np.ascontiguousarray(c, dtype=np.uint8)
    K, N = H.shape
    r = np.zeros(K, np.uint8)
    steps = ctypes.c_uint32(0)
    ands = ctypes.c_uint64(0)
    xors = ctypes.c_uint64(0)
    rc = lib().orc_pmult(K, N, _ptr(H), _ptr(c), _ptr(r), ctypes.byref(steps),
                         ctypes.byref(ands), ctypes.byref(xors))
    if rc != ORC_OK:
        raise ValueError(f"orc_pmult failed: {rc}")
    return r, steps.value, ands.value, xors.value


def enumerate_teps(cost_sorted, count: int):
    """First `count` patterns: (masks uint64[count, ceil(n/64)], costs uint64[count])."""
    cs = np.ascontiguousarray(cost_sorted, dtype=np.uint32)
    n = cs.size
    words = (n + 63) // 64
    masks = np.zeros((count, words), np.uint64)
    costs = np.zeros(count, np.uint64)
    got = lib().orc_enumerate(n, _ptr(cs), count, _ptr(masks), _ptr(costs))
    if got < 0:
        raise ValueError(f"orc_enumerate failed: {got}")
    return masks[:got], costs[:got]


def decode(h_rows: np.ndarray, N: int, rx: np.ndarray, M: int, noise_var: float, cap: int):
    """Returns (codeword words uint64[ceil(N/64)], q, abandoned)."""
    h = np.ascontiguousarray(h_rows, dtype=np.uint64)
    rx = np.ascontiguousarray(rx, dtype=np.float32)
    cw = np.zeros((N + 63) // 64, np.uint64)
    q = ctypes.c_uint64(0)
    ab = ctypes.c_uint8(0)
    rc = lib().orc_decode(N, h.shape[0], _ptr(h), _ptr(rx), M, float(noise_var), int(cap),
                          _ptr(cw), ctypes.byref(q), ctypes.byref(ab))
    if rc != ORC_OK:
        raise ValueError(f"orc_decode failed: {rc}")
    return cw, q.value, ab.value


def select_symbols(N: int, M: int, rx: np.ndarray, S: int):
    """Algorithm 2 Steps 1-3: bool[L], True for the min(S, L) least reliable
    symbols (smallest d1^2 + d2^2, ties by index)."""
    rx = np.ascontiguousarray(rx, dtype=np.float32)
    m = {4: 1, 16: 2, 64: 3, 256: 4, 1024: 5, 4096: 6}.get(M, 0)
    L = (N + 2 * m - 1) // (2 * m) if m else 1
    sel = np.zeros(L, np.uint8)
    n = ctypes.c_uint32(0)
    rc = lib().orc_select_symbols(N, M, _ptr(rx), int(S), _ptr(sel), ctypes.byref(n))
    if rc != ORC_OK:
        raise ValueError(f"orc_select_symbols failed: {rc}")
    return sel.astype(bool)


def decode_ex(h_rows: np.ndarray, N: int, rx: np.ndarray, M: int, noise_var: float, cap: int,
              cutoff: int):
    """orc_decode_ex: decode with Algorithm 2's symbol cut-off (0 = none)."""
    h = np.ascontiguousarray(h_rows, dtype=np.uint64)
    rx = np.ascontiguousarray(rx, dtype=np.float32)
    cw = np.zeros((N + 63) // 64, np.uint64)
    q = ctypes.c_uint64(0)
    ab = ctypes.c_uint8(0)
    rc = lib().orc_decode_ex(N, h.shape[0], _ptr(h), _ptr(rx), M, float(noise_var), int(cap),
                             int(cutoff), _ptr(cw), ctypes.byref(q), ctypes.byref(ab))
    if rc != ORC_OK:
        raise ValueError(f"orc_decode_ex failed: {rc}")
    return cw, q.value, ab.value


def decode_jobs(jobs, h_rows_of, nthreads: int | None = None, cap: int | None = None,
                cutoff: int = 0):
    """Decode a list of workload Jobs on a thread pool.

    h_rows_of(N, K) -> packed H rows.  Returns (codewords list, q array,
    abandoned array, per-decode seconds, threads used, wall seconds)."""
    n = len(jobs)
    arr = (OrcJob * n)()
    keep = []
    outs_cw, outs_q, outs_ab = [], np.zeros(n, np.uint64), np.zeros(n, np.uint8)
    for i, j in enumerate(jobs):
        h = np.ascontiguousarray(h_rows_of(j.N, j.K), dtype=np.uint64)
        rx = np.ascontiguousarray(j.rx, dtype=np.float32)
        cw = np.zeros((j.N + 63) // 64, np.uint64)
        keep += [h, rx, cw]
        outs_cw.append(cw)
        a = arr[i]
        a.N, a.rows, a.M = j.N, h.shape[0], j.M
        a.h_rows, a.rx = h.ctypes.data, rx.ctypes.data
        a.noise_var = float(j.noise_var)
        a.cap = int(j.cap if cap is None else cap)
        a.cutoff = int(cutoff)
        a.codeword_out = cw.ctypes.data
        a.q_out = outs_q.ctypes.data + 8 * i
        a.abandoned_out = outs_ab.ctypes.data + i
    nt = nthreads if nthreads else (os.cpu_count() or 1)
    t0 = time.perf_counter()
    used = lib().orc_decode_many(arr, n, nt)
    wall = time.perf_counter() - t0
    for i in range(n):
        if arr[i].status != ORC_OK:
            raise ValueError(f"oracle decode {i} failed: {arr[i].status}")
    secs = np.array([arr[i].seconds for i in range(n)])
    return outs_cw, outs_q, outs_ab, secs, used, wall
