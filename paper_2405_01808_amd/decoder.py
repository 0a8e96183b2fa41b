"""Python binding of the GRAND decoder: argument marshalling over the C ABI.

Every decoding step runs in the HIP library; torch provides device memory
and streams only.  Conventions are those of include/grand.h.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np

from . import _native as nat


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def received_count(n: int, M: int) -> int:
    """2L: the received floats of one word (L = ceil(n / log2 M) symbols)."""
    m = int(M).bit_length() - 1
    if M < 4 or M != 1 << m or m % 2:
        raise ValueError(f"M must be 4, 16, 64, 256, 1024 or 4096, not {M}")
    return 2 * (-(-int(n) // m))


class Code:
    """Decoder handle for a parity-check matrix H (rows x n, bit-packed rows).

    h_rows: uint64 array of shape (rows, ceil(n/64)); bit j of row i is bit
    j % 64 of h_rows[i, j // 64]."""

    def __init__(self, n: int, h_rows):
        h = np.ascontiguousarray(np.asarray(h_rows, dtype=np.uint64))
        if h.ndim != 2 or h.shape[1] != (n + 63) // 64:
            raise ValueError("h_rows must have shape (rows, ceil(n/64))")
        self._lib = nat.lib()
        handle = ctypes.c_void_p()
        nat.check(self._lib.grand_code_create(n, h.shape[0], _ptr(h), ctypes.byref(handle)))
        self.handle = handle
        self.n = n
        self.rows = h.shape[0]

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            self._lib.grand_code_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def init(device: int = 0):
    nat.check(nat.lib().grand_init(device))


def decode(code: Code, rx, M: int, noise_var: float, cap: int, cutoff: int = 0):
    """One decode with host buffers (synchronous); cutoff > 0 applies
    Algorithm 2's symbol cut-off S (grand_decode_ex).

    Returns (codeword uint64[ceil(n/64)], queries, abandoned)."""
    r = np.ascontiguousarray(np.asarray(rx, dtype=np.float32)).reshape(-1)
    if r.size < received_count(code.n, M):
        raise ValueError(f"rx holds {r.size} values; a word of n={code.n}, M={M} needs "
                         f"{received_count(code.n, M)}")
    cw = np.zeros((code.n + 63) // 64, np.uint64)
    q = ctypes.c_uint64(0)
    ab = ctypes.c_uint8(0)
    nat.check(nat.lib().grand_decode_ex(code.handle, _ptr(r), int(M), float(noise_var), int(cap),
                                        int(cutoff), _ptr(cw), ctypes.byref(q),
                                        ctypes.byref(ab)))
    return cw, q.value, ab.value


def check_batch_shapes(code_ns, code_index, M, cap, noise_var, rx_offset, rx_numel: int):
    """Raise ValueError unless every per-word array has one entry per word,
    every code index names a code, and every word's 2L received values lie
    inside rx (rx_numel floats).  Host-side only: this is what keeps the
    kernel's reads of rx in bounds."""
    count = len(code_index)
    for name, arr in (("M", M), ("cap", cap), ("noise_var", noise_var), ("rx_offset", rx_offset)):
        if np.ndim(arr) != 1 or len(arr) != count:
            raise ValueError(f"{name} has {np.size(arr)} entries; code_index has {count}")
    if not count:
        return
    ci = np.asarray(code_index, np.int64)
    if ci.min() < 0 or ci.max() >= len(code_ns):
        raise ValueError("code_index out of range")
    ns = np.asarray(code_ns, np.int64)[ci]
    need = np.array([received_count(n, m) for n, m in zip(ns, np.asarray(M))], np.int64)
    off = np.asarray(rx_offset, np.uint64)
    if np.any(off > np.uint64(rx_numel)) or np.any(off.astype(np.int64) + need > rx_numel):
        raise ValueError("a word's received values lie past the end of rx")


@dataclass
class BatchResult:
    codewords: "object"   # torch.int64 [count, 16] (uint64 bit patterns)
    queries: "object"     # torch.int64 [count]
    abandoned: "object"   # torch.uint8 [count]
    status: "object"      # torch.int32 [count]
    checks: "object"      # torch.int64 [count]


class BatchPlan:
    """Host metadata and device outputs of a batch, reusable across calls."""

    def __init__(self, codes, code_index, M, cap, noise_var, rx_offset, rx, device=None,
                 cutoff: int = 0, launch_mode: int = 0):
        import torch
        self.codes = list(codes)
        self.count = len(code_index)
        self.code_index = np.ascontiguousarray(code_index, dtype=np.uint32)
        self.M = np.ascontiguousarray(M, dtype=np.uint32)
        self.cap = np.ascontiguousarray(cap, dtype=np.uint64)
        self.noise_var = np.ascontiguousarray(noise_var, dtype=np.float32)
        self.rx_offset = np.ascontiguousarray(rx_offset, dtype=np.uint64)
        if not (isinstance(rx, torch.Tensor) and rx.is_cuda and rx.dtype == torch.float32):
            raise TypeError("rx must be a float32 CUDA (HIP) tensor")
        self.rx = rx.contiguous()
        check_batch_shapes([c.n for c in self.codes], self.code_index, self.M, self.cap,
                           self.noise_var, self.rx_offset, self.rx.numel())
        dev = rx.device if device is None else device
        n = self.count
        self.out = BatchResult(
            codewords=torch.zeros((max(n, 1), nat.CW_STRIDE), dtype=torch.int64, device=dev),
            queries=torch.zeros(max(n, 1), dtype=torch.int64, device=dev),
            abandoned=torch.zeros(max(n, 1), dtype=torch.uint8, device=dev),
            status=torch.zeros(max(n, 1), dtype=torch.int32, device=dev),
            checks=torch.zeros(max(n, 1), dtype=torch.int64, device=dev))
        self._handles = (ctypes.c_void_p * max(len(self.codes), 1))(
            *[c.handle.value for c in self.codes])
        b = nat.GrandBatch()
        b.count = n
        b.n_codes = len(self.codes)
        b.codes = ctypes.cast(self._handles, ctypes.POINTER(ctypes.c_void_p))
        b.code_index = _ptr(self.code_index)
        b.M = _ptr(self.M)
        b.query_cap = _ptr(self.cap)
        b.noise_var = _ptr(self.noise_var)
        b.rx_offset = _ptr(self.rx_offset)
        b.rx = self.rx.data_ptr()
        b.codeword_out = self.out.codewords.data_ptr()
        b.queries_out = self.out.queries.data_ptr()
        b.abandoned_out = self.out.abandoned.data_ptr()
        b.status_out = self.out.status.data_ptr()
        b.checks_out = self.out.checks.data_ptr()
        b.cutoff_symbols = int(cutoff)
        b.launch_mode = int(launch_mode)   # 0 auto, 1 one merged launch, 2 one per (n, M)
        b.rx_count = self.rx.numel()
        self.desc = b

    def launch(self, stream=None):
        """Enqueue the whole batch on `stream` (default: torch's current stream)."""
        import torch
        if stream is None:
            stream = torch.cuda.current_stream(self.rx.device)
        sp = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
        nat.check(nat.lib().grand_decode_batch(ctypes.byref(self.desc), ctypes.c_void_p(sp)))
        return self.out

    def launch_noalloc(self, stream=None):
        """The same decode through grand_decode_batch_noalloc (no device
        allocation; returns once the per-word tables are on the device)."""
        import torch
        if stream is None:
            stream = torch.cuda.current_stream(self.rx.device)
        sp = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
        nat.check(nat.lib().grand_decode_batch_noalloc(ctypes.byref(self.desc),
                                                       ctypes.c_void_p(sp)))
        return self.out


class BatchGraph:
    """A BatchPlan recorded once as a HIP graph (grand_graph_*): each launch
    decodes whatever rx the plan's buffer holds, into the plan's outputs."""

    def __init__(self, plan: BatchPlan):
        self.plan = plan
        h = ctypes.c_void_p()
        nat.check(nat.lib().grand_graph_create(ctypes.byref(plan.desc), ctypes.byref(h)))
        self.handle = h

    def launch(self, stream=None):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream(self.plan.rx.device)
        sp = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
        nat.check(nat.lib().grand_graph_launch(self.handle, ctypes.c_void_p(sp)))
        return self.plan.out

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            nat.lib().grand_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def decode_batch(codes, code_index, M, cap, noise_var, rx_offset, rx, stream=None,
                 cutoff: int = 0) -> BatchResult:
    """Decode many codewords on the GPU (asynchronous on `stream`); cutoff > 0
    applies Algorithm 2's symbol cut-off S to every word."""
    plan = BatchPlan(codes, code_index, M, cap, noise_var, rx_offset, rx, cutoff=cutoff)
    out = plan.launch(stream)
    out._plan = plan   # keep host metadata alive until the caller synchronises
    return out


def get_tuning(n: int, M: int) -> dict:
    t = nat.GrandTuning()
    nat.check(nat.lib().grand_tuning_get(n, M, ctypes.byref(t)))
    return {f: getattr(t, f) for f, _ in nat.GrandTuning._fields_}


def set_tuning(n: int, M: int, **kw):
    cur = get_tuning(n, M)
    cur.update(kw)
    t = nat.GrandTuning(**cur)
    nat.check(nat.lib().grand_tuning_set(n, M, ctypes.byref(t)))


def probe_xor_rate(steps: int = 1 << 14) -> tuple[float, float]:
    """Measured 32-bit XOR lane-operations per second of the current device
    and the timed launch's seconds (grand_probe_xor_rate)."""
    rate, sec = ctypes.c_double(0), ctypes.c_double(0)
    nat.check(nat.lib().grand_probe_xor_rate(int(steps), ctypes.byref(rate), ctypes.byref(sec)))
    return rate.value, sec.value


def probe_dense_pmult(code: Code, words: int, patterns: int, words_dev=None) -> tuple[float, int]:
    """Checks per second of one full Algorithm 1 product per pattern (the
    incremental syndrome's baseline), and the zero syndromes it found
    (grand_probe_dense_pmult).  words_dev: a device tensor of `words` hard
    words (ceil(n/64) int64 each), or None for hash-generated words."""
    rate, zeros = ctypes.c_double(0), ctypes.c_uint64(0)
    wp = None
    if words_dev is not None:
        if words_dev.numel() < words * ((code.n + 63) // 64):
            raise ValueError("words_dev holds fewer than `words` words")
        wp = ctypes.c_void_p(words_dev.data_ptr())
    nat.check(nat.lib().grand_probe_dense_pmult(code.handle, wp, int(words), int(patterns),
                                                ctypes.byref(rate), ctypes.byref(zeros)))
    return rate.value, zeros.value


def pmult(code: Code, x, stream=None):
    """Algorithm 1 on a batch (grand_pmult): x is a device int64 tensor of
    shape (count, ceil(n/64)); returns the syndromes as a device int64 tensor
    of shape (count, ceil(rows/64))."""
    import torch
    w64 = (code.n + 63) // 64
    if x.dim() != 2 or x.shape[1] != w64 or x.dtype != torch.int64 or not x.is_cuda:
        raise ValueError(f"x must be a CUDA int64 tensor of shape (count, {w64})")
    x = x.contiguous()
    out = torch.zeros((x.shape[0], (code.rows + 63) // 64), dtype=torch.int64, device=x.device)
    if stream is None:
        stream = torch.cuda.current_stream(x.device)
    sp = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
    nat.check(nat.lib().grand_pmult(code.handle, ctypes.c_void_p(x.data_ptr()), x.shape[0],
                                    ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(sp)))
    return out
