"""Python binding of the serving API (grand_server_* in include/grand.h):
argument marshalling only; admission, batching, launches and timing run in
the native library."""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np

from . import _native as nat


@dataclass
class Result:
    request_id: int
    codeword: np.ndarray   # uint64[16]
    queries: int
    checks: int
    status: int
    abandoned: int
    arrival_s: float
    submit_s: float
    complete_s: float

    @property
    def latency_s(self) -> float:
        return self.complete_s - self.arrival_s


def _result(r: nat.GrandResult) -> Result:
    return Result(r.request_id, np.array(r.codeword[:], np.uint64), r.queries, r.checks,
                  r.status, r.abandoned, r.arrival_s, r.submit_s, r.complete_s)


def request_bytes(n: int, M: int) -> int:
    return int(nat.lib().grand_request_bytes(n, M))


class Server:
    def __init__(self, max_inflight=4096, lanes=4, max_batch=2048, memory_budget=8 << 30,
                 persistent=False, wide_lanes=0):
        self._lib = nat.lib()
        mode = nat.SERVE_PERSISTENT if persistent else nat.SERVE_LANES
        cfg = nat.GrandServerConfig(max_inflight, lanes, max_batch, mode, memory_budget,
                                    wide_lanes, 0)
        h = ctypes.c_void_p()
        nat.check(self._lib.grand_server_create(ctypes.byref(cfg), ctypes.byref(h)))
        self.handle = h

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            self._lib.grand_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, code, rx, M, noise_var, cap) -> int:
        r = np.ascontiguousarray(np.asarray(rx, np.float32))
        rid = ctypes.c_uint64(0)
        nat.check(self._lib.grand_server_submit(self.handle, code.handle, r.ctypes.data, int(M),
                                                float(noise_var), int(cap), ctypes.byref(rid)))
        return rid.value

    def try_submit(self, code, rx, M, noise_var, cap):
        """Like submit, but returns None when admission is refused."""
        try:
            return self.submit(code, rx, M, noise_var, cap)
        except nat.GrandError as e:
            if e.code == nat.GRAND_EBUSY:
                return None
            raise

    def cancel(self, request_id: int):
        nat.check(self._lib.grand_server_cancel(self.handle, int(request_id)))

    def poll(self, max_out=1024) -> list[Result]:
        buf = (nat.GrandResult * max_out)()
        n = ctypes.c_uint32(0)
        nat.check(self._lib.grand_server_poll(self.handle, buf, max_out, ctypes.byref(n)))
        return [_result(buf[i]) for i in range(n.value)]

    def stats(self) -> dict:
        p, r, m = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
        nat.check(self._lib.grand_server_stats(self.handle, ctypes.byref(p), ctypes.byref(r),
                                               ctypes.byref(m)))
        return {"pending": p.value, "running": r.value, "memory_in_use": m.value}


class Trace:
    """A recorded arrival stream: codes, per-request metadata and rx."""

    def __init__(self, codes, code_index, M, cap, noise_var, rx_list, arrival_s):
        self.codes = list(codes)
        n = len(code_index)
        self.count = n
        self.reqs = (nat.GrandTraceReq * max(n, 1))()
        offs = np.cumsum([0] + [len(r) for r in rx_list[:-1]]) if n else np.zeros(0)
        self.rx = np.ascontiguousarray(np.concatenate(rx_list) if n else np.zeros(1),
                                       dtype=np.float32)
        for i in range(n):
            q = self.reqs[i]
            q.code_index = int(code_index[i])
            q.M = int(M[i])
            q.query_cap = int(cap[i])
            q.rx_offset = int(offs[i])
            q.noise_var = float(noise_var[i])
            q.arrival_s = float(arrival_s[i])
        self._handles = (ctypes.c_void_p * max(len(self.codes), 1))(
            *[c.handle.value for c in self.codes])

    def _collect(self, out):
        return [_result(out[i]) for i in range(self.count)]

    def run_server(self, server: Server):
        out = (nat.GrandResult * max(self.count, 1))()
        wall = ctypes.c_double(0)
        nat.check(nat.lib().grand_server_run_trace(
            server.handle, ctypes.cast(self._handles, ctypes.POINTER(ctypes.c_void_p)),
            len(self.codes), self.reqs, self.count, self.rx.ctypes.data, self.rx.size, out,
            ctypes.byref(wall)))
        return self._collect(out), wall.value

    def run_plain(self):
        out = (nat.GrandResult * max(self.count, 1))()
        wall = ctypes.c_double(0)
        nat.check(nat.lib().grand_plain_run_trace(
            ctypes.cast(self._handles, ctypes.POINTER(ctypes.c_void_p)), len(self.codes),
            self.reqs, self.count, self.rx.ctypes.data, self.rx.size, out, ctypes.byref(wall)))
        return self._collect(out), wall.value
