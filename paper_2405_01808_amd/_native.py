"""ctypes declarations of the C ABI in include/grand.h."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgrand.so")

GRAND_OK = 0
GRAND_EINVAL = -1
GRAND_ENOMEM = -2
GRAND_EDEVICE = -3
GRAND_EBUSY = -4
GRAND_ECAPACITY = -5
GRAND_ENOTFOUND = -6
GRAND_MAX_N = 1024
GRAND_MAX_CAP = 1 << 40
CW_STRIDE = 16   # uint64 words per codeword in batch outputs
SERVE_LANES = 0
SERVE_PERSISTENT = 1
LAUNCH_AUTO, LAUNCH_MERGED, LAUNCH_BUCKETS = 0, 1, 2

# Every symbol the header declares; tests check that the library exports them.
EXPORTS = [
    "grand_strerror", "grand_last_error", "grand_init",
    "grand_code_create", "grand_code_destroy", "grand_code_n", "grand_code_rows",
    "grand_decode", "grand_decode_ex", "grand_decode_batch", "grand_tuning_get", "grand_tuning_set",
    "grand_request_bytes", "grand_server_create", "grand_server_destroy", "grand_server_submit",
    "grand_server_cancel", "grand_server_poll", "grand_server_stats", "grand_server_run_trace",
    "grand_plain_run_trace", "grand_graph_create", "grand_graph_launch", "grand_graph_destroy",
    "grand_debug_fail_launches", "grand_probe_xor_rate", "grand_probe_dense_pmult",
    "grand_decode_batch_noalloc", "grand_pmult",
]
NOALLOC_MAX_WORDS = 65536
NOALLOC_MAX_CODES = 64


class GrandTuning(ctypes.Structure):
    _fields_ = [("low_bits", ctypes.c_uint32), ("block", ctypes.c_uint32),
                ("first_band", ctypes.c_uint32), ("band_growth", ctypes.c_uint32),
                ("node_cap", ctypes.c_uint32), ("grid_per_cu", ctypes.c_uint32)]


class GrandBatch(ctypes.Structure):
    _fields_ = [("count", ctypes.c_uint32), ("n_codes", ctypes.c_uint32),
                ("codes", ctypes.POINTER(ctypes.c_void_p)),
                ("code_index", ctypes.c_void_p), ("M", ctypes.c_void_p),
                ("query_cap", ctypes.c_void_p), ("noise_var", ctypes.c_void_p),
                ("rx_offset", ctypes.c_void_p), ("rx", ctypes.c_void_p),
                ("codeword_out", ctypes.c_void_p), ("queries_out", ctypes.c_void_p),
                ("abandoned_out", ctypes.c_void_p), ("status_out", ctypes.c_void_p),
                ("checks_out", ctypes.c_void_p),
                ("cutoff_symbols", ctypes.c_uint32), ("launch_mode", ctypes.c_uint32),
                ("rx_count", ctypes.c_uint64)]


class GrandServerConfig(ctypes.Structure):
    _fields_ = [("max_inflight", ctypes.c_uint32), ("lanes", ctypes.c_uint32),
                ("max_batch", ctypes.c_uint32), ("mode", ctypes.c_uint32),
                ("memory_budget", ctypes.c_uint64), ("wide_lanes", ctypes.c_uint32),
                ("pad", ctypes.c_uint32)]


WIDE_ITEMS = 512   # GRAND_WIDE_ITEMS: 2L from which a request goes to the wide lanes


class GrandResult(ctypes.Structure):
    _fields_ = [("request_id", ctypes.c_uint64), ("codeword", ctypes.c_uint64 * 16),
                ("queries", ctypes.c_uint64), ("checks", ctypes.c_uint64),
                ("status", ctypes.c_int32), ("abandoned", ctypes.c_uint8),
                ("pad", ctypes.c_uint8 * 3), ("arrival_s", ctypes.c_double),
                ("submit_s", ctypes.c_double), ("complete_s", ctypes.c_double)]


class GrandTraceReq(ctypes.Structure):
    _fields_ = [("code_index", ctypes.c_uint32), ("M", ctypes.c_uint32),
                ("query_cap", ctypes.c_uint64), ("rx_offset", ctypes.c_uint64),
                ("noise_var", ctypes.c_float), ("pad", ctypes.c_float),
                ("arrival_s", ctypes.c_double)]


class GrandError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{msg} (error {code})")
        self.code = code


_lib = None


def lib():
    """Load libgrand.so; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2405_01808_amd.build "
                           "(or __graft_entry__.build()); there is no CPU fallback")
    L = ctypes.CDLL(LIB_PATH)
    vp, u32, u64, i32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
    L.grand_strerror.argtypes = [i32]
    L.grand_strerror.restype = ctypes.c_char_p
    L.grand_last_error.argtypes = []
    L.grand_last_error.restype = ctypes.c_char_p
    L.grand_init.argtypes = [i32]
    L.grand_init.restype = i32
    L.grand_code_create.argtypes = [u32, u32, vp, ctypes.POINTER(vp)]
    L.grand_code_create.restype = i32
    L.grand_code_destroy.argtypes = [vp]
    L.grand_code_destroy.restype = None
    L.grand_code_n.argtypes = [vp]
    L.grand_code_n.restype = u32
    L.grand_code_rows.argtypes = [vp]
    L.grand_code_rows.restype = u32
    L.grand_decode.argtypes = [vp, vp, u32, ctypes.c_float, u64, vp, vp, vp]
    L.grand_decode.restype = i32
    L.grand_decode_ex.argtypes = [vp, vp, u32, ctypes.c_float, u64, u32, vp, vp, vp]
    L.grand_decode_ex.restype = i32
    L.grand_decode_batch.argtypes = [ctypes.POINTER(GrandBatch), vp]
    L.grand_decode_batch.restype = i32
    L.grand_decode_batch_noalloc.argtypes = [ctypes.POINTER(GrandBatch), vp]
    L.grand_decode_batch_noalloc.restype = i32
    L.grand_graph_create.argtypes = [ctypes.POINTER(GrandBatch), ctypes.POINTER(vp)]
    L.grand_graph_create.restype = i32
    L.grand_graph_launch.argtypes = [vp, vp]
    L.grand_graph_launch.restype = i32
    L.grand_graph_destroy.argtypes = [vp]
    L.grand_graph_destroy.restype = None
    L.grand_debug_fail_launches.argtypes = [u32]
    L.grand_debug_fail_launches.restype = None
    L.grand_probe_xor_rate.argtypes = [u32, ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(ctypes.c_double)]
    L.grand_probe_xor_rate.restype = i32
    L.grand_probe_dense_pmult.argtypes = [vp, vp, u32, u32, ctypes.POINTER(ctypes.c_double),
                                          ctypes.POINTER(ctypes.c_uint64)]
    L.grand_pmult.argtypes = [vp, vp, u32, vp, vp]
    L.grand_pmult.restype = i32
    L.grand_probe_dense_pmult.restype = i32
    L.grand_tuning_get.argtypes = [u32, u32, ctypes.POINTER(GrandTuning)]
    L.grand_tuning_get.restype = i32
    L.grand_tuning_set.argtypes = [u32, u32, ctypes.POINTER(GrandTuning)]
    L.grand_tuning_set.restype = i32
    L.grand_request_bytes.argtypes = [u32, u32]
    L.grand_request_bytes.restype = u64
    L.grand_server_create.argtypes = [ctypes.POINTER(GrandServerConfig), ctypes.POINTER(vp)]
    L.grand_server_create.restype = i32
    L.grand_server_destroy.argtypes = [vp]
    L.grand_server_destroy.restype = None
    L.grand_server_submit.argtypes = [vp, vp, vp, u32, ctypes.c_float, u64,
                                      ctypes.POINTER(u64)]
    L.grand_server_submit.restype = i32
    L.grand_server_cancel.argtypes = [vp, u64]
    L.grand_server_cancel.restype = i32
    L.grand_server_poll.argtypes = [vp, ctypes.POINTER(GrandResult), u32, ctypes.POINTER(u32)]
    L.grand_server_poll.restype = i32
    L.grand_server_stats.argtypes = [vp, ctypes.POINTER(u64), ctypes.POINTER(u64),
                                     ctypes.POINTER(u64)]
    L.grand_server_stats.restype = i32
    L.grand_server_run_trace.argtypes = [vp, ctypes.POINTER(vp), u32,
                                         ctypes.POINTER(GrandTraceReq), u32, vp, u64,
                                         ctypes.POINTER(GrandResult), ctypes.POINTER(ctypes.c_double)]
    L.grand_server_run_trace.restype = i32
    L.grand_plain_run_trace.argtypes = [ctypes.POINTER(vp), u32, ctypes.POINTER(GrandTraceReq),
                                        u32, vp, u64, ctypes.POINTER(GrandResult),
                                        ctypes.POINTER(ctypes.c_double)]
    L.grand_plain_run_trace.restype = i32
    _lib = L
    return L


def check(rc: int):
    if rc != GRAND_OK:
        L = lib()
        raise GrandError(rc, f"{L.grand_strerror(rc).decode()}: {L.grand_last_error().decode()}")
