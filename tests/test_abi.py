"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/grand.h declares, and rejects bad arguments before
touching a device."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "grand.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(grand_[a-z_0-9]+)\s*\(", text)))


def test_header_matches_binding_list():
    from paper_2405_01808_amd import _native as nat
    assert declared_functions() == sorted(nat.EXPORTS)


def test_library_exports_every_declared_symbol():
    from paper_2405_01808_amd import _native as nat
    assert os.path.exists(nat.LIB_PATH), "build libgrand.so first"
    out = subprocess.run(["nm", "-D", "--defined-only", nat.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (grand_\w+)", out))
    missing = [f for f in declared_functions() if f not in exported]
    assert not missing, missing
    L = nat.lib()
    for f in declared_functions():
        assert hasattr(L, f)


def test_strerror_covers_every_code():
    from paper_2405_01808_amd import _native as nat
    L = nat.lib()
    for code in (0, -1, -2, -3, -4, -5, -6):
        s = L.grand_strerror(code).decode()
        assert s and s != "unknown error"
    assert L.grand_strerror(-99).decode() == "unknown error"


def test_code_create_rejects_bad_arguments_on_host():
    from paper_2405_01808_amd import _native as nat
    L = nat.lib()
    h = np.zeros((16, 1), np.uint64)
    out = ctypes.c_void_p()
    for n, rows in [(48, 16), (2048, 16), (1, 0), (32, 0), (32, 32), (1024, 513)]:
        rc = L.grand_code_create(n, rows, h.ctypes.data, ctypes.byref(out))
        assert rc == nat.GRAND_EINVAL, (n, rows)
    assert L.grand_code_create(32, 16, None, ctypes.byref(out)) == nat.GRAND_EINVAL
    hb = np.zeros((16, 1), np.uint64)
    hb[3, 0] = 1 << 40                 # bit beyond n = 32
    assert L.grand_code_create(32, 16, hb.ctypes.data, ctypes.byref(out)) == nat.GRAND_EINVAL
    assert "beyond" in L.grand_last_error().decode()


def test_decode_rejects_null_arguments_on_host():
    from paper_2405_01808_amd import _native as nat
    L = nat.lib()
    rc = L.grand_decode(None, None, 4, 1.0, 10, None, None, None)
    assert rc == nat.GRAND_EINVAL
    b = nat.GrandBatch()
    b.count = 3
    assert L.grand_decode_batch(ctypes.byref(b), None) == nat.GRAND_EINVAL
    assert L.grand_decode_batch(None, None) == nat.GRAND_EINVAL
    b.count = 0
    assert L.grand_decode_batch(ctypes.byref(b), None) == nat.GRAND_OK


def test_tuning_table_roundtrip_and_validation():
    import paper_2405_01808_amd as g
    t = g.get_tuning(128, 16)
    assert t["block"] % 64 == 0 and 0 <= t["low_bits"] <= 13
    g.set_tuning(2, 4096, low_bits=3, block=64, first_band=7)
    assert g.get_tuning(2, 4096)["first_band"] == 7
    with pytest.raises(g.GrandError):
        g.set_tuning(2, 4096, block=100)
    with pytest.raises(g.GrandError):
        g.set_tuning(2, 4096, low_bits=14)
    with pytest.raises(g.GrandError):
        g.set_tuning(2, 4096, first_band=0)
    with pytest.raises(g.GrandError):
        g.set_tuning(2, 4096, node_cap=(1 << 22) + 1)
    with pytest.raises(g.GrandError):              # 2^b above 8 merge outputs per thread
        g.set_tuning(2, 4096, block=64, low_bits=10)
    with pytest.raises(g.GrandError):
        g.set_tuning(2, 4096, block=1088)                 # above 1024 threads
    g.set_tuning(2, 4096, block=512)                      # wide workgroups are valid
    assert g.get_tuning(2, 4096)["block"] == 512


def test_server_configuration_rejected_on_host():
    from paper_2405_01808_amd import _native as nat
    L = nat.lib()
    out = ctypes.c_void_p()
    for cfg in [(0, 1, 1, 0, 1 << 20), (4, 0, 1, 0, 1 << 20), (4, 33, 1, 0, 1 << 20),
                (4, 1, 0, 0, 1 << 20), (4, 1, 1, 0, 0), ((1 << 20) + 1, 1, 1, 0, 1 << 20),
                (4, 1, 1, 2, 1 << 20), (0, 0, 0, 1, 1 << 20), (4, 0, 0, 1, 0),
                (4, 1, 1, 1, 1 << 20)]:   # persistent mode is switched off
        c = nat.GrandServerConfig(*cfg)
        assert L.grand_server_create(ctypes.byref(c), ctypes.byref(out)) == nat.GRAND_EINVAL, cfg
    assert L.grand_server_create(None, ctypes.byref(out)) == nat.GRAND_EINVAL
    assert L.grand_server_submit(None, None, None, 4, 1.0, 1, None) == nat.GRAND_EINVAL
    assert L.grand_server_poll(None, None, 0, None) == nat.GRAND_EINVAL
    assert L.grand_server_cancel(None, 1) == nat.GRAND_EINVAL


def test_request_bytes_reflects_tuned_store():
    import paper_2405_01808_amd as g
    from paper_2405_01808_amd import _native as nat
    assert nat.lib().grand_request_bytes(48, 4) == 0
    assert nat.lib().grand_request_bytes(32, 8) == 0
    b = g.request_bytes(1024, 4)
    t = g.get_tuning(1024, 4)
    assert b > 16 * t["node_cap"]


def test_graph_calls_rejected_on_host():
    from paper_2405_01808_amd import _native as nat
    L = nat.lib()
    out = ctypes.c_void_p()
    assert L.grand_graph_create(None, ctypes.byref(out)) == nat.GRAND_EINVAL
    b = nat.GrandBatch()
    b.count = 0
    assert L.grand_graph_create(ctypes.byref(b), ctypes.byref(out)) == nat.GRAND_EINVAL
    assert L.grand_graph_launch(None, None) == nat.GRAND_EINVAL
    L.grand_graph_destroy(None)   # no-op


def test_xor_rate_probe_rejects_bad_arguments_on_host():
    from paper_2405_01808_amd import _native as nat
    L = nat.lib()
    r = ctypes.c_double()
    assert L.grand_probe_xor_rate(0, ctypes.byref(r), None) == nat.GRAND_EINVAL
    assert L.grand_probe_xor_rate(12, ctypes.byref(r), None) == nat.GRAND_EINVAL   # not a multiple of 8
    assert L.grand_probe_xor_rate(8, None, None) == nat.GRAND_EINVAL
    assert L.grand_probe_xor_rate((1 << 20) + 8, ctypes.byref(r), None) == nat.GRAND_EINVAL


def test_dense_pmult_probe_rejects_bad_arguments_on_host():
    from paper_2405_01808_amd import _native as nat
    L = nat.lib()
    r = ctypes.c_double()
    assert L.grand_probe_dense_pmult(None, None, 1, 1, ctypes.byref(r), None) == nat.GRAND_EINVAL
    assert L.grand_pmult(None, None, 1, None, None) == nat.GRAND_EINVAL
    assert L.grand_pmult(None, None, 0, None, None) == nat.GRAND_EINVAL


def test_batch_shape_checks_on_host():
    """Per-word arrays of the wrong length, a bad code index, and received
    values past the end of rx are rejected before anything reaches the C ABI
    (the kernel reads 2L floats from each word's offset)."""
    from paper_2405_01808_amd.decoder import check_batch_shapes, received_count
    assert received_count(128, 16) == 64
    assert received_count(32, 64) == 12        # 6 symbols, pad bits in the last one
    assert received_count(1024, 4) == 1024
    with pytest.raises(ValueError):
        received_count(128, 8)
    ns = [128, 32]
    ok = dict(code_index=[0, 1], M=[16, 64], cap=[10, 10], noise_var=[1.0, 1.0],
              rx_offset=np.array([0, 64], np.uint64), rx_numel=76)
    check_batch_shapes(ns, **ok)
    with pytest.raises(ValueError):
        check_batch_shapes(ns, **dict(ok, rx_numel=75))         # last word one float short
    with pytest.raises(ValueError):
        check_batch_shapes(ns, **dict(ok, rx_offset=np.array([0, 2**63], np.uint64)))
    with pytest.raises(ValueError):
        check_batch_shapes(ns, **dict(ok, M=[16]))              # short metadata
    with pytest.raises(ValueError):
        check_batch_shapes(ns, **dict(ok, noise_var=[1.0, 1.0, 1.0]))
    with pytest.raises(ValueError):
        check_batch_shapes(ns, **dict(ok, code_index=[0, 2]))
    check_batch_shapes(ns, code_index=[], M=[], cap=[], noise_var=[],
                       rx_offset=np.zeros(0, np.uint64), rx_numel=0)


def test_single_decode_rejects_short_rx_on_host():
    """decode() checks the length of rx before calling grand_decode_ex."""
    import paper_2405_01808_amd as g

    class FakeCode:
        n, handle = 128, None
    with pytest.raises(ValueError):
        g.decode(FakeCode(), np.zeros(63, np.float32), 16, 1.0, 10)


def test_noalloc_entry_rejects_bad_batches_on_host():
    """grand_decode_batch_noalloc rejects a null batch and null arrays, and
    accepts an empty batch, before touching a device."""
    from paper_2405_01808_amd import _native as nat
    L = nat.lib()
    assert L.grand_decode_batch_noalloc(None, None) == nat.GRAND_EINVAL
    b = nat.GrandBatch()
    assert L.grand_decode_batch_noalloc(ctypes.byref(b), None) == nat.GRAND_OK
    b.count = 1
    assert L.grand_decode_batch_noalloc(ctypes.byref(b), None) == nat.GRAND_EINVAL
