"""MI355X (gfx950) GRAND decoder for Gray M-QAM modulated polar codewords
(arXiv 2405.01808).  The decoding path is the HIP library libgrand.so; this
package only marshals arguments to its C ABI (include/grand.h)."""
from .decoder import (Code, BatchGraph, BatchPlan, BatchResult, decode, decode_batch,  # noqa: F401
                      get_tuning, init, pmult, probe_dense_pmult, probe_xor_rate,
                      set_tuning)
from ._native import GrandError, CW_STRIDE, GRAND_MAX_CAP  # noqa: F401
from .server import Server, Trace, Result, request_bytes  # noqa: F401
from .autotune import autotune, autotune_batch  # noqa: F401,E402
