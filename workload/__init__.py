"""Seeded synthetic workloads for GRAND decoding of Gray M-QAM polar codewords.

This package only produces inputs (codes, received symbols, noise variances,
query caps, arrival times).  It is shared by the tests, the benchmark and the
oracle's callers, and holds none of the decoder's arithmetic.
"""
from .polar import (PolarCode, polar_code, pack_bits, unpack_bits, frozen_set,  # noqa: F401
                    rref_basis)
from .channel import (modulate, awgn, noise_variance, bits_per_axis,  # noqa: F401
                      symbols_per_codeword)
from .configs import (Job, make_jobs, CONFIGS, config_jobs, config_jobs_parallel,  # noqa: F401
                      poisson_arrivals, jobs_from_spec)
