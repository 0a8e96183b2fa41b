"""Workload presets: synthetic Polar + Gray M-QAM + AWGN codewords.

Every codeword is a pure function of (seed, index): codeword i of a preset
draws its parameters, information bits and noise from
numpy.random.default_rng([seed, i]).  A prefix or a sample of a workload is
therefore identical to the same codewords inside the full workload.

The paper's own evaluation (Section IV) is a Monte-Carlo simulation of this
same kind (rate 1/2 polar codes, M-QAM, AWGN); no dataset is involved.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .channel import awgn, modulate, noise_variance
from .polar import polar_code


@dataclass
class Job:
    N: int
    K: int          # information bits; H has N - K rows
    M: int
    ebn0_db: float
    noise_var: float
    cap: int
    rx: np.ndarray  # float32, 2L values (a_1, b_1, a_2, b_2, ...) in lattice units
    cw: np.ndarray  # uint8, the transmitted codeword (N bits)
    index: int = 0
    arrival_s: float = 0.0


@dataclass
class Spec:
    name: str
    seed: int
    count: int
    cap: int
    Ns: tuple
    Ms: tuple
    ebn0: tuple          # ("fixed", v) | ("uniform", lo, hi) | ("choice", v1, v2, ...)
    rate: float = 0.5
    arrival_rate: float = 0.0   # requests per second (serving mix), 0 = batch
    notes: str = ""
    extra: dict = field(default_factory=dict)


CONFIGS = {
    # One decode per call, the small case.
    "polar32_qpsk": Spec("polar32_qpsk", seed=0, count=1000, cap=10_000,
                         Ns=(32,), Ms=(4,), ebn0=("fixed", 4.0)),
    # One batch in one persistent launch; the benchmark's workload.
    "polar128_16qam": Spec("polar128_16qam", seed=1, count=8192, cap=1 << 16,
                           Ns=(128,), Ms=(16,), ebn0=("uniform", 3.0, 7.0)),
    # Uneven batch of mixed sizes and modulations.
    "uneven_mix": Spec("uneven_mix", seed=2, count=16384, cap=1 << 18,
                       Ns=(64, 128, 256, 512), Ms=(4, 16, 64), ebn0=("uniform", 2.0, 8.0)),
    # Longest codewords, highest order used here.
    "polar1024_256qam": Spec("polar1024_256qam", seed=3, count=2048, cap=1 << 20,
                             Ns=(1024,), Ms=(256,), ebn0=("choice", 10.0, 12.0, 14.0)),
    # Request stream with Poisson arrivals.
    "serving_mix": Spec("serving_mix", seed=4, count=200_000, cap=1 << 18,
                        Ns=(32, 64, 128, 256, 512, 1024), Ms=(4, 16, 64, 256),
                        ebn0=("uniform", 2.0, 14.0), arrival_rate=2e5),
}


def _draw_ebn0(spec: Spec, rng: np.random.Generator) -> float:
    kind = spec.ebn0[0]
    if kind == "fixed":
        return float(spec.ebn0[1])
    if kind == "uniform":
        return float(rng.uniform(spec.ebn0[1], spec.ebn0[2]))
    if kind == "choice":
        vals = spec.ebn0[1:]
        return float(vals[int(rng.integers(0, len(vals)))])
    raise ValueError(kind)


def make_job(spec: Spec, i: int, cap: int | None = None) -> Job:
    rng = np.random.default_rng([spec.seed, i])
    N = int(spec.Ns[int(rng.integers(0, len(spec.Ns)))]) if len(spec.Ns) > 1 else int(spec.Ns[0])
    M = int(spec.Ms[int(rng.integers(0, len(spec.Ms)))]) if len(spec.Ms) > 1 else int(spec.Ms[0])
    ebn0 = _draw_ebn0(spec, rng)
    K = int(round(N * spec.rate))
    code = polar_code(N, K)
    u = rng.integers(0, 2, size=K, dtype=np.uint8)
    cw = code.encode(u)
    sigma2 = noise_variance(M, ebn0)
    rx = awgn(modulate(cw, M).astype(np.float64), sigma2, rng).reshape(-1)
    return Job(N=N, K=K, M=M, ebn0_db=ebn0, noise_var=sigma2,
               cap=int(spec.cap if cap is None else cap), rx=rx, cw=cw, index=i)


def poisson_arrivals(spec: Spec, count: int) -> np.ndarray:
    """Arrival times (s) of a Poisson stream at spec.arrival_rate."""
    rng = np.random.default_rng([spec.seed, 0x5EED])
    gaps = rng.exponential(1.0 / spec.arrival_rate, size=count)
    return np.cumsum(gaps)


def make_jobs(spec: Spec, indices, cap: int | None = None) -> list[Job]:
    jobs = [make_job(spec, int(i), cap) for i in indices]
    if spec.arrival_rate > 0 and len(jobs):
        t = poisson_arrivals(spec, int(max(indices)) + 1)
        for j in jobs:
            j.arrival_s = float(t[j.index])
    return jobs


def config_jobs(name: str, count: int | None = None, cap: int | None = None,
                start: int = 0) -> list[Job]:
    spec = CONFIGS[name]
    n = spec.count if count is None else count
    return make_jobs(spec, range(start, start + n), cap)


def jobs_from_spec(name: str, seed: int, count: int, cap: int, Ns, Ms, ebn0) -> list[Job]:
    """An ad-hoc workload with the same recipe (used by tests for edge cases)."""
    spec = Spec(name, seed=seed, count=count, cap=cap, Ns=tuple(Ns), Ms=tuple(Ms), ebn0=ebn0)
    return make_jobs(spec, range(count))


def _chunk(args):
    name, start, count, cap = args
    jobs = config_jobs(name, count=count, cap=cap, start=start)
    return jobs


def config_jobs_parallel(name: str, count: int | None = None, cap: int | None = None,
                         start: int = 0, workers: int = 8) -> list[Job]:
    """config_jobs over a process pool: the same Jobs (each word is a pure
    function of its seed and index), generated in chunks."""
    spec = CONFIGS[name]
    n = spec.count if count is None else count
    if workers <= 1 or n < 4096:
        return config_jobs(name, count=n, cap=cap, start=start)
    import concurrent.futures as cf
    import multiprocessing as mp
    step = max(1024, -(-n // (4 * workers)))
    parts = [(name, start + k, min(step, n - k), cap) for k in range(0, n, step)]
    out: list[Job] = []
    # fresh interpreters, not forks: the caller may have initialised a GPU
    with cf.ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
        for jobs in ex.map(_chunk, parts):
            out.extend(jobs)
    return out
