"""Benchmark: GRAND decoding of Polar N=128 K=64, Gray 16-QAM, AWGN Eb/N0 ~
U[3, 7] dB, 8192 codewords in one persistent launch, query cap 2^16.

One step = one full decode of the batch (demap, ranking, Algorithm 1
syndrome, ordered pattern checks, early exit or abandonment for every
codeword).  Inputs are resident in device memory before timing starts.

Prints one JSON line.  `value` is useful TEP syndrome checks per second: the
sum over codewords of the query count q (the 1-based rank of the accepted
pattern, or the cap on abandonment), divided by the timed wall time.

Beside the headline the line carries the other workloads (the small per-call
case, the uneven batch merged and per (N, M) bucket, the long-codeword batch,
single-codeword latency, the served request stream against one decode per
request), the per-pattern pMult baseline on the same received words, the
sparsest basis of H, Algorithm 2's symbol cut-off, and the oracle timed on
the host cores with a parity check of its samples against the GPU results.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

WORKLOAD = "polar128_16qam"
WORKLOAD_DESC = ("Polar N=128 K=64 (PW frozen set), Gray 16-QAM, AWGN Eb/N0 uniform in [3,7] dB, "
                 "8192 codewords per step in one persistent launch, query cap 2^16")
# 32-bit integer lane-ops/s: 256 CU x 128 lanes/clk x 2.4 GHz.  The fp32 vector
# peak (157.3 TFLOP/s) is 2 flops x the same 128 lanes/clk/CU, and bitwise VALU
# ops issue at that per-lane rate: the XOR probe measures ~5.8e13/s, well above
# a 64-lane/clk figure.
ALU_PEAK = 256 * 128 * 2.4e9
STEP_WEIGHTS = os.path.join(ROOT, "tests", "golden", "step_weights_polar128_16qam.json")
STEP_WEIGHTS_UNEVEN = os.path.join(ROOT, "tests", "golden", "step_weights_uneven_mix.json")
SERVE_LANES = 14                     # server streams, each on its own hardware queue
SERVE_WIDE = 4                       # of which serve only long words (2L >= 512)
SERVE_BATCH = 256                    # requests per server launch at most
HW_QUEUES = "16"                     # HIP hardware queues for this process (HIP's default is 4)
COPY_BYTES = 256 << 20               # bytes read (and written) by one calibration copy
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "grand_decode_kernel_polar128_16qam_traffic.md")
# oracle samples (bounded CPU work) and parity samples per workload
CPU_SAMPLES = {"polar32_qpsk": 1000, "uneven_mix": 256, "polar1024_256qam": 8,
               "serving_mix": 500}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def measured_traffic():
    """HBM bytes per launch of the decode kernel from the committed counter
    runs, or None when the kernel's sources or build flags have changed since
    they were taken."""
    import re
    try:
        text = open(TRAFFIC_FILE).read()
        rec = json.loads(re.search(r"```json\n(.*?)\n```", text, re.S).group(1))
        from paper_2405_01808_amd.build import kernel_source_sha256
        src = kernel_source_sha256()
    except (OSError, AttributeError, ValueError):
        return None
    if rec.get("kernel_source_sha256") != src:
        return None
    return float(rec["hbm_bytes_per_launch"])



def workers() -> int:
    return max(1, min(16, len(os.sched_getaffinity(0))))


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def device_batch(g, jobs, codes=None, launch_mode=0, cap=None, cutoff=0):
    """A BatchPlan over jobs (rx copied to the device), and its code list."""
    import torch
    import workload as w
    codes = {} if codes is None else codes
    order = []
    idx = []
    for j in jobs:
        if (j.N, j.K) not in codes:
            codes[(j.N, j.K)] = g.Code(j.N, w.polar_code(j.N, j.K).h_rows)
        c = codes[(j.N, j.K)]
        if c not in order:
            order.append(c)
        idx.append(order.index(c))
    lens = np.array([len(j.rx) for j in jobs])
    offs = np.concatenate([[0], np.cumsum(lens)[:-1]]).astype(np.uint64)
    rx = torch.from_numpy(np.concatenate([j.rx for j in jobs])).cuda()
    caps = [j.cap if cap is None else cap for j in jobs]
    plan = g.BatchPlan(order, np.array(idx, np.uint32), [j.M for j in jobs], caps,
                       [j.noise_var for j in jobs], offs, rx, cutoff=cutoff,
                       launch_mode=launch_mode)
    return plan, order


def host_outputs(plan, n):
    o = plan.out
    return (o.codewords.cpu().numpy().view(np.uint64)[:n].copy(),
            o.queries.cpu().numpy().view(np.uint64)[:n].copy(),
            o.abandoned.cpu().numpy()[:n].copy(), o.status.cpu().numpy()[:n].copy())


def time_launches(launch, reps, stream):
    """Mean ms of `reps` launches, each bracketed by events on `stream`."""
    import torch
    launch(stream)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(reps)]
    for a, b in ev:
        a.record(stream)
        launch(stream)
        b.record(stream)
    torch.cuda.synchronize()
    return float(np.mean([a.elapsed_time(b) for a, b in ev]))


def serving(g, w, jobs, plain_count: int):
    """Poisson replay of the serving mix (2e5 requests/s) through the server,
    with and without lanes for long words, and a window of the same stream
    through one grand_decode per request."""
    codes, order, idx = {}, [], []
    for j in jobs:
        if (j.N, j.K) not in codes:
            codes[(j.N, j.K)] = len(order)
            order.append(g.Code(j.N, w.polar_code(j.N, j.K).h_rows))
        idx.append(codes[(j.N, j.K)])
    arrivals = np.array([j.arrival_s for j in jobs]) - jobs[0].arrival_s
    Ms = [j.M for j in jobs]
    caps = [j.cap for j in jobs]
    nvs = [j.noise_var for j in jobs]
    trace = g.Trace(order, idx, Ms, caps, nvs, [j.rx for j in jobs], arrivals)
    nw = min(2000, len(jobs))
    warm = g.Trace(order, idx[:nw], Ms[:nw], caps[:nw], nvs[:nw], [j.rx for j in jobs[:nw]],
                   arrivals[:nw])

    def replay(lanes, wide):
        srv = g.Server(max_inflight=16384, lanes=lanes, max_batch=SERVE_BATCH,
                       memory_budget=48 << 30, wide_lanes=wide)
        warm.run_server(srv)          # first launches, code objects, page mappings
        res, wall = trace.run_server(srv)
        srv.close()
        assert all(r.status == 0 for r in res), "server request errors"
        lat = np.array([r.latency_s for r in res]) * 1e3
        groups = {}
        for j, l in zip(jobs, lat):
            groups.setdefault((j.N, j.M), []).append(l)
        per = {f"{N},{M}": {"requests": len(v), "p50_ms": float(np.percentile(v, 50)),
                            "p99_ms": float(np.percentile(v, 99))}
               for (N, M), v in sorted(groups.items())}
        worst = max(per.items(), key=lambda kv: kv[1]["p99_ms"])
        q = np.array([r.queries for r in res], dtype=np.float64)
        return res, {"lanes": lanes, "wide_lanes": wide, "max_batch": SERVE_BATCH,
                     "requests": len(jobs), "arrival_rate": 2e5, "wall_s": wall,
                     "p50_ms": float(np.percentile(lat, 50)),
                     "p99_ms": float(np.percentile(lat, 99)), "max_ms": float(lat.max()),
                     "worst_group_p99": {"group": worst[0], "p99_ms": worst[1]["p99_ms"]},
                     "codewords_per_s": len(jobs) / wall, "checks_per_s": float(q.sum()) / wall,
                     "abandon_rate": float(np.mean([r.abandoned for r in res])),
                     "per_group": per}

    res, out = replay(SERVE_LANES, SERVE_WIDE)
    log(f"served {len(jobs)} requests: p50 {out['p50_ms']:.3f} ms p99 {out['p99_ms']:.3f} ms, "
        f"worst group {out['worst_group_p99']}")
    nres, narrow = replay(SERVE_LANES, 0)
    out["without_wide_lanes"] = {k: narrow[k] for k in ("lanes", "p50_ms", "p99_ms", "max_ms",
                                                        "worst_group_p99", "codewords_per_s")}
    out["identical_with_and_without_wide_lanes"] = bool(all(
        a.queries == b.queries and a.abandoned == b.abandoned and
        np.array_equal(a.codeword, b.codeword) for a, b in zip(res, nres)))
    out["hw_queues"] = int(os.environ.get("GPU_MAX_HW_QUEUES", "0"))
    if plain_count:
        sub = jobs[:plain_count]
        ptrace = g.Trace(order, idx[:plain_count], Ms[:plain_count], caps[:plain_count],
                         nvs[:plain_count], [j.rx for j in sub], arrivals[:plain_count])
        pres, pwall = ptrace.run_plain()
        plat = np.array([r.latency_s for r in pres]) * 1e3
        pq = np.array([r.queries for r in pres], dtype=np.float64)
        out["plain"] = {"requests": plain_count,
                        "window": f"the first {plain_count} requests of the same stream",
                        "wall_s": pwall,
                        "p50_ms": float(np.percentile(plat, 50)),
                        "p99_ms": float(np.percentile(plat, 99)),
                        "codewords_per_s": plain_count / pwall,
                        "checks_per_s": float(pq.sum()) / pwall,
                        "identical_results": bool(all(
                            r.queries == p.queries and r.abandoned == p.abandoned and
                            np.array_equal(r.codeword[:(j.N + 63) // 64],
                                           p.codeword[:(j.N + 63) // 64])
                            for r, p, j in zip(res, pres, sub)))}
    return out, res


def latency(g, w, reps: int):
    """One N=1024 256-QAM codeword (cap 2^20) per call, `reps` different
    codewords: host-to-host grand_decode, and the device launch alone."""
    import torch
    jobs = w.config_jobs("polar1024_256qam", count=reps)
    code = g.Code(1024, w.polar_code(1024, 512).h_rows)
    host_ms, dev_ms, qs, abs_ = [], [], [], []
    for j in jobs:
        t0 = time.perf_counter()
        _, q, ab = g.decode(code, j.rx, j.M, j.noise_var, j.cap)
        host_ms.append((time.perf_counter() - t0) * 1e3)
        qs.append(q)
        abs_.append(ab)
    stream = torch.cuda.current_stream()
    for j in jobs:
        rx = torch.from_numpy(j.rx).cuda()
        plan = g.BatchPlan([code], np.zeros(1, np.uint32), [j.M], [j.cap], [j.noise_var],
                           np.zeros(1, np.uint64), rx)
        plan.launch(stream)          # first use of this plan's buffers
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        plan.launch(stream)
        b.record(stream)
        torch.cuda.synchronize()
        dev_ms.append(a.elapsed_time(b))
    return {"workload": "polar1024_256qam: N=1024 K=512, 256-QAM, Eb/N0 in {10,12,14} dB, "
                        "cap 2^20, one codeword per call", "reps": reps,
            "host_p50_ms": float(np.percentile(host_ms, 50)),
            "host_p99_ms": float(np.percentile(host_ms, 99)),
            "device_p50_ms": float(np.percentile(dev_ms, 50)),
            "device_p99_ms": float(np.percentile(dev_ms, 99)),
            "mean_q": float(np.mean(qs)), "abandon_rate": float(np.mean(abs_))}


def cutoff_mode(g, w, jobs, code, rx, offs, S: int, reps: int = 5):
    """Algorithm 2 with its symbol cut-off S (Section IV uses S = 8) on the
    same batch: throughput of the batched launch, and the device time of one
    codeword alone beside Proposition 3.1's 2n + 2S + 4 cycle bound (which
    assumes 4^S parallel pMult circuits)."""
    import torch
    stream = torch.cuda.current_stream()
    plan = g.BatchPlan([code], np.zeros(len(jobs), np.uint32), [j.M for j in jobs],
                       [j.cap for j in jobs], [j.noise_var for j in jobs], offs, rx, cutoff=S)
    plan.launch(stream)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(reps)]
    for a, b in ev:
        a.record(stream)
        out = plan.launch(stream)
        b.record(stream)
    torch.cuda.synchronize()
    ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    q = out.queries.cpu().numpy().view(np.uint64).astype(np.float64)
    ab = out.abandoned.cpu().numpy()
    chk = out.checks.cpu().numpy().view(np.uint64).astype(np.float64)
    single = []
    L2 = len(jobs[0].rx)
    for i in range(min(50, len(jobs))):
        one = g.BatchPlan([code], np.zeros(1, np.uint32), [jobs[i].M], [jobs[i].cap],
                          [jobs[i].noise_var], np.zeros(1, np.uint64),
                          rx[i * L2:(i + 1) * L2].contiguous(), cutoff=S)
        one.launch(stream)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        one.launch(stream)
        b.record(stream)
        torch.cuda.synchronize()
        single.append(a.elapsed_time(b))
    n = int(np.log2(jobs[0].N))
    p50 = float(np.percentile(single, 50))
    return {"S": S, "ms_per_launch": ms, "codewords_per_s": len(jobs) / (ms / 1e3),
            "useful_checks_per_s": q.sum() / (ms / 1e3),
            "performed_checks_per_s": chk.sum() / (ms / 1e3), "mean_q": float(q.mean()),
            "abandon_rate": float(ab.mean()), "single_codeword_device_p50_us": p50 * 1e3,
            "single_codeword_cycles_p50_at_2.4GHz": p50 * 1e-3 * 2.4e9,
            "paper_cycle_bound_2n_2S_4": 2 * n + 2 * S + 4}


def long_batch(g, w, jobs, reps: int = 3):
    """The long-codeword batch: 2048 N=1024 256-QAM codewords (Eb/N0 in
    {10, 12, 14} dB, cap 2^20) in one launch."""
    import torch
    plan, _ = device_batch(g, jobs)
    ms = time_launches(plan.launch, reps, torch.cuda.current_stream())
    out = host_outputs(plan, len(jobs))
    q = out[1].astype(np.float64)
    chk = plan.out.checks.cpu().numpy().view(np.uint64)[:len(jobs)].astype(np.float64)
    return {"workload": "polar1024_256qam: 2048 words, N=1024 K=512, 256-QAM, Eb/N0 in "
                        "{10,12,14} dB, cap 2^20, one launch", "ms_per_launch": ms,
            "useful_checks_per_s": q.sum() / (ms / 1e3),
            "performed_checks_per_s": chk.sum() / (ms / 1e3),
            "codewords_per_s": len(jobs) / (ms / 1e3), "mean_q": float(q.mean()),
            "abandon_rate": float(out[2].mean())}, out


def plain_small(g, w, jobs):
    """The small case: 1000 N=32 QPSK codewords (4 dB, cap 10^4), one
    grand_decode call per codeword (host buffers in and out)."""
    code = g.Code(32, w.polar_code(32, 16).h_rows)
    g.decode(code, jobs[0].rx, jobs[0].M, jobs[0].noise_var, jobs[0].cap)   # warm
    us, qs, cws, abs_ = [], [], [], []
    t0 = time.perf_counter()
    for j in jobs:
        t = time.perf_counter()
        cw, q, ab = g.decode(code, j.rx, j.M, j.noise_var, j.cap)
        us.append((time.perf_counter() - t) * 1e6)
        qs.append(q)
        cws.append(cw)
        abs_.append(ab)
    wall = time.perf_counter() - t0
    return ({"workload": "polar32_qpsk: N=32 K=16, QPSK, 4 dB, cap 10^4, one grand_decode per "
                         "codeword", "codewords": len(jobs), "calls_per_s": len(jobs) / wall,
             "useful_checks_per_s": float(np.sum(qs)) / wall, "mean_q": float(np.mean(qs)),
             "p50_us": float(np.percentile(us, 50)), "p99_us": float(np.percentile(us, 99))},
            (np.array(cws), np.array(qs, np.uint64), np.array(abs_, np.uint8),
             np.zeros(len(jobs), np.int32)))


def uneven_roofline(jobs, q, ms):
    """Algorithmic lane-ops of the uneven batch ((mean w + 1) x ceil(rows/32)
    per useful check, mean w per (N, M) bucket from the oracle) per ms."""
    sw = json.load(open(STEP_WEIGHTS_UNEVEN))["buckets"]
    ops = sum(float(qi) * sw[f"{j.N},{j.M}"]["lane_ops_per_query"] for j, qi in zip(jobs, q))
    achieved = ops / (ms / 1e3)
    return {"bound": "alu", "achieved": achieved, "peak": ALU_PEAK, "unit": "int32 lane-ops/s",
            "frac": achieved / ALU_PEAK,
            "work": "(mean w + 1) x ceil(N/2/32) lane-ops per useful check, mean w per (N, M) "
                    "bucket (tests/golden/step_weights_uneven_mix.json)"}


def uneven_batch(g, w, jobs, reps: int = 5, tune: bool = True):
    """The uneven batch (16384 words, N in {64..512}, M in {4, 16, 64}, cap
    2^18): the merged launch with the wildcard tuning autotuned on the whole
    batch (eager and as a replayed HIP graph), against one launch per (N, M)
    bucket with each bucket's tuning autotuned on its own words."""
    import torch
    stream = torch.cuda.current_stream()
    codes = {}
    plan, order = device_batch(g, jobs, codes)
    before = g.get_tuning(0, 0)
    bucket_keys = sorted({(j.N, j.M) for j in jobs})
    saved = {k: g.get_tuning(*k) for k in bucket_keys}
    tuned = None
    buckets = {}
    try:
        if tune:   # on the whole batch: the best launch shape depends on the word count
            tuned = g.autotune_batch(plan.codes, plan.code_index, plan.M, plan.cap,
                                     plan.noise_var, plan.rx_offset, plan.rx, reps=2)
        graph = g.BatchGraph(plan)
        eager_ms = time_launches(plan.launch, reps, stream)
        r_eager = host_outputs(plan, len(jobs))
        graph_ms = time_launches(graph.launch, reps, stream)
        r_graph = host_outputs(plan, len(jobs))
        graph.close()
        # one launch per (N, M) bucket, each bucket tuned on its own words
        if tune:
            for (N, M) in bucket_keys:
                sel = [j for j in jobs if (j.N, j.M) == (N, M)]
                L2 = len(sel[0].rx)
                rxb = torch.from_numpy(np.concatenate([j.rx for j in sel])).cuda()
                t = g.autotune(codes[(N, N // 2)], M, rxb, np.arange(len(sel), dtype=np.uint64) * L2,
                               [j.cap for j in sel], [j.noise_var for j in sel], reps=2)
                buckets[f"{N},{M}"] = {"words": len(sel), "best": t["best"], "ms": t["ms"]}
        bplan, _ = device_batch(g, jobs, codes, launch_mode=2)
        bucket_ms = time_launches(bplan.launch, reps, stream)
        r_bucket = host_outputs(bplan, len(jobs))
    finally:
        g.set_tuning(0, 0, **before)
        for k, t in saved.items():
            g.set_tuning(*k, **t)
    q = r_graph[1].astype(np.float64)
    return {"workload": "uneven_mix: 16384 words, N in {64,128,256,512} (K=N/2), M in {4,16,64}, "
                        "Eb/N0 ~ U[2,8] dB, cap 2^18, one merged launch",
            "eager_ms": eager_ms, "graph_ms": graph_ms,
            "useful_checks_per_s": q.sum() / (graph_ms / 1e3),
            "codewords_per_s": len(jobs) / (graph_ms / 1e3), "mean_q": float(q.mean()),
            "abandon_rate": float(r_graph[2].mean()),
            "status_errors": int((r_graph[3] != 0).sum()),
            "graph_equals_eager": all(np.array_equal(x, y) for x, y in zip(r_eager, r_graph)),
            "roofline": uneven_roofline(jobs, q, graph_ms),
            "autotuned": ({"best": tuned["best"], "sample_ms": tuned["ms"],
                           "default_sample_ms": next((t["ms"] for t in tuned["table"]
                                                      if t["tuning"] == before), None)}
                          if tuned else None),
            "per_bucket_launches": {"ms": bucket_ms, "tunings": buckets,
                                    "useful_checks_per_s": q.sum() / (bucket_ms / 1e3),
                                    "identical_results": all(np.array_equal(x, y) for x, y in
                                                             zip(r_bucket, r_graph)),
                                    "merged_over_buckets": bucket_ms / graph_ms}}, r_graph


def hard_words(g, w, jobs):
    """The hard-decision words yhat of jobs as decoded by the library with a
    query cap of 1 (device tensor, ceil(N/64) int64 per word)."""
    import torch
    plan, _ = device_batch(g, jobs, cap=1)
    plan.launch()
    torch.cuda.synchronize()
    nw = (jobs[0].N + 63) // 64
    return plan.out.codewords[:len(jobs), :nw].contiguous()


def dense_baseline(g, w, jobs128, jobs1k, inc_rate):
    """The paper's Step 5 model (one full Algorithm 1 product per pattern) on
    the hard decisions of the benchmark's own received words."""
    code = g.Code(128, w.polar_code(128, 64).h_rows)
    code1k = g.Code(1024, w.polar_code(1024, 512).h_rows)
    y128 = hard_words(g, w, jobs128)
    y1k = hard_words(g, w, jobs1k)
    d128, _ = g.probe_dense_pmult(code, len(jobs128), 4096, words_dev=y128)
    d1k, _ = g.probe_dense_pmult(code1k, len(jobs1k), 256, words_dev=y1k)
    return {"what": "one full Algorithm 1 product per pattern (Step 5 as printed), "
                    "grand_probe_dense_pmult, on the hard decisions of the workload's received "
                    "words (polar128_16qam x 4096 patterns, polar1024_256qam x 256 patterns)",
            "N128_checks_per_s": d128, "N1024_checks_per_s": d1k,
            "incremental_performed_checks_per_s_N128": inc_rate,
            "incremental_over_dense_N128": inc_rate / d128}


def other_basis(g, w, jobs, ref, reps: int = 10):
    """The batch decoded with the sparsest basis of H (reduced row echelon,
    Table II's basis: 984 ones at N = 128 against 1768): time and results."""
    import torch
    h = w.polar_code(128, 64).h_dense
    hr = w.rref_basis(h)
    code = g.Code(128, w.pack_bits(hr))
    plan, _ = device_batch(g, jobs, codes={(128, 64): code})
    ms = time_launches(plan.launch, reps, torch.cuda.current_stream())
    out = host_outputs(plan, len(jobs))
    return {"basis": "RREF of H (pivot columns from the left)", "ones": int(hr.sum()),
            "ones_frozen_column_basis": int(h.sum()), "ms_per_launch": ms,
            "identical_results": all(np.array_equal(x, y) for x, y in zip(out, ref))}


def cpu_leg(jobs_by_cfg, gpu_by_cfg, cpu_sample: int):
    """The oracle on the host cores: the headline workload's baseline on a
    bounded sample, the other workloads' samples, and the parity of every
    sample (the whole headline batch included) with the GPU results."""
    import oracle
    import workload as w
    oracle.build(force=False)
    nthreads = workers()
    h_rows = lambda N, K: w.polar_code(N, K).h_rows    # noqa: E731
    parity, per_config = {}, {}
    base = None
    for cfg, jobs in jobs_by_cfg.items():
        gcw, gq, gab, gst = gpu_by_cfg[cfg]
        if cfg == WORKLOAD:
            # timed baseline sample first, then the rest of the batch for parity
            a = oracle.decode_jobs(jobs[:cpu_sample], h_rows, nthreads=nthreads)
            b = oracle.decode_jobs(jobs[cpu_sample:], h_rows, nthreads=nthreads)
            cws = list(a[0]) + list(b[0])
            q = np.concatenate([a[1], b[1]])
            ab = np.concatenate([a[2], b[2]])
            secs, used, wall = a[3], a[4], a[5]
            sq = float(a[1].sum())
            base = {"value": sq / wall, "unit": "TEP syndrome checks/s", "cores": int(used),
                    "kind": "oracle", "cpu_model": cpu_model(),
                    "sample": f"first {cpu_sample} of the {len(jobs)} codewords (same seeds), "
                              f"{wall:.2f} s wall, {secs.sum():.1f} s of CPU work",
                    "codewords_per_s": cpu_sample / wall,
                    "p50_ms_per_decode_1thread": float(np.percentile(secs, 50) * 1e3),
                    "p99_ms_per_decode_1thread": float(np.percentile(secs, 99) * 1e3)}
        else:
            cws, q, ab, secs, used, wall = oracle.decode_jobs(jobs, h_rows, nthreads=nthreads)
            per_config[cfg] = {"codewords": len(jobs), "checks_per_s": float(q.sum()) / wall,
                               "codewords_per_s": len(jobs) / wall, "cores": int(used),
                               "wall_s": wall, "cpu_s": float(secs.sum()),
                               "p50_ms_per_decode_1thread": float(np.percentile(secs, 50) * 1e3),
                               "p99_ms_per_decode_1thread": float(np.percentile(secs, 99) * 1e3)}
        bad = 0
        for i, j in enumerate(jobs):
            nw = (j.N + 63) // 64
            if (int(gq[i]) != int(q[i]) or int(gab[i]) != int(ab[i]) or int(gst[i]) != 0 or
                    not np.array_equal(np.asarray(gcw[i])[:nw], cws[i])):
                bad += 1
        parity[cfg] = {"codewords": len(jobs), "mismatches": bad}
        log(f"oracle {cfg}: {len(jobs)} words, {bad} mismatches")
    base["per_config"] = per_config
    return base, parity


# Eb/N0 grids (dB, energy per coded bit) where each order's BLER falls.
SWEEP_EBN0 = {M: tuple(lo + 2 * k for k in range(7))
              for M, lo in ((4, 0), (16, 4), (64, 8), (256, 12), (1024, 16), (4096, 20))}
SWEEP_CHUNK = 25000   # codewords per launch (bounds host and device memory)


def bler_sweep(g, w, trials: int, S: int):
    """BLER and abandon rate of Algorithm 2 with cut-off S over N = 32..1024
    and M = 4..4096 (the grid of Section V's Figure 4), `trials` seeded
    codewords per point, decoded in batches on the GPU."""
    import torch
    rows = []
    t0 = time.time()
    for N in (32, 64, 128, 256, 512, 1024):
        code_w = w.polar_code(N, N // 2)
        code = g.Code(N, code_w.h_rows)
        for M in (4, 16, 64, 256, 1024, 4096):
            for ebn0 in SWEEP_EBN0[M]:
                rng = np.random.default_rng(N * 1_000_003 + M * 101 + ebn0)
                s2 = w.noise_variance(M, ebn0)
                errors = abandons = 0
                ms = 0.0
                for c0 in range(0, trials, SWEEP_CHUNK):
                    cnt = min(SWEEP_CHUNK, trials - c0)
                    u = rng.integers(0, 2, (cnt, N // 2), dtype=np.uint8)
                    c = code_w.encode(u)
                    rx = w.awgn(w.modulate(c, M).astype(np.float64), s2, rng).reshape(cnt, -1)
                    L2 = rx.shape[1]
                    plan = g.BatchPlan([code], np.zeros(cnt, np.uint32), [M] * cnt,
                                       [4 ** S] * cnt, [s2] * cnt,
                                       np.arange(cnt, dtype=np.uint64) * L2,
                                       torch.from_numpy(np.ascontiguousarray(rx).reshape(-1)).cuda(),
                                       cutoff=S)
                    a = torch.cuda.Event(enable_timing=True)
                    b = torch.cuda.Event(enable_timing=True)
                    a.record()
                    out = plan.launch()
                    b.record()
                    torch.cuda.synchronize()
                    ms += a.elapsed_time(b)
                    nw = (N + 63) // 64
                    dec = out.codewords.cpu().numpy().view(np.uint64)[:, :nw]
                    errors += int((~np.all(dec == w.pack_bits(c), axis=1)).sum())
                    abandons += int(out.abandoned.cpu().numpy().sum())
                rows.append({"N": N, "M": M, "ebn0_db": ebn0, "bler": errors / trials,
                             "abandon": abandons / trials, "ms": ms})
            log(f"sweep N={N} M={M} done ({time.time() - t0:.1f}s)")
    return {"metric": "BLER / abandon rate", "S": S, "cap": 4 ** S, "trials_per_point": trials,
            "ebn0": "dB per coded bit", "data": "synthetic", "points": rows}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--count", type=int, default=8192)
    ap.add_argument("--cpu-sample", type=int, default=2048)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serve-count", type=int, default=200_000)
    ap.add_argument("--plain-count", type=int, default=20_000)
    ap.add_argument("--latency-reps", type=int, default=100)
    ap.add_argument("--bler-sweep", type=int, default=0, metavar="TRIALS",
                    help="only run the BLER/abandon sweep with TRIALS codewords per point "
                         "and print its JSON line")
    ap.add_argument("--no-uneven", dest="uneven", action="store_false",
                    help="skip the uneven (mixed-size), small and long-codeword workloads")
    ap.add_argument("--no-dense-baseline", dest="dense_baseline", action="store_false",
                    help="skip the dense per-pattern pMult baseline and the RREF basis")
    ap.add_argument("--cutoff", type=int, default=8,
                    help="also time Algorithm 2 with this symbol cut-off S (0: skip)")
    ap.add_argument("--pipeline-streams", type=int, default=2)
    ap.add_argument("--no-xor-probe", dest="xor_probe", action="store_false",
                    help="skip the measured bitwise peak (grand_probe_xor_rate)")
    ap.add_argument("--uneven-only", type=int, default=0, metavar="REPS",
                    help="only time REPS replays of the uneven batch's merged launch (no "
                         "autotuning) and print its JSON line (for profiling that launch)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain device copy of 256 MiB three times (the reference "
                         "kernel for scaling HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this decoder runs on one GPU; --gpus must be 1 "
                                   "(codewords are independent: see the sharding note)"}))
        sys.exit(2)

    # more hardware queues than server lanes plus the other streams, so every
    # lane's launches run side by side (read by HIP when it initialises)
    os.environ["GPU_MAX_HW_QUEUES"] = HW_QUEUES
    import workload as w
    if args.uneven_only:
        ujobs = w.config_jobs_parallel("uneven_mix", workers=workers())
        import torch
        import paper_2405_01808_amd as g
        assert torch.cuda.is_available(), "bench.py needs a GPU"
        g.init(0)
        plan, _ = device_batch(g, ujobs)
        graph = g.BatchGraph(plan)
        ms = time_launches(graph.launch, args.uneven_only, torch.cuda.current_stream())
        q = plan.out.queries.cpu().numpy().view(np.uint64)[:len(ujobs)].astype(np.float64)
        graph.close()
        print(json.dumps({"workload": "uneven_mix merged launch (graph replay)", "reps":
                          args.uneven_only, "ms_per_launch": ms,
                          "useful_checks_per_s": q.sum() / (ms / 1e3),
                          "roofline": uneven_roofline(ujobs, q, ms)}), flush=True)
        return
    # inputs first, before anything touches the GPU
    t0 = time.time()
    nwk = workers()
    jobs = w.config_jobs_parallel(WORKLOAD, count=args.count, workers=nwk)
    small_jobs = long_jobs = uneven_jobs = serve_jobs = None
    if args.uneven:
        small_jobs = w.config_jobs("polar32_qpsk")
        long_jobs = w.config_jobs_parallel("polar1024_256qam", workers=nwk)
        uneven_jobs = w.config_jobs_parallel("uneven_mix", workers=nwk)
    if args.serve_count:
        serve_jobs = w.config_jobs_parallel("serving_mix", count=args.serve_count, workers=nwk)
    log(f"generated inputs in {time.time() - t0:.1f}s ({nwk} workers)")

    import torch
    import paper_2405_01808_amd as g

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    g.init(0)
    if args.bler_sweep:
        print(json.dumps(bler_sweep(g, w, args.bler_sweep, args.cutoff or 8)), flush=True)
        return
    code = g.Code(128, w.polar_code(128, 64).h_rows)
    L2 = len(jobs[0].rx)
    rx = torch.from_numpy(np.concatenate([j.rx for j in jobs])).to(dev)
    offs = np.arange(len(jobs), dtype=np.uint64) * L2
    plan = g.BatchPlan([code], np.zeros(len(jobs), np.uint32), [j.M for j in jobs],
                       [j.cap for j in jobs], [j.noise_var for j in jobs], offs, rx)
    stream = torch.cuda.current_stream(dev)

    for i in range(args.warmup):
        plan.launch(stream)
        torch.cuda.synchronize()
        log(f"warmup {i + 1}/{args.warmup} done")
    if args.copy_calibration:
        src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log(f"copy calibration: 3 x {COPY_BYTES >> 20} MiB device copies done")

    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t_begin = time.perf_counter()
    for i in range(args.steps):
        starts[i].record(stream)
        out = plan.launch(stream)
        ends[i].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_begin
    launch_ms = [s.elapsed_time(e) for s, e in zip(starts, ends)]
    log(f"timed {args.steps} steps: {wall:.3f}s wall, launch ms {launch_ms}")

    # the same K steps with consecutive batches on two streams, so one
    # batch's last words overlap the next batch's start (reported beside the
    # headline, which keeps one launch at a time)
    pipe = None
    if args.pipeline_streams > 1:
        S = args.pipeline_streams
        pstreams = [torch.cuda.Stream(dev) for _ in range(S)]
        pplans = [plan] + [g.BatchPlan([code], np.zeros(len(jobs), np.uint32),
                                       [j.M for j in jobs], [j.cap for j in jobs],
                                       [j.noise_var for j in jobs], offs, rx) for _ in range(S - 1)]
        torch.cuda.synchronize()
        for p, st in zip(pplans, pstreams):
            p.launch(st)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for i in range(args.steps):
            pplans[i % S].launch(pstreams[i % S])
        torch.cuda.synchronize()
        pwall = time.perf_counter() - t1
        ref_q = plan.out.queries.cpu().numpy()
        pipe = {"streams": S, "steps": args.steps, "ms_per_step": pwall * 1e3 / args.steps,
                "identical_results": bool(all(np.array_equal(p.out.queries.cpu().numpy(), ref_q)
                                              for p in pplans))}
        log(f"pipelined {args.steps} steps on {S} streams: {pwall:.3f}s wall")

    # The timed steps relaunch one plan, so its job table stays resident on
    # the device.  Alternating it with the same words in reverse order makes
    # every launch upload its table first (host-to-device copy + dispatch).
    rev = np.arange(len(jobs))[::-1]
    rplan = g.BatchPlan([code], np.zeros(len(jobs), np.uint32), [jobs[i].M for i in rev],
                        [jobs[i].cap for i in rev], [jobs[i].noise_var for i in rev],
                        offs[rev].copy(), rx)
    fplans = [plan, rplan]
    fev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for i, (a, b) in enumerate(fev):
        a.record(stream)
        fplans[i % 2].launch(stream)
        b.record(stream)
    torch.cuda.synchronize()
    fwall = time.perf_counter() - t2
    fresh = {"ms_per_step": fwall * 1e3 / args.steps,
             "avg_launch_ms": float(np.mean([a.elapsed_time(b) for a, b in fev])),
             "identical_results": bool(np.array_equal(
                 rplan.out.queries.cpu().numpy()[::-1], plan.out.queries.cpu().numpy()))}
    log(f"fresh-table steps: {fwall:.3f}s wall")

    q = out.queries.cpu().numpy().view(np.uint64)
    ab = out.abandoned.cpu().numpy()
    st = out.status.cpu().numpy()
    checks = out.checks.cpu().numpy().view(np.uint64)
    cws = out.codewords.cpu().numpy().view(np.uint64)
    assert np.all(st == 0), f"device status errors: {np.unique(st)}"
    headline_out = host_outputs(plan, len(jobs))
    sum_q = float(q.sum())
    sum_checks = float(checks.sum())
    ms_per_step = wall * 1e3 / args.steps
    value = sum_q * args.steps / wall
    bler = float(np.mean([not np.array_equal(w.unpack_bits(cws[i, :2], 128), jobs[i].cw)
                          for i in range(len(jobs))]))
    avg_launch_s = float(np.mean(launch_ms)) / 1e3
    # per-check work of the incremental syndrome: (w + 1) * ceil(rows / 32)
    # 32-bit lane-ops, w = columns XORed from the parent (mean over queries)
    sw = json.load(open(STEP_WEIGHTS))
    ops_per_check = float(sw["lane_ops_per_query"])
    # the headline counts useful checks (the query counts q); checks performed
    # past a word's answer in its last band are reported beside it
    achieved = sum_q * ops_per_check / avg_launch_s
    achieved_performed = sum_checks * ops_per_check / avg_launch_s
    # the measured bitwise peak beside the unit-count one (after the timed region)
    probe_rate, _ = g.probe_xor_rate(1 << 14) if args.xor_probe else (None, None)

    result = {
        "metric": "TEP syndrome checks/s",
        "value": value,
        "unit": "checks/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": WORKLOAD_DESC, "codewords": len(jobs), "N": 128, "K": 64,
                   "M": 16, "query_cap": 1 << 16},
        "codewords_per_s": len(jobs) * args.steps / wall,
        "pipelined": (dict(pipe, value=sum_q * args.steps / (pipe["ms_per_step"] * args.steps / 1e3))
                      if pipe else None),
        "fresh_tables": dict(fresh, value=sum_q / (fresh["ms_per_step"] / 1e3)),
        "performed_checks_per_s": sum_checks * args.steps / wall,
        "mean_q": sum_q / len(jobs),
        "abandon_rate": float(ab.mean()),
        "bler": bler,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": ALU_PEAK,
                     "unit": "int32 lane-ops/s", "frac": achieved / ALU_PEAK,
                     "traffic": measured_traffic(), "traffic_unit": "HBM bytes per launch",
                     "kernel": "grand_decode_kernel_fixed<64, 9, true>",
                     "work": f"{ops_per_check:.3f} lane-ops ((mean w {sw['mean_w']:.3f} + 1) x "
                             f"ceil(64/32)) x {int(sum_q)} useful checks (sum of q) per launch",
                     "avg_launch_ms": avg_launch_s * 1e3,
                     "performed_checks_per_launch": int(sum_checks),
                     "achieved_with_performed_checks": achieved_performed,
                     "frac_with_performed_checks": achieved_performed / ALU_PEAK,
                     "measured_peak": probe_rate,
                     "frac_of_measured_peak": achieved / probe_rate if probe_rate else None},
    }
    gpu_by_cfg = {WORKLOAD: headline_out}
    cpu_jobs = {WORKLOAD: jobs}
    if serve_jobs:
        t0 = time.time()
        result["serving"], sres = serving(g, w, serve_jobs, args.plain_count)
        n5 = CPU_SAMPLES["serving_mix"]
        gpu_by_cfg["serving_mix"] = (np.array([r.codeword for r in sres[:n5]]),
                                     np.array([r.queries for r in sres[:n5]], np.uint64),
                                     np.array([r.abandoned for r in sres[:n5]], np.uint8),
                                     np.array([r.status for r in sres[:n5]], np.int32))
        cpu_jobs["serving_mix"] = serve_jobs[:n5]
        del sres
        log(f"serving replay done in {time.time() - t0:.1f}s")
    if args.uneven:
        t0 = time.time()
        result["plain_small"], o1 = plain_small(g, w, small_jobs)
        gpu_by_cfg["polar32_qpsk"] = o1
        cpu_jobs["polar32_qpsk"] = small_jobs[:CPU_SAMPLES["polar32_qpsk"]]
        result["long_batch"], o4 = long_batch(g, w, long_jobs)
        n4 = CPU_SAMPLES["polar1024_256qam"]
        gpu_by_cfg["polar1024_256qam"] = tuple(x[:n4] for x in o4)
        cpu_jobs["polar1024_256qam"] = long_jobs[:n4]
        result["uneven_batch"], o3 = uneven_batch(g, w, uneven_jobs)
        n3 = CPU_SAMPLES["uneven_mix"]
        gpu_by_cfg["uneven_mix"] = tuple(x[:n3] for x in o3)
        cpu_jobs["uneven_mix"] = uneven_jobs[:n3]
        log(f"small, long and uneven batches done in {time.time() - t0:.1f}s")
    if args.dense_baseline:
        t0 = time.time()
        dj = long_jobs if long_jobs else w.config_jobs("polar1024_256qam")
        result["dense_pmult_baseline"] = dense_baseline(g, w, jobs, dj,
                                                        sum_checks * args.steps / wall)
        result["rref_basis"] = other_basis(g, w, jobs, headline_out)
        result["rref_basis"]["frozen_column_basis_ms"] = avg_launch_s * 1e3
        log(f"dense pMult baseline and RREF basis done in {time.time() - t0:.1f}s")
    if args.cutoff:
        t0 = time.time()
        result["alg2_cutoff"] = cutoff_mode(g, w, jobs, code, rx, offs, args.cutoff)
        log(f"cut-off mode done in {time.time() - t0:.1f}s")
    if args.latency_reps:
        t0 = time.time()
        result["latency"] = latency(g, w, args.latency_reps)
        log(f"latency mode done in {time.time() - t0:.1f}s")
    if not args.no_cpu_baseline:
        t0 = time.time()
        base, parity = cpu_leg(cpu_jobs, gpu_by_cfg, min(args.cpu_sample, len(jobs)))
        result["parity_sample"] = parity
        result["cpu_baseline"] = base
        log(f"oracle leg done in {time.time() - t0:.1f}s")
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
