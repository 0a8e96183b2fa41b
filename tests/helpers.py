"""Shared helpers of the parity tests: run a list of workload Jobs through the
oracle and through the HIP library, and compare element by element."""
from __future__ import annotations

import numpy as np

import workload as w


def h_rows(N, K):
    return w.polar_code(N, K).h_rows


def oracle_results(jobs, nthreads=None, cap=None, cutoff=0):
    import oracle
    cws, q, ab, secs, used, wall = oracle.decode_jobs(jobs, h_rows, nthreads=nthreads, cap=cap,
                                                      cutoff=cutoff)
    return cws, q, ab


class GpuCodes:
    """One Code handle per (N, K), created on demand."""

    def __init__(self):
        self.codes = {}
        self.order = []

    def index(self, N, K):
        import paper_2405_01808_amd as g
        key = (N, K)
        if key not in self.codes:
            self.codes[key] = (len(self.order), g.Code(N, h_rows(N, K)))
            self.order.append(self.codes[key][1])
        return self.codes[key][0]


def gpu_batch(jobs, codes: GpuCodes | None = None, cap=None, stream=None, cutoff=0):
    """Decode jobs in one grand_decode_batch call; returns numpy arrays
    (codewords [count, 16] uint64, q uint64, abandoned uint8, status int32,
    checks uint64)."""
    import torch
    import paper_2405_01808_amd as g
    codes = codes or GpuCodes()
    idx = np.array([codes.index(j.N, j.K) for j in jobs], np.uint32)
    offs = np.zeros(len(jobs), np.uint64)
    parts = []
    o = 0
    for i, j in enumerate(jobs):
        offs[i] = o
        parts.append(np.asarray(j.rx, np.float32))
        o += len(j.rx)
    rx = torch.from_numpy(np.concatenate(parts) if parts else np.zeros(1, np.float32)).cuda()
    caps = np.array([j.cap if cap is None else cap for j in jobs], np.uint64)
    nv = np.array([j.noise_var for j in jobs], np.float32)
    Ms = np.array([j.M for j in jobs], np.uint32)
    plan = g.BatchPlan(codes.order, idx, Ms, caps, nv, offs, rx, cutoff=cutoff)
    out = plan.launch(stream)
    torch.cuda.synchronize()
    return (out.codewords.cpu().numpy().view(np.uint64), out.queries.cpu().numpy().view(np.uint64),
            out.abandoned.cpu().numpy(), out.status.cpu().numpy(),
            out.checks.cpu().numpy().view(np.uint64))


def assert_parity(jobs, gpu, orc, indices=None, label=""):
    """Bit-exact decoded word, query count and abandon flag."""
    gcw, gq, gab, gst, gchk = gpu
    ocw, oq, oab = orc
    idxs = range(len(jobs)) if indices is None else indices
    bad = []
    for k, i in enumerate(idxs):
        j = jobs[i] if indices is None else jobs[i]
        nw = (j.N + 63) // 64
        o_k = i if indices is None else k
        ok = (gst[i] == 0 and int(gq[i]) == int(oq[o_k]) and int(gab[i]) == int(oab[o_k])
              and np.array_equal(gcw[i, :nw], ocw[o_k]))
        if not ok:
            bad.append((i, j.N, j.M, int(gst[i]), int(gq[i]), int(oq[o_k]), int(gab[i]),
                        int(oab[o_k])))
    assert not bad, f"{label}: {len(bad)} mismatches, first: {bad[:5]}"
    # performed checks are at least the query count
    for i in idxs:
        assert int(gchk[i]) >= int(gq[i]) or gab[i], (i, int(gchk[i]), int(gq[i]))


def make_plan(g, jobs):
    import torch
    codes, order, idx = {}, [], []
    for j in jobs:
        if (j.N, j.K) not in codes:
            codes[(j.N, j.K)] = len(order)
            order.append(g.Code(j.N, w.polar_code(j.N, j.K).h_rows))
        idx.append(codes[(j.N, j.K)])
    lens = [len(j.rx) for j in jobs]
    offs = np.concatenate([[0], np.cumsum(lens)[:-1]]).astype(np.uint64)
    rx = torch.from_numpy(np.concatenate([j.rx for j in jobs])).cuda()
    plan = g.BatchPlan(order, np.array(idx, np.uint32), [j.M for j in jobs],
                       [j.cap for j in jobs], [j.noise_var for j in jobs], offs, rx)
    return plan, order


def outputs(plan):
    o = plan.out
    return [t.cpu().numpy().copy() for t in (o.codewords, o.queries, o.abandoned, o.status,
                                              o.checks)]


def gf2_rref(A):
    """Reduced row echelon form over GF(2) (pivot columns left to right)."""
    A = (np.array(A, dtype=np.uint8) & 1).copy()
    r = 0
    for c in range(A.shape[1]):
        piv = [i for i in range(r, A.shape[0]) if A[i, c]]
        if not piv:
            continue
        A[[r, piv[0]]] = A[[piv[0], r]]
        for i in range(A.shape[0]):
            if i != r and A[i, c]:
                A[i] ^= A[r]
        r += 1
        if r == A.shape[0]:
            break
    return A
