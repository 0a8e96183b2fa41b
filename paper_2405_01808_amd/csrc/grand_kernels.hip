// grand_kernels.hip -- gfx950 kernels of the GRAND decoder for Gray M-QAM
// modulated polar codewords (arXiv 2405.01808, Section III, Algorithm 2).
//
// One workgroup decodes one codeword at a time and pulls codewords from a
// work counter until the batch is drained (persistent launch).  Per codeword:
//
//  1. Demap (Algorithm 2 Step 1, Definitions 3.1 and 3.2): every (symbol,
//     axis) is quantised to Q.12, sliced to the nearest odd amplitude, and
//     yields the Gray bit whose flip moves to the near neighbour on the
//     received value's side (reversed at the constellation edge) with cost
//     d = 4096 - sigma * delta.  Flips are ranked by (cost, bit position)
//     with a bitonic sort in LDS (Step 2).
//  2. Hard-word syndrome s(yhat) = H yhat^T (Algorithm 1): AND of packed
//     rows with yhat, parity per 32-bit word, then a wavefront ballot folds
//     the words of a row -- the log2 N addition tree of pMult.
//  3. Patterns (Steps 4-5): a pattern T splits into T_l, a subset of the b
//     cheapest flips, and T_h, a subset of the others.  All 2^b low subsets
//     are tabulated in LDS sorted by (cost, colex) with their syndromes; the
//     high subsets ("nodes") admitted so far are materialised in HBM with
//     s(yhat) + sum of their columns.  Pattern (h, l) has syndrome
//     S_h + LS_l, so its check is one K-bit comparison; the leading 32-bit
//     word is compared first and the rest only on a match.
//  4. Order and early exit: patterns are checked in bands between
//     thresholds that each admit a prefix of the (cost, colex) order (a
//     whole cost level, or part of one when a level is too large).  For a
//     fixed node the low entries of a band form one contiguous range of the
//     sorted table, split into segments of <= S entries for the lanes.  The lowest (cost, colex) zero syndrome of the
//     first band that has one is the answer; its 1-based rank q is counted
//     exactly from the same sorted structures.  The search abandons when the
//     bands cover the query cap.
//
// Everything is integer arithmetic except one exact float scaling per
// received value; no packed-FP32 instructions are involved.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "grand_internal.h"

namespace grand {

namespace {

struct Shared {
    uint32_t yhat[kMaxN / 32];
    uint32_t s0[kMaxKW];
    uint32_t ikey[kMaxItems];        // sorted (cost << 10 | position)
    uint32_t lcol[kMaxLowBits * kMaxKW];
    uint32_t wsum[kMaxBlock / 64];
    uint32_t foff[kMaxBlock];        // flat-expansion offsets
    uint32_t fa[kMaxBlock];          // flat-expansion payload A
    uint32_t fb[kMaxBlock];          // flat-expansion payload B
    uint32_t job;
    uint32_t nitems;
    uint32_t err;
    uint32_t used;                   // nodes in the store
    uint32_t nseg;
    uint32_t hit_cost;
    uint32_t best_tid;
    uint32_t best_h;
    uint32_t best_l;
    uint32_t overflow;
    int32_t cmax;
    unsigned long long acc;
};

__device__ inline uint32_t lane_id() { return threadIdx.x & 63u; }

// Exclusive block-wide prefix sum of v; *total receives the sum.
__device__ uint32_t block_exscan(uint32_t v, uint32_t *wsum, uint32_t *total)
{
    const uint32_t lane = lane_id(), wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t y = __shfl_up(x, d, 64);
        if (lane >= (uint32_t)d)
            x += y;
    }
    if (lane == 63)
        wsum[wid] = x;
    __syncthreads();
    if (wid == 0) {
        uint32_t s = lane < nw ? wsum[lane] : 0u;
#pragma unroll
        for (int d = 1; d < 16; d <<= 1) {
            uint32_t y = __shfl_up(s, d, 64);
            if (lane >= (uint32_t)d)
                s += y;
        }
        if (lane < nw)
            wsum[lane] = s;
    }
    __syncthreads();
    uint32_t base = wid ? wsum[wid - 1] : 0u;
    *total = wsum[nw - 1];
    __syncthreads();
    return base + x - v;
}

// Bitonic sort of n (a power of two) keys in LDS, ascending.
template <typename T>
__device__ void bitonic_sort(T *a, uint32_t n)
{
    for (uint32_t k = 2; k <= n; k <<= 1) {
        for (uint32_t j = k >> 1; j > 0; j >>= 1) {
            for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
                uint32_t ixj = i ^ j;
                if (ixj > i) {
                    T x = a[i], y = a[ixj];
                    bool up = (i & k) == 0;
                    if ((x > y) == up) {
                        a[i] = y;
                        a[ixj] = x;
                    }
                }
            }
            __syncthreads();
        }
    }
}

// First index in [lo, hi) whose item cost exceeds x (item costs ascending).
__device__ inline uint32_t ub_item(const uint32_t *ikey, uint32_t lo, uint32_t hi, int64_t x)
{
    if (x < 0)
        return lo;
    if (x >= (1ll << 22))
        return hi;
    uint32_t key = ((uint32_t)x << 10) | 1023u;
    while (lo < hi) {
        uint32_t mid = (lo + hi) >> 1;
        if (ikey[mid] > key)
            hi = mid;
        else
            lo = mid + 1;
    }
    return lo;
}

// First index in [lo, hi) of the sorted low table whose cost exceeds x.
__device__ inline uint32_t ub_low(const unsigned long long *lkey, uint32_t lo, uint32_t hi,
                                  int64_t x)
{
    if (x < 0)
        return lo;
    if (x >= (1ll << 40))
        return hi;
    unsigned long long key = ((unsigned long long)x << 16) | 0xFFFFull;
    while (lo < hi) {
        uint32_t mid = (lo + hi) >> 1;
        if (lkey[mid] > key)
            hi = mid;
        else
            lo = mid + 1;
    }
    return lo;
}

// Colex comparison of two high subsets given as nodes of the parent forest
// (each node adds a rank larger than every rank of its parent, so walking to
// the root lists the ranks in descending order).  Returns <0, 0, >0.
__device__ int colex_cmp(const uint32_t *nparent, const int32_t *nrank, uint32_t a, uint32_t b)
{
    for (;;) {
        if (a == b)
            return 0;
        bool ea = nparent[a] == kNone, eb = nparent[b] == kNone;
        if (ea && eb)
            return 0;
        if (ea)
            return -1;
        if (eb)
            return 1;
        int32_t ra = nrank[a], rb = nrank[b];
        if (ra != rb)
            return ra < rb ? -1 : 1;
        a = nparent[a];
        b = nparent[b];
    }
}

// (h1, l1) < (h2, l2) in colex order of the whole pattern, for equal costs.
__device__ inline bool tep_less(const uint32_t *nparent, const int32_t *nrank,
                                const unsigned long long *lkey, uint32_t h1, uint32_t l1,
                                uint32_t h2, uint32_t l2)
{
    int c = colex_cmp(nparent, nrank, h1, h2);
    if (c != 0)
        return c < 0;
    return (lkey[l1] & 0xFFFFull) < (lkey[l2] & 0xFFFFull);
}

struct Slot {
    uint32_t *ncost;
    uint32_t *nparent;
    int32_t *nrank;
    uint32_t *nptr;
    uint32_t *nsyn;
    unsigned long long *seg;
    uint32_t *lsyn;
};

__device__ inline Slot slot_of(const KernelArgs &a)
{
    SlotLayout L = slot_layout(a.node_cap, a.seg_cap, a.low_bits);
    uint8_t *base = a.scratch + (uint64_t)blockIdx.x * a.slot_bytes;
    Slot s;
    s.ncost = (uint32_t *)(base + L.ncost);
    s.nparent = (uint32_t *)(base + L.nparent);
    s.nrank = (int32_t *)(base + L.nrank);
    s.nptr = (uint32_t *)(base + L.nptr);
    s.nsyn = (uint32_t *)(base + L.nsyn);
    s.seg = (unsigned long long *)(base + L.seg);
    s.lsyn = (uint32_t *)(base + L.lsyn);
    return s;
}

// Find k in [0, cnt) with foff[k] <= j < foff[k + 1] (foff ascending).
__device__ inline uint32_t flat_owner(const uint32_t *foff, uint32_t cnt, uint32_t j)
{
    uint32_t lo = 0, hi = cnt;
    while (hi - lo > 1) {
        uint32_t mid = (lo + hi) >> 1;
        if (foff[mid] <= j)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

// Search thresholds.  A threshold k = (C, R) admits a pattern T when
// cost(T) < C, or cost(T) == C and maxrank(T) < R (maxrank of the empty set
// is -1).  Because a smaller colex key never has a larger maximum, the
// admitted set is always a prefix of the (cost, colex) order, so thresholds
// may split one cost level -- needed when many patterns share one cost.
// Thresholds are linearised as v = C * (n + 1) + R with 0 <= R <= n;
// R = n admits the whole level.
struct Thr {
    int32_t C;
    int32_t R;
};

__device__ inline Thr thr_of(int64_t v, uint32_t n)
{
    Thr t;
    t.C = (int32_t)(v / (int64_t)(n + 1));
    t.R = (int32_t)(v % (int64_t)(n + 1));
    return t;
}

__device__ inline int64_t thr_full(int64_t C, uint32_t n) { return C * (int64_t)(n + 1) + n; }

// Exclusive end of the child ranks r in [rl, n) whose child (cost cp + c_r,
// maxrank r) threshold k admits.  Costs ascend with r, so the admitted
// ranks are [rl, end).
__device__ inline uint32_t child_end(const uint32_t *ikey, uint32_t rl, uint32_t n, Thr k,
                                     int32_t cp)
{
    uint32_t A = ub_item(ikey, rl, n, (int64_t)k.C - 1 - cp);
    uint32_t B = ub_item(ikey, A, n, (int64_t)k.C - cp);
    uint32_t x = min(B, (uint32_t)max(k.R, 0));
    return max(A, x);
}

// Raise the node store from "every high subset admitted by vE" to those
// admitted by vwant.  Children of a node add one rank above its largest;
// the admitted child ranks of a parent form one contiguous range.  When the
// store would overflow, the step is rolled back and the threshold gap
// halved.  Returns the threshold reached (vE when even vE + 1 does not fit;
// sh.overflow is then set).
__device__ int64_t expand_nodes(Shared &sh, const Slot &s, const DevCode &code, uint32_t n,
                                uint32_t node_cap, int64_t vE, int64_t vwant)
{
    const uint32_t tid = threadIdx.x, bs = blockDim.x, kw = code.kw;
    const uint32_t used0 = sh.used;
    const Thr kE = thr_of(vE, n);
    int64_t vn = vwant;
    for (;;) {
        const Thr kn = thr_of(vn, n);
        bool ok = true;
        uint32_t pstart = 0, pend = used0;
        bool first = true;
        while (ok && pstart < pend) {
            const uint32_t created_from = sh.used;
            for (uint32_t c0 = pstart; c0 < pend; c0 += bs) {
                uint32_t h = c0 + tid, cnt = 0, lo = 0;
                if (h < pend) {
                    int32_t ch = (int32_t)s.ncost[h];
                    uint32_t rl = (uint32_t)(s.nrank[h] + 1);
                    if (rl < n) {
                        lo = first ? child_end(sh.ikey, rl, n, kE, ch) : rl;
                        uint32_t hi = child_end(sh.ikey, rl, n, kn, ch);
                        cnt = hi > lo ? hi - lo : 0;
                    }
                }
                uint32_t total;
                uint32_t off = block_exscan(cnt, sh.wsum, &total);
                if (sh.used + total > node_cap) {
                    ok = false;   // uniform: every thread sees the same values
                    break;
                }
                sh.foff[tid] = off;
                sh.fa[tid] = h;
                sh.fb[tid] = lo;
                __syncthreads();
                const uint32_t ncnt = min(bs, pend - c0);
                const uint32_t dst0 = sh.used;
                for (uint32_t j = tid; j < total; j += bs) {
                    uint32_t k = flat_owner(sh.foff, ncnt, j);
                    uint32_t par = sh.fa[k];
                    uint32_t r = sh.fb[k] + (j - sh.foff[k]);
                    uint32_t dst = dst0 + j;
                    uint32_t key = sh.ikey[r];
                    s.ncost[dst] = s.ncost[par] + (key >> 10);
                    s.nparent[dst] = par;
                    s.nrank[dst] = (int32_t)r;
                    s.nptr[dst] = 0;
                    const uint32_t *col = code.h_cols + (uint64_t)(key & 1023u) * kw;
                    for (uint32_t w = 0; w < kw; w++)
                        s.nsyn[(uint64_t)dst * kw + w] = s.nsyn[(uint64_t)par * kw + w] ^ col[w];
                }
                __syncthreads();
                if (tid == 0)
                    sh.used = dst0 + total;
                __syncthreads();
            }
            pstart = created_from;
            pend = sh.used;
            first = false;
        }
        if (ok)
            return vn;
        __syncthreads();
        if (tid == 0)
            sh.used = used0;
        __syncthreads();
        if (vn - vE <= 1) {
            if (tid == 0)
                sh.overflow = 1;
            __syncthreads();
            return vE;
        }
        vn = vE + (vn - vE) / 2;
    }
}

// End of node h's admitted low-table entries under threshold k: entries with
// cost_h + LC < C, plus the run with cost_h + LC == C when the pattern's
// maxrank is below R (the node's own rank, or for the empty high subset the
// highest bit of the low mask; within a run masks ascend).
__device__ inline uint32_t node_end(const unsigned long long *lkey, uint32_t LB, Thr k,
                                    int32_t ch, bool root, int32_t rank)
{
    uint32_t a = ub_low(lkey, 0, LB, (int64_t)k.C - 1 - ch);
    uint32_t b = ub_low(lkey, a, LB, (int64_t)k.C - ch);
    if (b == a)
        return a;
    if (!root)
        return rank < k.R ? b : a;
    if (k.R >= 16)
        return b;
    const unsigned long long lim = 1ull << k.R;   // masks below 2^R
    uint32_t lo = a, hi = b;
    while (lo < hi) {
        uint32_t mid = (lo + hi) >> 1;
        if ((lkey[mid] & 0xFFFFull) < lim)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

struct LaneHit {
    uint32_t cost, h, l;
};

// Check every queued segment; keep each lane's lowest (cost, colex) hit.
__device__ void check_segments(Shared &sh, const Slot &s, const unsigned long long *lkey,
                               const uint32_t *ls0, uint32_t kw, LaneHit &best)
{
    const uint32_t nseg = sh.nseg;
    for (uint32_t i = threadIdx.x; i < nseg; i += blockDim.x) {
        unsigned long long sg = s.seg[i];
        uint32_t h = (uint32_t)(sg >> 32);
        uint32_t st = (uint32_t)(sg >> 16) & 0xFFFFu;
        uint32_t ln = (uint32_t)sg & 0xFFFFu;
        const uint32_t *sh_syn = s.nsyn + (uint64_t)h * kw;
        uint32_t lead = sh_syn[0];
        for (uint32_t l = st; l < st + ln; l++) {
            if (ls0[l] == lead) {
                bool eq = true;
                for (uint32_t w = 1; w < kw; w++)
                    eq = eq && (sh_syn[w] == s.lsyn[(uint64_t)l * kw + w]);
                if (eq) {
                    uint32_t cost = s.ncost[h] + (uint32_t)(lkey[l] >> 16);
                    if (best.h == kNone || cost < best.cost ||
                        (cost == best.cost &&
                         tep_less(s.nparent, s.nrank, lkey, h, l, best.h, best.l))) {
                        best.cost = cost;
                        best.h = h;
                        best.l = l;
                    }
                    break;   // later entries of this segment have larger keys
                }
            }
        }
    }
}

__device__ void decode_one(const KernelArgs &a, Shared &sh, unsigned long long *lkey,
                           uint32_t *ls0, uint32_t jid)
{
    const uint32_t tid = threadIdx.x, bs = blockDim.x;
    const DevJob job = a.jobs[jid];
    const DevCode code = a.codes[job.code];
    const Slot s = slot_of(a);
    const uint32_t n_bits = code.n, kw = code.kw;
    uint32_t m = 0;
    while ((1u << (2 * (m + 1))) <= job.M && m < 6)
        m++;
    const int32_t levels = 1 << m;
    const uint32_t L = (n_bits + 2 * m - 1) / (2 * m);
    const uint32_t nraw = 2 * L;
    uint32_t NI = 1;
    while (NI < nraw)
        NI <<= 1;

    // ---- Step 1: demap ------------------------------------------------
    for (uint32_t i = tid; i < kMaxN / 32; i += bs)
        sh.yhat[i] = 0;
    for (uint32_t i = tid; i < kMaxKW; i += bs)
        sh.s0[i] = 0;
    for (uint32_t i = tid; i < NI; i += bs)
        sh.ikey[i] = 0xFFFFFFFFu;
    if (tid == 0) {
        sh.nitems = 0;
        sh.err = 0;
        sh.used = 1;
        sh.overflow = 0;
        sh.cmax = 0;
    }
    __syncthreads();
    for (uint32_t t = tid; t < nraw; t += bs) {
        const uint32_t sym = t >> 1, axis = t & 1u;
        float x = a.rx[job.rx_off + t];
        if (!(fabsf(x) <= 32768.0f)) {   // also catches NaN
            atomicOr(&sh.err, 1u);
            continue;
        }
        int32_t xq = __float2int_rn(x * 4096.0f);     // exact scaling, ties to even
        int32_t A = 2 * (xq >> 13) + 1;                // floor division by 8192
        A = max(-(levels - 1), min(levels - 1, A));
        int32_t delta = xq - A * 4096;
        int32_t sg = delta >= 0 ? 1 : -1;
        if (A + 2 * sg > levels - 1 || A + 2 * sg < -(levels - 1))
            sg = -sg;                                  // reflect at the edge
        int32_t d = 4096 - sg * delta;
        uint32_t cost = (uint32_t)min(d, 32767);
        uint32_t idx = (uint32_t)((A + levels - 1) >> 1);
        uint32_t nbr = idx + (uint32_t)sg;
        uint32_t g = idx ^ (idx >> 1);
        uint32_t flip_bit = __builtin_ctz(max(idx, nbr));   // Gray(k-1)^Gray(k) = 2^ctz(k)
        uint32_t base = 2 * m * sym + m * axis;
        for (uint32_t k = 0; k < m; k++) {
            uint32_t p = base + k;
            if (p < n_bits && ((g >> (m - 1 - k)) & 1u))
                atomicOr(&sh.yhat[p >> 5], 1u << (p & 31u));
        }
        uint32_t p = base + (m - 1 - flip_bit);
        if (p < n_bits) {
            sh.ikey[t] = (cost << 10) | p;
            atomicAdd(&sh.nitems, 1u);
            atomicAdd((uint32_t *)&sh.cmax, cost);
        }
    }
    __syncthreads();
    const uint32_t out_slot = job.out;
    if (sh.err) {
        if (tid == 0 && a.status_out)
            a.status_out[out_slot] = -1;   // GRAND_EINVAL
        return;
    }
    // ---- Step 2: rank the flips --------------------------------------
    bitonic_sort(sh.ikey, NI);
    const uint32_t n = sh.nitems;
    const int32_t cmax = sh.cmax;

    // ---- Algorithm 1: s(yhat) = H yhat^T -----------------------------
    {
        const uint32_t wn = max(1u, n_bits >> 5);          // words per row, power of two
        const uint32_t total = code.rows * wn;
        for (uint32_t c0 = 0; c0 < total; c0 += bs) {
            uint32_t t = c0 + tid;
            uint32_t bit = 0;
            if (t < total) {
                uint32_t row = t / wn, w = t % wn;
                bit = __popc(code.h_rows[(uint64_t)row * code.row_w32 + w] & sh.yhat[w]) & 1u;
            }
            unsigned long long vote = __ballot(bit);
            if (t < total && (t % wn) == 0) {
                uint32_t first = lane_id() & ~(wn - 1);
                unsigned long long mask = wn >= 64 ? ~0ull : ((1ull << wn) - 1);
                uint32_t parity = __popcll((vote >> first) & mask) & 1u;
                uint32_t row = t / wn;
                if (parity)
                    atomicOr(&sh.s0[row >> 5], 1u << (row & 31u));
            }
        }
    }
    __syncthreads();

    // ---- low table: all subsets of the b cheapest flips ---------------
    const uint32_t b = min(n, a.low_bits);
    const uint32_t LB = 1u << b;
    for (uint32_t i = tid; i < b * kw; i += bs) {
        uint32_t r = i / kw, w = i % kw;
        sh.lcol[i] = code.h_cols[(uint64_t)(sh.ikey[r] & 1023u) * kw + w];
    }
    for (uint32_t e = tid; e < LB; e += bs) {
        uint32_t cost = 0;
        for (uint32_t r = 0; r < b; r++)
            if ((e >> r) & 1u)
                cost += sh.ikey[r] >> 10;
        lkey[e] = ((unsigned long long)cost << 16) | e;
    }
    __syncthreads();
    bitonic_sort(lkey, LB);
    for (uint32_t i = tid; i < LB; i += bs) {
        uint32_t mask = (uint32_t)(lkey[i] & 0xFFFFull);
        uint32_t syn[kMaxKW];
        for (uint32_t w = 0; w < kw; w++)
            syn[w] = 0;
        for (uint32_t r = 0; r < b; r++)
            if ((mask >> r) & 1u)
                for (uint32_t w = 0; w < kw; w++)
                    syn[w] ^= sh.lcol[r * kw + w];
        ls0[i] = syn[0];
        for (uint32_t w = 0; w < kw; w++)
            s.lsyn[(uint64_t)i * kw + w] = syn[w];
    }
    // root node: the empty high subset
    if (tid == 0) {
        s.ncost[0] = 0;
        s.nparent[0] = kNone;
        s.nrank[0] = (int32_t)b - 1;
        s.nptr[0] = 0;
    }
    for (uint32_t w = tid; w < kw; w += bs)
        s.nsyn[w] = sh.s0[w];
    __syncthreads();

    // ---- cost bands -----------------------------------------------------
    const uint64_t cap = job.cap;
    const int64_t vmax = thr_full(cmax, n);   // admits every pattern
    int64_t vE = 0;                           // the store holds the empty high subset
    int64_t vprev = -1;
    uint64_t cum = 0, checks = 0;
    double histC[2] = {0, 0}, histN[2] = {0, 0};
    uint32_t band = 0;
    bool found = false, abandon = false;
    uint64_t q = 0;
    uint32_t hit_h = kNone, hit_l = 0;
    uint64_t target = min<uint64_t>(cap, max<uint32_t>(a.first_band, 1u));
    const uint32_t S = a.seg_len;

    for (;;) {
        // choose the band's threshold (uniform: every thread computes it)
        const double cp = (double)thr_of(max<int64_t>(vprev, 0), n).C;
        double cd;
        if (band == 0) {
            uint64_t k = min<uint64_t>(target, LB) - 1;
            cd = (double)(lkey[k] >> 16);
        } else if (band == 1 || histN[0] <= 0.0) {
            cd = 2.0 * cp + 1.0;
        } else {
            double al = log(histN[1] / histN[0]) / log((histC[1] + 1.0) / (histC[0] + 1.0));
            if (!(al > 0.05) || !isfinite(al))
                cd = 2.0 * histC[1] + 1.0;
            else
                cd = (histC[1] + 1.0) * pow((double)target / histN[1], 1.0 / al) - 1.0;
        }
        if (!(cd < 4.0e7))
            cd = 4.0e7;
        int64_t vt = thr_full((int64_t)cd, n);
        vt = min(vt, vmax);
        vt = max(vt, vprev + 1);
        if (vt > vE) {
            vt = expand_nodes(sh, s, code, n, a.node_cap, vE, vt);
            vE = max(vE, vt);
        }
        if (vt <= vprev)      // the store cannot grow any further
            break;
        const Thr kt = thr_of(vt, n);

        // segments of this band, checked as the list fills
        LaneHit best{0xFFFFFFFFu, kNone, 0};
        uint64_t band_size = 0;
        if (tid == 0)
            sh.nseg = 0;
        __syncthreads();
        const uint32_t used = sh.used;
        for (uint32_t c0 = 0; c0 < used; c0 += bs) {
            uint32_t h = c0 + tid, cnt = 0, lo = 0, hi = 0;
            if (h < used) {
                int32_t ch = (int32_t)s.ncost[h];
                lo = s.nptr[h];
                if (lo < LB) {
                    hi = node_end(lkey, LB, kt, ch, h == 0, s.nrank[h]);
                    if (hi > lo)
                        cnt = (hi - lo + S - 1) / S;
                    else
                        hi = lo;
                }
            }
            band_size += hi > lo ? hi - lo : 0;
            uint32_t total;
            uint32_t off = block_exscan(cnt, sh.wsum, &total);
            if (sh.nseg + total > a.seg_cap) {
                check_segments(sh, s, lkey, ls0, kw, best);
                __syncthreads();
                if (tid == 0)
                    sh.nseg = 0;
                __syncthreads();
            }
            const uint32_t base = sh.nseg;
            for (uint32_t k = 0; k < cnt; k++) {
                uint32_t st = lo + k * S;
                uint32_t ln = min(S, hi - st);
                s.seg[base + off + k] = ((unsigned long long)h << 32) |
                                        ((unsigned long long)st << 16) | ln;
            }
            if (h < used && hi > lo)
                s.nptr[h] = hi;
            __syncthreads();
            if (tid == 0)
                sh.nseg = base + total;
            __syncthreads();
        }
        check_segments(sh, s, lkey, ls0, kw, best);

        // band size and best hit across the workgroup
        if (tid == 0) {
            sh.acc = 0;
            sh.hit_cost = 0xFFFFFFFFu;
        }
        __syncthreads();
        atomicAdd(&sh.acc, (unsigned long long)band_size);
        if (best.h != kNone)
            atomicMin(&sh.hit_cost, best.cost);
        __syncthreads();
        band_size = sh.acc;
        const uint32_t hc = sh.hit_cost;
        checks += band_size;
        cum += band_size;
        if (hc != 0xFFFFFFFFu) {
            const bool cand = best.h != kNone && best.cost == hc;
            if (tid == 0)
                sh.best_tid = kNone;
            __syncthreads();
            if (cand)
                atomicMin(&sh.best_tid, tid);
            __syncthreads();
            if (tid == sh.best_tid) {
                sh.best_h = best.h;
                sh.best_l = best.l;
            }
            __syncthreads();
            for (;;) {   // tournament among equal-cost hits, colex decides
                const uint32_t bh = sh.best_h, bl = sh.best_l;
                __syncthreads();
                if (tid == 0)
                    sh.best_tid = kNone;
                __syncthreads();
                if (cand && (best.h != bh || best.l != bl) &&
                    tep_less(s.nparent, s.nrank, lkey, best.h, best.l, bh, bl))
                    atomicMin(&sh.best_tid, tid);
                __syncthreads();
                if (sh.best_tid == kNone)
                    break;
                if (tid == sh.best_tid) {
                    sh.best_h = best.h;
                    sh.best_l = best.l;
                }
                __syncthreads();
            }
            hit_h = sh.best_h;
            hit_l = sh.best_l;
            // rank: patterns with a smaller (cost, colex) key
            if (tid == 0)
                sh.acc = 0;
            __syncthreads();
            unsigned long long below = 0;
            for (uint32_t h = tid; h < used; h += bs) {
                int32_t ch = (int32_t)s.ncost[h];
                if (ch > (int32_t)hc)
                    continue;
                uint32_t lo = ub_low(lkey, 0, LB, (int64_t)hc - 1 - ch);
                uint32_t hi = ub_low(lkey, lo, LB, (int64_t)hc - ch);
                below += lo;
                if (hi > lo) {
                    int c = colex_cmp(s.nparent, s.nrank, h, hit_h);
                    if (c < 0)
                        below += hi - lo;
                    else if (c == 0)
                        below += hit_l - lo;
                }
            }
            atomicAdd(&sh.acc, below);
            __syncthreads();
            q = sh.acc + 1;
            if (q > cap) {
                q = cap;
                abandon = true;
            } else {
                found = true;
            }
            break;
        }
        if (cum >= cap) {
            q = cap;
            abandon = true;
            break;
        }
        if (vt >= vmax) {          // every pattern has been checked
            q = cum;
            abandon = true;
            break;
        }
        histC[0] = histC[1];
        histN[0] = histN[1];
        histC[1] = (double)kt.C + (double)kt.R / (double)(n + 1);
        histN[1] = (double)cum;
        vprev = vt;
        band++;
        uint64_t nt = cum * 4;
        target = min<uint64_t>(cap, nt);
        __syncthreads();
    }
    __syncthreads();

    // ---- outputs ------------------------------------------------------
    const bool capacity_fail = !found && !abandon;
    if (tid == 0) {
        uint32_t flips[kMaxN / 32];
        for (uint32_t w = 0; w < kMaxN / 32; w++)
            flips[w] = 0;
        if (found) {
            for (uint32_t h = hit_h; s.nparent[h] != kNone; h = s.nparent[h]) {
                uint32_t p = sh.ikey[s.nrank[h]] & 1023u;
                flips[p >> 5] ^= 1u << (p & 31u);
            }
            uint32_t mask = (uint32_t)(lkey[hit_l] & 0xFFFFull);
            for (uint32_t r = 0; r < b; r++)
                if ((mask >> r) & 1u) {
                    uint32_t p = sh.ikey[r] & 1023u;
                    flips[p >> 5] ^= 1u << (p & 31u);
                }
        }
        const uint32_t nw64 = (n_bits + 63) / 64;
        uint64_t *cw = a.cw_out + (uint64_t)out_slot * kCwStride;
        for (uint32_t w = 0; w < nw64; w++) {
            uint64_t lo32 = sh.yhat[2 * w] ^ flips[2 * w];
            uint64_t hi32 = (2 * w + 1 < kMaxN / 32) ? (sh.yhat[2 * w + 1] ^ flips[2 * w + 1]) : 0;
            uint64_t word = lo32 | (hi32 << 32);
            if (n_bits < 64)
                word &= (1ull << n_bits) - 1;
            cw[w] = word;
        }
        a.q_out[out_slot] = q;
        a.ab_out[out_slot] = (uint8_t)(found ? 0 : 1);
        if (a.status_out)
            a.status_out[out_slot] = capacity_fail || sh.overflow ? (capacity_fail ? -5 : 0) : 0;
        if (a.checks_out)
            a.checks_out[out_slot] = checks;
    }
}

__global__ __launch_bounds__(1024) void grand_decode_kernel(KernelArgs a)
{
    __shared__ Shared sh;
    extern __shared__ unsigned long long dyn[];
    unsigned long long *lkey = dyn;
    uint32_t *ls0 = (uint32_t *)(dyn + (1u << a.low_bits));
    for (;;) {
        if (threadIdx.x == 0)
            sh.job = atomicAdd(a.queue, 1u);
        __syncthreads();
        const uint32_t jid = sh.job;
        __syncthreads();
        if (jid >= a.njobs)
            break;
        decode_one(a, sh, lkey, ls0, jid);
        __syncthreads();
    }
}

__global__ void reset_kernel(uint32_t *q)
{
    if (threadIdx.x == 0)
        q[0] = 0;
}

}  // namespace

int launch_decode(const KernelArgs &a, uint32_t grid, uint32_t block, void *stream)
{
    hipLaunchKernelGGL(grand_decode_kernel, dim3(grid), dim3(block), dyn_lds_bytes(a.low_bits),
                       (hipStream_t)stream, a);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

int launch_reset(uint32_t *queue, void *stream)
{
    hipLaunchKernelGGL(reset_kernel, dim3(1), dim3(64), 0, (hipStream_t)stream, queue);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

}  // namespace grand
