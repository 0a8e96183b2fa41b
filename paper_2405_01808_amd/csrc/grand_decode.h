// grand_decode.h -- device code of the GRAND decoder for Gray M-QAM modulated
// polar codewords (arXiv 2405.01808, Section III, Algorithm 2), shared by the
// kernel files: grand_kernels.hip (generic, merged-batch and wide launch
// shapes, and the launchers) and grand_kernels_n128.hip (the N = 128 16-QAM
// shape, built on its own).
//
// One workgroup decodes one codeword at a time and pulls codewords from a
// work counter until the batch is drained (persistent launch).  The sorted
// flips, the low table and per-block staging live in LDS; the store of high
// subsets lives in the workgroup's HBM slot and is read block by block with
// coalesced loads.  Per codeword:
//
//  1. Demap (Algorithm 2 Step 1, Definitions 3.1 and 3.2): every (symbol,
//     axis) is quantised to Q.12, sliced to the nearest odd amplitude, and
//     yields the Gray bit whose flip moves to the near neighbour on the
//     received value's side (reversed at the constellation edge) with cost
//     d = 4096 - sigma * delta.  Flips are ranked by (cost, bit position)
//     (Step 2): each of up to 256 keys counts the keys below it, a bitonic
//     sort ranks more.
//  2. Hard-word syndrome s(yhat) = H yhat^T (Algorithm 1): AND of packed
//     rows with yhat, parity per 32-bit word, then a wavefront ballot folds
//     the words of a row -- the log2 N addition tree of pMult.
//  3. Patterns (Steps 4-5): a pattern T splits into T_l, a subset of the b
//     cheapest flips, and T_h, a subset of the others.  The 2^b low subsets
//     are tabulated sorted by (cost, colex): the subsets of the first six
//     are ranked in registers, then each further flip merges the table with
//     itself shifted by that flip (merge path).
//     The high subsets admitted so far ("nodes") form a forest: each node
//     adds one rank above its parent's largest.  Pattern (h, l) has syndrome
//     S_h + LS_l with S_h = s(yhat) + the node's columns, so checking it is
//     one comparison.  Only the leading 32-bit syndrome word is kept per
//     entry; the full K-bit comparison is rebuilt from the columns when the
//     leading words match.
//  4. Order and early exit: patterns are checked in bands between
//     thresholds that each admit a prefix of the (cost, colex) order (a
//     whole cost level, or part of one when a level is too large).  For a
//     fixed node the band's low entries form one contiguous range of the
//     sorted table, and one of them can have a zero syndrome only if its
//     leading word equals the node's: a Bloom filter of the table's
//     leading words rules out most nodes with one LDS read, and the rest
//     compare their range entry by entry.  The lowest (cost, colex) zero
//     syndrome of the first band that has one is the answer; its 1-based
//     rank q is counted exactly from the same sorted structures.  The search
//     abandons when the bands cover the query cap.
//
// Everything is integer arithmetic except one exact float scaling per
// received value; no packed-FP32 instructions are involved.

#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "grand_internal.h"

namespace grand {

namespace {

// Per-workgroup scalars (static LDS).
struct Shared {
    uint32_t job;
    uint32_t nitems;
    uint32_t err;
    uint32_t used;                   // nodes in the store
    uint32_t hit_cost;
    uint32_t best_tid;
    uint32_t best_h;
    uint32_t best_l;
    uint32_t ncand;                  // threads holding a hit of the band's lowest cost
    uint32_t overflow;
    int32_t cmax;
    unsigned long long acc;
    unsigned long long wband[kMaxBlock / 64];   // each wave's checks in the band
    uint32_t alloc;                  // node slots claimed in the current expansion
    uint32_t next;                   // next block of the check loop to take
    uint32_t fertile[2];             // by pass parity: a child created may have children
};

// Per-slot staging of one block of parents during an expansion pass (one
// slot per thread).
struct Stage {
    uint32_t *foff;    // flat offsets of the slots' child ranges
    uint32_t *fa;      // parent node of each slot
    uint32_t *fb;      // first child rank of each slot
    uint32_t *fcost;   // cost of each slot's parent
    uint32_t *flead;   // leading syndrome word of each slot's parent
    uint32_t *fown;    // marks of the parents' first children in a window of 64
};

// Per-workgroup arrays in dynamic LDS, sized for the launch (lds_layout).
struct Arr {
    uint32_t *yhat;    // hard word, 32-bit words
    uint32_t *s0;      // s(yhat)
    uint32_t *ikey;    // sorted flips (cost << 10 | position)
    uint32_t *col0;    // leading syndrome word of each rank's column
    uint32_t *lcol;    // full columns of the low flips
    Stage st;          // staging of a block, 64 slots per wave
    uint32_t *iidx;    // bucket index of the ranked flips
    uint32_t *lidx;    // bucket index of the low table
    uint32_t *lfilt;   // Bloom filter of the low table's leading words
};

// The low table's filter of its leading words is a blocked Bloom filter of
// 2^fbits bits in 32-bit words.  A multiplicative hash of word x picks one
// filter word by its top fbits - 5 bits (bits 21-31 at most) and three bits
// of that word by hash bits 6-10, 11-15 and 16-20.  Entering x ORs the three
// bits into the word; x can be in the table only if all three are set.  A
// test is one LDS read, as with a one-bit bitmap of the same size, and at 32
// bits per entry a tenth as many words pass it falsely (0.3 % against 3 %).
struct FiltKey {
    uint32_t word, mask;
};

__device__ inline FiltKey filt_key(uint32_t x, uint32_t fbits)
{
    const uint32_t h = x * 0x9E3779B1u;
    // (a field of width 0 at fbits = 5: the filter's only word)
    return FiltKey{__builtin_amdgcn_ubfe(h, 37u - fbits, fbits - 5u),
                   (1u << ((h >> 6) & 31u)) | (1u << ((h >> 11) & 31u)) | (1u << ((h >> 16) & 31u))};
}

// Node store in the workgroup's HBM slot: one 16-byte record per node, so a
// node is read or written whole with one instruction.
//   x  cost of the high subset
//   y  leading word of s(yhat) + its columns
//   z  parent (bits 0-20; node 0, the empty subset, has none) | first child
//      rank = own rank + 1 (b for node 0) << 21
//   w  low-table entries already checked with this node (bits 0-15) | first
//      child rank not yet in the store << 16; each half is also written alone
constexpr uint32_t kParBits = 21;
constexpr uint32_t kParMask = (1u << kParBits) - 1;

struct Nodes {
    uint4 *rec;

    __device__ uint32_t cost(uint32_t h) const { return rec[h].x; }
    __device__ uint32_t par(uint32_t h) const { return rec[h].z & kParMask; }
    __device__ uint32_t rl(uint32_t h) const { return rec[h].z >> kParBits; }
    __device__ void set_ptr(uint32_t h, uint32_t v) const
    {
        reinterpret_cast<uint16_t *>(rec + h)[6] = (uint16_t)v;
    }
    __device__ void set_cnext(uint32_t h, uint32_t v) const
    {
        reinterpret_cast<uint16_t *>(rec + h)[7] = (uint16_t)v;
    }
    __device__ void set(uint32_t h, uint32_t c, uint32_t ld, uint32_t p, uint32_t r1,
                        uint32_t pt, uint32_t cn) const
    {
        rec[h] = make_uint4(c, ld, (p & kParMask) | (r1 << kParBits), pt | (cn << 16));
    }
};

__device__ inline uint32_t lane_id() { return threadIdx.x & 63u; }

// Threads per workgroup: a compile-time constant in the kernels built for
// one launch shape (BS > 0), blockDim.x otherwise.
template <uint32_t BS>
__device__ inline uint32_t block_size()
{
    return BS ? BS : blockDim.x;
}

// Inclusive prefix sum across the 64 lanes of a wave, in data-parallel
// primitives (DPP) instead of LDS round trips: shifts by 1, 2, 4 and 8
// within each row of 16 lanes (lanes with no source add 0), then the last
// lane of row 0 is added to row 1, of row 2 to row 3 (row_bcast:15), and of
// row 1 to rows 2 and 3 (row_bcast:31).
__device__ inline uint32_t wave_incl_scan(uint32_t x)
{
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xf, 0xf, false);  // row_shr:1
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xf, 0xf, false);  // row_shr:2
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xf, 0xf, false);  // row_shr:4
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xf, 0xf, false);  // row_shr:8
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xa, 0xf, false);  // row_bcast:15
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xc, 0xf, false);  // row_bcast:31
    return x;
}

// Inclusive maximum across the 64 lanes of a wave, with the same DPP steps
// as wave_incl_scan (lanes with no source take 0).
__device__ inline uint32_t wave_incl_max(uint32_t x)
{
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xf, 0xf, false));
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xf, 0xf, false));
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xf, 0xf, false));
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xf, 0xf, false));
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xa, 0xf, false));
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xc, 0xf, false));
    return x;
}

// Orders the LDS accesses of one wave's lanes around it (no workgroup
// barrier): the compiler keeps them on their side, and the hardware runs
// one wave's LDS operations in order.
__device__ inline void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Bitonic sort of n (a power of two) keys in LDS, ascending.
template <uint32_t BS>
__device__ void bitonic_sort(uint32_t *a, uint32_t n)
{
    for (uint32_t k = 2; k <= n; k <<= 1) {
        for (uint32_t j = k >> 1; j > 0; j >>= 1) {
            for (uint32_t i = threadIdx.x; i < n; i += block_size<BS>()) {
                uint32_t ixj = i ^ j;
                if (ixj > i) {
                    uint32_t x = a[i], y = a[ixj];
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

// Sort n <= 2 * blockDim distinct keys in LDS by counting, for each key,
// the keys below it (one pass, all reads broadcast).  Pads (0xFFFFFFFF) are
// first made distinct and stay above every real key.
template <uint32_t BS>
__device__ void rank_sort(uint32_t *a, uint32_t n)
{
    for (uint32_t i = threadIdx.x; i < n; i += block_size<BS>())
        if (a[i] == 0xFFFFFFFFu)
            a[i] = 0xFFFF0000u | i;
    __syncthreads();
    uint32_t key[2] = {0, 0}, rank[2] = {0, 0};
    for (uint32_t c = 0; c < 2; c++) {
        uint32_t i = threadIdx.x + c * block_size<BS>();
        if (i < n) {
            key[c] = a[i];
            uint32_t r = 0;
            for (uint32_t j = 0; j < n; j++)
                r += a[j] < key[c];
            rank[c] = r;
        }
    }
    __syncthreads();
    for (uint32_t c = 0; c < 2; c++)
        if (threadIdx.x + c * block_size<BS>() < n)
            a[rank[c]] = key[c];
    __syncthreads();
}

// Low-table keys: cost << 13 | mask (cost < 2^19 for b <= 13 flips).
constexpr uint32_t kMaskBits = 13;
constexpr uint32_t kMaskAll = (1u << kMaskBits) - 1;

// Bucket index over keys sorted by cost (cost = key >> kshift): idx[u] is
// the first position whose cost >> shift is at least u, for u in [0, nb].
// A search for "first cost above x" then scans only x's bucket.
struct Buckets {
    const uint32_t *idx;
    uint32_t shift, nb;
};

__device__ inline uint32_t bucket_shift(uint32_t cmax, uint32_t nb)
{
    uint32_t s = 0;
    while ((cmax >> s) >= nb)
        s++;
    return s;
}

// The buckets up to the first key's and past the last key's are filled by
// all threads together (they can be half the index); the ones between two
// consecutive keys by the thread of the upper key.
template <uint32_t BS>
__device__ void build_buckets(const uint32_t *keys, uint32_t cnt, uint32_t kshift, uint32_t shift,
                              uint32_t nb, uint32_t *idx)
{
    const uint32_t head = cnt ? min((keys[0] >> kshift) >> shift, nb) : nb;
    const uint32_t tail = cnt ? ((keys[cnt - 1] >> kshift) >> shift) + 1 : nb + 1;
    for (uint32_t u = threadIdx.x; u <= nb; u += block_size<BS>()) {
        if (u <= head)
            idx[u] = 0;
        else if (u >= tail)
            idx[u] = cnt;
    }
    for (uint32_t i = 1 + threadIdx.x; i < cnt; i += block_size<BS>()) {
        const uint32_t u0 = ((keys[i - 1] >> kshift) >> shift) + 1;
        const uint32_t u1 = min((keys[i] >> kshift) >> shift, nb);
        for (uint32_t u = u0; u <= u1; u++)
            idx[u] = i;
    }
}

// First index in [lo, hi) whose cost exceeds x (keys sorted by cost; x
// below xlim, the bound that keeps x << kshift within 32 bits).  Costs and
// thresholds are 32-bit: a pattern of at most 1024 flips of cost below
// 2^15 costs less than 2^25, and thresholds stay below 2^26.
__device__ inline uint32_t ub_bucket(const uint32_t *keys, Buckets bk, uint32_t kshift,
                                     int32_t xlim, uint32_t lo, uint32_t hi, int32_t x)
{
    if (x < 0)
        return lo;
    if (x >= xlim)
        return hi;
    const uint32_t u = (uint32_t)x >> bk.shift;
    if (u >= bk.nb)
        return hi;
    uint32_t a = max(lo, bk.idx[u]), b = min(hi, bk.idx[u + 1]);
    const uint32_t key = ((uint32_t)x << kshift) | ((1u << kshift) - 1u);
    while (a < b) {
        uint32_t mid = (a + b) >> 1;
        if (keys[mid] > key)
            b = mid;
        else
            a = mid + 1;
    }
    return min(a, hi);
}

// Colex comparison of two high subsets given as nodes of the forest (each
// node adds a rank larger than every rank of its parent, so walking to the
// root lists the ranks in descending order).  Returns <0, 0, >0.
__device__ int colex_cmp(const Nodes &nd, uint32_t a, uint32_t b)
{
    for (;;) {
        if (a == b)
            return 0;
        if (a == 0)
            return -1;
        if (b == 0)
            return 1;
        const uint32_t za = nd.rec[a].z, zb = nd.rec[b].z;
        const uint32_t ra = za >> kParBits, rb = zb >> kParBits;
        if (ra != rb)
            return ra < rb ? -1 : 1;
        a = za & kParMask;
        b = zb & kParMask;
    }
}

// (h1, l1) < (h2, l2) in colex order of the whole pattern, for equal costs.
__device__ inline bool tep_less(const Nodes &nd, const uint32_t *lkey, uint32_t h1, uint32_t l1,
                                uint32_t h2, uint32_t l2)
{
    int c = colex_cmp(nd, h1, h2);
    if (c != 0)
        return c < 0;
    return (lkey[l1] & kMaskAll) < (lkey[l2] & kMaskAll);
}

// Full K-bit syndrome test of pattern (h, l) whose leading words matched:
// s(yhat) + columns of node h's ranks + columns of the low mask.
__device__ bool full_zero(const Arr &A, const Nodes &nd, const DevCode &code,
                          const uint32_t *lkey, uint32_t h, uint32_t l)
{
    const uint32_t kw = code.kw;
    const uint32_t mask = lkey[l] & kMaskAll;
    for (uint32_t w = 1; w < kw; w++) {
        uint32_t acc = A.s0[w];
        for (uint32_t x = h; x != 0; x = nd.par(x)) {
            uint32_t p = A.ikey[nd.rl(x) - 1] & 1023u;
            acc ^= code.h_cols[(uint64_t)p * kw + w];
        }
        for (uint32_t m = mask; m; m &= m - 1)
            acc ^= A.lcol[(__builtin_ctz(m)) * kw + w];
        if (acc)
            return false;
    }
    return true;
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

// The band loop keeps thresholds as (C, R) pairs and divides only on the
// rare store roll-back.
__device__ inline int64_t thr_lin(Thr t, uint32_t n) { return (int64_t)t.C * (n + 1) + t.R; }
__device__ inline bool thr_less(Thr a, Thr b) { return a.C < b.C || (a.C == b.C && a.R < b.R); }
__device__ inline Thr thr_whole(int32_t C, uint32_t n) { return Thr{C, (int32_t)n}; }
// the next threshold after t (admits one more rank step)
__device__ inline Thr thr_succ(Thr t, uint32_t n)
{
    return t.R < (int32_t)n ? Thr{t.C, t.R + 1} : Thr{t.C + 1, 0};
}

// Exclusive end of the child ranks r in [rl, n) whose child (cost cp + c_r,
// maxrank r) threshold k admits.  Costs ascend with r, so the admitted
// ranks are [rl, end).
__device__ inline uint32_t child_end(const uint32_t *ikey, Buckets ib, uint32_t rl, uint32_t n,
                                     Thr k, int32_t cp)
{
    // ranks [A, B) cost exactly C - cp; A is searched for only when that
    // run is not empty, which is rare
    const uint32_t B = ub_bucket(ikey, ib, 10, 1 << 22, rl, n, k.C - cp);
    if (B == rl || cp + (int32_t)(ikey[B - 1] >> 10) != k.C)
        return B;
    const uint32_t A = ub_bucket(ikey, ib, 10, 1 << 22, rl, B, k.C - 1 - cp);
    return max(A, min(B, (uint32_t)max(k.R, 0)));
}

// End of node h's admitted low-table entries under threshold k: entries with
// cost_h + LC < C, plus the run with cost_h + LC == C when the pattern's
// maxrank is below R (the node's own rank, or for the empty high subset the
// highest bit of the low mask; within a run masks ascend).
//
// SelectExits: the two early exits (nothing new in the node's range, or the
// whole rest of the table) are taken as selects after reading the first
// unchecked entry and the cost bucket at clamped indexes, instead of as
// nested branches.  The kernel of the N = 128 16-QAM shape uses this
// (measured 2 % faster); in the other shapes a branch-free search cost
// registers and time, so they keep the branches.
template <bool SelectExits = false>
__device__ inline uint32_t node_end(const uint32_t *lkey, Buckets lb, uint32_t LB, Thr k,
                                    int32_t ch, uint32_t h, uint32_t rl, uint32_t ptr)
{
    uint32_t b;
    if constexpr (SelectExits) {
        const int32_t x = k.C - ch;
        const uint32_t e0 = lkey[min(ptr, LB - 1)];
        const uint32_t ux = (uint32_t)max(x, 0) >> lb.shift;
        const uint32_t uc = min(ux, lb.nb - 1);
        const uint32_t i0 = lb.idx[uc], i1 = lb.idx[uc + 1];
        // nothing new (x >= 0 otherwise, as entry costs are not negative)
        const bool none = ptr >= LB || (int32_t)(e0 >> kMaskBits) > x;
        const bool rest = x >= (1 << 19) || ux >= lb.nb;   // every entry left
        uint32_t a = none ? ptr : (rest ? LB : max(ptr, i0));
        b = none ? ptr : (rest ? LB : min(LB, i1));
        const uint32_t key = ((uint32_t)min(x, (1 << 19) - 1) << kMaskBits) | kMaskAll;
        while (a < b) {   // first entry past cost x in the bucket
            const uint32_t mid = (a + b) >> 1;
            if (lkey[mid] > key)
                b = mid;
            else
                a = mid + 1;
        }
    } else {
        // entries before ptr are already checked, and the end never moves back
        if (ptr >= LB || ch + (int32_t)(lkey[ptr] >> kMaskBits) > k.C)
            return ptr;
        b = ub_bucket(lkey, lb, kMaskBits, 1 << 19, ptr, LB, k.C - ch);
    }
    // entries [a, b) cost exactly C - ch; a is searched for only when that
    // run is not empty, which is rare
    if (b == ptr || ch + (int32_t)(lkey[b - 1] >> kMaskBits) != k.C)
        return b;
    const uint32_t a = ub_bucket(lkey, lb, kMaskBits, 1 << 19, ptr, b, k.C - 1 - ch);
    if (b == a)
        return a;
    if (h != 0)
        return (int32_t)(rl - 1) < k.R ? b : a;
    if (k.R >= (int32_t)kMaskBits)
        return b;
    const uint32_t lim = 1u << k.R;   // masks below 2^R
    uint32_t lo = a, hi = b;
    while (lo < hi) {
        uint32_t mid = (lo + hi) >> 1;
        if ((lkey[mid] & kMaskAll) < lim)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

// Child rank r of a parent with cost cp is admitted by threshold k.
__device__ inline bool child_admitted(const uint32_t *ikey, uint32_t r, Thr k, int32_t cp)
{
    const int32_t c = cp + (int32_t)(ikey[r] >> 10);
    return c < k.C || (c == k.C && (int32_t)r < k.R);
}

// Raise the node store from "every high subset admitted by kE" to those
// admitted by kwant.  The admitted child ranks of a parent form one
// contiguous range; children of old parents not admitted by kE are new, and
// so are all admitted children of new parents, so the store grows one
// forest level per pass.  Within a pass each wave takes every nw-th block of
// 64 parents on its own and claims its children's slots with one LDS atomic
// (slot order varies from run to run; nothing computed from the store
// depends on it).  When the store would overflow, the step is rolled back
// and the threshold gap halved.  Returns the threshold reached (kE when even
// the next threshold after kE does not fit; sh.overflow is then set).
template <uint32_t BS>
__device__ Thr expand_nodes(Shared &sh, const Arr &A, Buckets ibk, const Nodes &nd,
                            uint32_t n, uint32_t node_cap, Thr kE, Thr kwant, uint32_t &used_out)
{
    const uint32_t tid = threadIdx.x, bs = block_size<BS>();
    const uint32_t lane = lane_id();
    const uint32_t wid = (uint32_t)__builtin_amdgcn_readfirstlane((int)(tid >> 6));
    const uint32_t wstride = bs;   // 64 parents per wave and block
    const Stage S = Stage{A.st.foff + wid * 64, A.st.fa + wid * 64, A.st.fb + wid * 64,
                          A.st.fcost + wid * 64, A.st.flead + wid * 64, A.st.fown + wid * 64};
    const uint32_t used0 = sh.used;
    Thr kn = kwant;
    for (;;) {
        if (tid == 0) {
            sh.alloc = used0;
            sh.fertile[0] = 0;
        }
        __syncthreads();
        uint32_t pstart = 0, pend = used0, par = 0;
        bool first = true;
        for (;;) {   // one pass per forest level
            // the record of this lane's slot in the wave's next block is
            // loaded while the current block is processed (parents are not
            // written during a pass, except each one's own frontier).  The
            // load is unconditional, at an index clamped to the pass's last
            // parent (a line the workgroup has just used, so a load past the
            // end stays in the cache), and its fields are taken only in the
            // next iteration, so nothing waits for it before then.
            uint4 nx = nd.rec[min(pstart + wid * 64 + lane, pend - 1)];
            for (uint32_t c0 = pstart + wid * 64; c0 < pend; c0 += wstride) {
                const uint32_t h = c0 + lane;
                uint32_t cnt = 0, lead = 0;
                const uint4 v = nx;
                nx = nd.rec[min(h + wstride, pend - 1)];
                const uint32_t ch = v.x, ld = v.y;
                const uint32_t lo = first ? v.w >> 16 : v.z >> kParBits;
                if (h < pend && lo < n && child_admitted(A.ikey, lo, kn, (int32_t)ch)) {
                    lead = ld;
                    cnt = child_end(A.ikey, ibk, lo, n, kn, (int32_t)ch) - lo;
                }
                const uint32_t xs = wave_incl_scan(cnt);
                const uint32_t off = xs - cnt;
                const uint32_t total = (uint32_t)__builtin_amdgcn_readlane((int)xs, 63);
                uint32_t base = 0;
                if (lane == 0 && total)
                    base = atomicAdd(&sh.alloc, total);
                base = (uint32_t)__builtin_amdgcn_readlane((int)base, 0);
                // children past the capacity are not written; the pass then
                // ends in a roll-back
                const bool fits = (uint64_t)base + total <= node_cap;
                if (h < pend && (cnt || !first))
                    nd.set_cnext(h, lo + cnt);
                if (!total || !fits)
                    continue;
                wave_sync();   // the previous block's children are written
                S.fa[lane] = h;
                S.fb[lane] = lo;
                S.fcost[lane] = ch;
                S.flead[lane] = lead;
                S.foff[lane] = off;
                // children are written 64 at a time; the parent of child j
                // is the last lane whose first child is at or before j: each
                // parent marks its first child's slot in the window (lane + 1;
                // a window's other slots hold 0), and a wave maximum scan
                // carries the marks forward, starting from the previous
                // window's last parent
                bool fert = false;
                uint32_t carry = 0;
                for (uint32_t j0 = 0; j0 < total; j0 += 64) {
                    S.fown[lane] = 0;
                    wave_sync();
                    if (cnt && off >= j0 && off < j0 + 64)
                        S.fown[off - j0] = lane + 1;
                    wave_sync();
                    const uint32_t k1 = wave_incl_max(max(S.fown[lane], lane == 0 ? carry : 0u));
                    carry = (uint32_t)__builtin_amdgcn_readlane((int)k1, 63);
                    const uint32_t j = j0 + lane;
                    if (j < total) {
                        const uint32_t k = k1 - 1;
                        const uint32_t r = S.fb[k] + (j - S.foff[k]);
                        const uint32_t cc = S.fcost[k] + (A.ikey[r] >> 10);
                        nd.set(base + j, cc, S.flead[k] ^ A.col0[r], S.fa[k], r + 1, 0, r + 1);
                        // the next pass tests this child as a parent the same way
                        fert |= r + 1 < n && child_admitted(A.ikey, r + 1, kn, (int32_t)cc);
                    }
                    wave_sync();   // the marks are read before the next window clears them
                }
                if (__ballot(fert) && lane == 0)
                    sh.fertile[par] = 1;
            }
            // the pass's children are the next pass's parents; a pass whose
            // children cannot have children under kn is the last one
            __syncthreads();
            const uint32_t created = sh.alloc;
            const bool more = sh.fertile[par] != 0;
            if (tid == 0)
                sh.fertile[par ^ 1] = 0;
            __syncthreads();   // read before the next pass claims slots
            if (created > node_cap || created == pend || !more)
                break;
            pstart = pend;
            pend = created;
            first = false;
            par ^= 1;
        }
        const uint32_t used = sh.alloc;
        if (used <= node_cap) {
            if (tid == 0)
                sh.used = used;
            __syncthreads();
            used_out = used;
            return kn;
        }
        // roll back: drop the new nodes and restore the old child frontiers
        for (uint32_t h = tid; h < used0; h += bs)
            nd.set_cnext(h, child_end(A.ikey, ibk, nd.rl(h), n, kE, (int32_t)nd.cost(h)));
        __syncthreads();
        const int64_t vE = thr_lin(kE, n), vn = thr_lin(kn, n);
        if (vn - vE <= 1) {
            if (tid == 0)
                sh.overflow = 1;
            __syncthreads();
            used_out = used0;
            return kE;
        }
        kn = thr_of(vE + (vn - vE) / 2, n);
    }
}

struct LaneHit {
    uint32_t cost, h, l;
};

__device__ inline void keep_best(LaneHit &best, const Nodes &nd, const uint32_t *lkey,
                                 uint32_t cost, uint32_t h, uint32_t l)
{
    if (best.h == kNone || cost < best.cost ||
        (cost == best.cost && tep_less(nd, lkey, h, l, best.h, best.l))) {
        best.cost = cost;
        best.h = h;
        best.l = l;
    }
}

// Low table: the 2^b subsets of the b cheapest flips as keys cost <<
// kMaskBits | mask, ascending (cost, then colex, which is the mask's integer
// order), with their leading syndrome words and a Bloom filter of those
// words (three bits of one filter word each, by filt_key).  The subsets of the first b0 =
// min(b, 6) flips are ranked in wave 0's registers: lane l holds subset l
// and counts the smaller keys with readlane, with no LDS round trip.  Each
// further flip j then merges the table with itself plus flip j (levels
// alternate between two buffers, one barrier per level, starting in the
// one that makes the last level land in lkey).  Node 0 (the empty high
// subset) is stored while the merges run.
template <uint32_t BS>
__device__ void build_low_table(const Arr &A, const Nodes &nd, uint32_t b, uint32_t *ltmp,
                                uint32_t *lkey, uint32_t *ls0)
{
    const uint32_t tid = threadIdx.x, bs = block_size<BS>(), LB = 1u << b;
    const uint32_t b0 = min(b, 6u), n0 = 1u << b0;
    uint32_t *src = ((b - b0) & 1) ? ltmp : lkey, *dst = ((b - b0) & 1) ? lkey : ltmp;
    if (tid < 64) {
        // the six costs are read at once and selected without branches; the
        // 64 comparisons are unrolled into four independent counts (lanes
        // past n0 hold the largest key and count for no one)
        uint32_t c6[6];
        for (uint32_t k = 0; k < 6; k++)
            c6[k] = k < b0 ? A.ikey[k] >> 10 : 0u;
        uint32_t cost = 0;
        for (uint32_t k = 0; k < 6; k++)
            cost += (tid >> k) & 1u ? c6[k] : 0u;
        const uint32_t key = tid < n0 ? (cost << kMaskBits) | tid : 0xFFFFFFFFu;
        uint32_t r4[4] = {0, 0, 0, 0};
#pragma unroll
        for (uint32_t m = 0; m < 64; m++)
            r4[m & 3] += (uint32_t)__builtin_amdgcn_readlane((int)key, (int)m) < key ? 1u : 0u;
        if (tid < n0)
            src[(r4[0] + r4[1]) + (r4[2] + r4[3])] = key;
    }
    const uint32_t fbits = filter_log2(b);
    for (uint32_t i = tid; i < (1u << (fbits - 5)); i += bs)
        A.lfilt[i] = 0;
    __syncthreads();   // also makes s(yhat) and the leading words visible
    if (tid == 0) {
        nd.set(0, 0, A.s0[0], 0, b, 0, b);
    }
    // XOR over every subset of the lower and of the upper half of the b
    // flips' leading words, behind the merge buffer
    const uint32_t blo = (b + 1) / 2, nlo = 1u << blo, nhi = 1u << (b - blo);
    uint32_t *sub = ltmp + LB;
    for (uint32_t i = tid; i < nlo + nhi; i += bs) {
        const bool upper = i >= nlo;
        const uint32_t first = upper ? blo : 0u;
        uint32_t acc = 0;
        for (uint32_t z = upper ? i - nlo : i; z; z &= z - 1)
            acc ^= A.col0[first + __builtin_ctz(z)];
        sub[i] = acc;
    }
    for (uint32_t j = b0; j < b; j++) {
        const uint32_t len = 1u << j, outn = 2 * len;
        const uint32_t add = ((A.ikey[j] >> 10) << kMaskBits) | (1u << j);
        const uint32_t per = (outn + bs - 1) / bs;   // <= kMergePer (checked on the host)
        const uint32_t i0 = min(outn, tid * per), i1 = min(outn, i0 + per);
        if (i0 < i1) {
            // co-rank: number of entries of the first list among the first
            // i0 outputs
            uint32_t lo = i0 > len ? i0 - len : 0, hi = min(i0, len);
            while (lo < hi) {
                uint32_t mid = (lo + hi) >> 1;
                if (src[mid] < src[i0 - mid - 1] + add)
                    lo = mid + 1;
                else
                    hi = mid;
            }
            uint32_t ia = lo, ib = i0 - lo;
            for (uint32_t o = i0; o < i1; o++) {
                bool takeA = ib >= len || (ia < len && src[ia] < src[ib] + add);
                dst[o] = takeA ? src[ia] : src[ib] + add;
                ia += takeA;
                ib += !takeA;
            }
        }
        __syncthreads();
        uint32_t *t = src;
        src = dst;
        dst = t;
    }
    if (b == b0)
        __syncthreads();   // the subset tables
    for (uint32_t i = tid; i < LB; i += bs) {
        const uint32_t msk = lkey[i] & kMaskAll;
        const uint32_t x = sub[msk & (nlo - 1)] ^ sub[nlo + (msk >> blo)];
        ls0[i] = x;
        const FiltKey fk = filt_key(x, fbits);
        atomicOr(&A.lfilt[fk.word], fk.mask);
    }
}

// Outputs of a word that could not be decoded (status < 0): q = 0 (never
// the result of a decode), abandoned, an all-zero codeword.  Thread 0 only.
__device__ void fail_word(const KernelArgs &a, uint32_t out_slot, int32_t status)
{
    uint64_t *cw = a.cw_out + (uint64_t)out_slot * kCwStride;
    for (uint32_t w = 0; w < kCwStride; w++)
        cw[w] = 0;
    a.q_out[out_slot] = 0;
    a.ab_out[out_slot] = 1;
    if (a.status_out)
        a.status_out[out_slot] = status;
    if (a.checks_out)
        a.checks_out[out_slot] = 0;
}

// Returns the word's output slot.  LBITS > 0: the launch's low-table bits
// are LBITS (a compile-time constant), else a.low_bits.
template <uint32_t BS, uint32_t LBITS, bool SelectExits = false>
__device__ uint32_t decode_one(const KernelArgs &a, Shared &sh, const Arr &A, uint32_t *lkey,
                               uint32_t *ltmp, uint32_t *ls0, const Nodes &nd, uint32_t jid)
{
    const uint32_t tid = threadIdx.x, bs = block_size<BS>();
    const DevJob job = a.jobs[jid];
    const DevCode code = a.codes[job.code];
    const uint32_t n_bits = code.n, kw = code.kw;
    uint32_t m = 0;
    while ((1u << (2 * (m + 1))) <= job.M && m < 6)
        m++;
    if (m == 0 || job.M != (1u << (2 * m)) || n_bits < 2 || n_bits > kMaxN || kw > kMaxKW ||
        2 * ((n_bits + 2 * m - 1) / (2 * m)) > a.ni) {
        // metadata the host never produces: fail the word rather than loop
        if (threadIdx.x == 0)
            fail_word(a, job.out, -1);   // GRAND_EINVAL
        return job.out;
    }
    const int32_t levels = 1 << m;
    const uint32_t L = (n_bits + 2 * m - 1) / (2 * m);
    const uint32_t nraw = 2 * L;
    uint32_t NI = 1;
    while (NI < nraw)
        NI <<= 1;

    // ---- Step 1: demap ------------------------------------------------
    for (uint32_t i = tid; i < kMaxN / 32; i += bs)
        A.yhat[i] = 0;
    for (uint32_t i = tid; i < kMaxKW; i += bs)
        A.s0[i] = 0;
    for (uint32_t i = tid; i < NI; i += bs)
        A.ikey[i] = 0xFFFFFFFFu;
    if (tid == 0) {
        sh.nitems = 0;
        sh.err = 0;
        sh.used = 1;
        sh.overflow = 0;
        sh.cmax = 0;
    }
    __syncthreads();
    uint32_t my_items = 0, my_cost = 0;   // at most 1024 flips of cost < 2^15
    const uint32_t cut = job.cutoff < L ? job.cutoff : 0u;   // Algorithm 2's S (0: none)
    for (uint32_t t = tid; t < nraw; t += bs) {
        const uint32_t sym = t >> 1, axis = t & 1u;
        float x = a.rx[job.rx_off + t];
        if (!(fabsf(x) <= 32768.0f)) {   // also catches NaN
            atomicOr(&sh.err, 1u);
            continue;
        }
        int32_t xq = __float2int_rn(x * 4096.0f);     // exact scaling, ties to even
        int32_t amp = 2 * (xq >> 13) + 1;                // floor division by 8192
        amp = max(-(levels - 1), min(levels - 1, amp));
        int32_t delta = xq - amp * 4096;
        int32_t sg = delta >= 0 ? 1 : -1;
        if (amp + 2 * sg > levels - 1 || amp + 2 * sg < -(levels - 1))
            sg = -sg;                                  // reflect at the edge
        int32_t d = 4096 - sg * delta;
        uint32_t cost = (uint32_t)min(d, 32767);
        uint32_t idx = (uint32_t)((amp + levels - 1) >> 1);
        uint32_t nbr = idx + (uint32_t)sg;
        uint32_t g = idx ^ (idx >> 1);
        uint32_t flip_bit = __builtin_ctz(max(idx, nbr));   // Gray(k-1)^Gray(k) = 2^ctz(k)
        uint32_t base = 2 * m * sym + m * axis;
        for (uint32_t k = 0; k < m; k++) {
            uint32_t p = base + k;
            if (p < n_bits && ((g >> (m - 1 - k)) & 1u))
                atomicOr(&A.yhat[p >> 5], 1u << (p & 31u));
        }
        uint32_t p = base + (m - 1 - flip_bit);
        if (p < n_bits) {
            A.ikey[t] = (cost << 10) | p;
            my_items++;
            my_cost += cost;
        }
        if (cut)
            A.col0[t] = cost;   // both axes, pad bits or not (col0 is free until Step 2)
    }
    {   // one atomic per wave for the flip count and the summed costs
        const uint32_t wi = wave_incl_scan(my_items), wc = wave_incl_scan(my_cost);
        if (lane_id() == 63) {
            atomicAdd(&sh.nitems, wi);
            atomicAdd((uint32_t *)&sh.cmax, wc);
        }
    }
    __syncthreads();
    const uint32_t out_slot = job.out;
    if (sh.err) {
        if (tid == 0)
            fail_word(a, out_slot, -1);   // GRAND_EINVAL
        return out_slot;
    }
    // ---- Algorithm 2 Steps 1-3 (cut-off): only the flips of the S least
    // reliable symbols take part.  A symbol's reliability is Definition
    // 3.1's L = sqrt(d1^2 + d2^2), compared as d1^2 + d2^2 of its two axes'
    // costs; ties go to the lower symbol index. ------------------------------
    if (cut) {
        for (uint32_t i = tid; i < L; i += bs) {
            const uint32_t c0 = A.col0[2 * i], c1 = A.col0[2 * i + 1];
            ltmp[i] = c0 * c0 + c1 * c1;   // < 2^31
        }
        if (tid == 0) {
            sh.nitems = 0;
            sh.cmax = 0;
        }
        __syncthreads();
        for (uint32_t i = tid; i < L; i += bs) {
            const uint32_t li = ltmp[i];
            uint32_t r = 0;
            for (uint32_t j = 0; j < L; j++) {
                const uint32_t lj = ltmp[j];
                r += lj < li || (lj == li && j < i);
            }
            if (r >= cut) {
                A.ikey[2 * i] = 0xFFFFFFFFu;
                A.ikey[2 * i + 1] = 0xFFFFFFFFu;
            }
        }
        __syncthreads();
        uint32_t ki = 0, kc = 0;
        for (uint32_t t = tid; t < nraw; t += bs) {
            const uint32_t k = A.ikey[t];
            if (k != 0xFFFFFFFFu) {
                ki++;
                kc += k >> 10;
            }
        }
        const uint32_t wi = wave_incl_scan(ki), wc = wave_incl_scan(kc);
        if (lane_id() == 63) {
            atomicAdd(&sh.nitems, wi);
            atomicAdd((uint32_t *)&sh.cmax, wc);
        }
        __syncthreads();
    }
    // ---- Step 2: rank the flips --------------------------------------
    if (NI <= 256 && NI <= 2 * bs)
        rank_sort<BS>(A.ikey, NI);
    else
        bitonic_sort<BS>(A.ikey, NI);
    const uint32_t n = sh.nitems;
    const int32_t cmax = sh.cmax;
    const uint32_t b = min(n, LBITS ? LBITS : a.low_bits);
    const uint32_t LB = 1u << b;

    // ---- Algorithm 1: s(yhat) = H yhat^T -----------------------------
    {
        const uint32_t wn = max(1u, n_bits >> 5);          // words per row, power of two
        const uint32_t total = code.rows * wn;
        for (uint32_t c0 = 0; c0 < total; c0 += bs) {
            uint32_t t = c0 + tid;
            uint32_t bit = 0;
            if (t < total) {
                uint32_t row = t / wn, w = t % wn;
                bit = __popc(code.h_rows[(uint64_t)row * code.row_w32 + w] & A.yhat[w]) & 1u;
            }
            unsigned long long vote = __ballot(bit);
            if (t < total && (t % wn) == 0) {
                uint32_t first = lane_id() & ~(wn - 1);
                unsigned long long mask = wn >= 64 ? ~0ull : ((1ull << wn) - 1);
                uint32_t parity = __popcll((vote >> first) & mask) & 1u;
                uint32_t row = t / wn;
                if (parity)
                    atomicOr(&A.s0[row >> 5], 1u << (row & 31u));
            }
        }
    }
    const uint32_t nbi = kBucketsPerKey * NI;
    const Buckets ibk{A.iidx, bucket_shift(n ? A.ikey[n - 1] >> 10 : 0u, nbi), nbi};
    build_buckets<BS>(A.ikey, n, 10, ibk.shift, nbi, A.iidx);
    // leading words of every rank's column, full columns of the low flips
    for (uint32_t r = tid; r < n; r += bs)
        A.col0[r] = code.h_cols[(uint64_t)(A.ikey[r] & 1023u) * kw];
    for (uint32_t i = tid; i < b * kw; i += bs) {
        uint32_t r = i / kw, w = i % kw;
        A.lcol[i] = code.h_cols[(uint64_t)(A.ikey[r] & 1023u) * kw + w];
    }
    // ---- low table: the 2^b subsets of the b cheapest flips in (cost,
    // colex) order, with their leading syndrome words -------------------
    build_low_table<BS>(A, nd, b, ltmp, lkey, ls0);
    const uint32_t nbl = kBucketsPerKey * LB;
    const Buckets lbk{A.lidx, bucket_shift(lkey[LB - 1] >> kMaskBits, nbl), nbl};
    build_buckets<BS>(lkey, LB, kMaskBits, lbk.shift, nbl, A.lidx);
    if (tid == 0)
        sh.next = bs;
    __syncthreads();

    // ---- bands ------------------------------------------------------------
    const uint64_t cap = job.cap;
    const Thr kmax = thr_whole(cmax, n);       // admits every pattern
    Thr kE{0, 0};                              // the store holds the empty high subset
    Thr kprev{-1, (int32_t)n};                 // nothing checked yet
    uint32_t used = 1;                         // nodes in the store (uniform)
    uint64_t cum = 0, checks = 0;
    float histC[2] = {0, 0}, histN[2] = {0, 0};
    uint32_t band = 0;
    bool found = false, abandon = false;
    uint64_t q = 0;
    uint32_t hit_h = kNone, hit_l = 0;
    uint64_t target = min<uint64_t>(cap, max<uint32_t>(a.first_band, 1u));

    for (;;) {
        // the band's threshold (uniform: every thread computes the same).
        // Only the amount of work per band depends on it, never the result:
        // the count grows roughly like a power of the cost threshold, so
        // the next threshold extrapolates the last two bands on a log scale.
        const float cp = (float)max(kprev.C, 0);
        float cd;
        if (band == 0) {
            uint64_t k = min<uint64_t>(target, max(1u, LB / 4)) - 1;
            cd = (float)(lkey[k] >> kMaskBits);
        } else if (band == 1 || histN[0] <= 0.0f) {
            cd = 2.0f * cp + 1.0f;
        } else {
            float al = __log2f(histN[1] / histN[0]) / __log2f((histC[1] + 1.0f) / (histC[0] + 1.0f));
            if (!(al > 0.05f) || !isfinite(al))
                cd = 2.0f * histC[1] + 1.0f;
            else
                cd = (histC[1] + 1.0f) * exp2f(__log2f((float)target / histN[1]) / al) - 1.0f;
        }
        if (!(cd < 4.0e7f))
            cd = 4.0e7f;
        Thr kt = thr_whole((int32_t)cd, n);
        if (thr_less(kmax, kt))
            kt = kmax;
        if (thr_less(kt, thr_succ(kprev, n)))
            kt = thr_succ(kprev, n);
        if (thr_less(kE, kt)) {
            kt = expand_nodes<BS>(sh, A, ibk, nd, n, a.node_cap, kE, kt, used);
            if (thr_less(kE, kt))
                kE = kt;
        }
        if (!thr_less(kprev, kt))      // the store cannot grow any further
            break;

        // checks.  Each wave takes blocks of 64 nodes on its own (its first
        // by its index, the others from a shared counter), with no workgroup
        // barrier until the band ends; each lane takes one node of the
        // block.  Pattern (node, entry) has a zero leading syndrome word iff
        // the entry's leading word equals the node's, so a node whose word
        // is not in the low table's filter has no candidate in its whole
        // range; the others (the filter's false positives and the real
        // matches) compare their range entry by entry.
        LaneHit best{0xFFFFFFFFu, kNone, 0};
        // (the wave index is uniform in a wave: readfirstlane keeps the
        // loop's bookkeeping in scalar registers)
        const uint32_t lane = lane_id(), nwv = bs >> 6;
        const uint32_t wid = (uint32_t)__builtin_amdgcn_readfirstlane((int)(tid >> 6));
        const uint32_t fbits = filter_log2(b);
        uint32_t lane_size = 0;
        // the record of this lane's slot in the wave's next block is loaded
        // while the current block is processed (unconditionally, at an
        // index clamped to the last node of the store; its fields are taken
        // in the next iteration)
        const uint32_t last = used - 1;
        uint4 nx = nd.rec[min(wid * 64 + lane, last)];
        for (uint32_t c0 = wid * 64; c0 < used;) {
            const uint32_t h = c0 + lane;
            const uint4 v = nx;
            const uint32_t lo = v.w & 0xFFFFu, ch = v.x, ld = v.y, rl = v.z >> kParBits;
            uint32_t cnt = 0;
            // the wave's next block comes from a shared counter, so waves
            // that finish early take more blocks; its records are requested
            // before this block's ranges are computed
            uint32_t cn = 0;
            if (lane == 0)
                cn = atomicAdd(&sh.next, 64u);
            cn = (uint32_t)__builtin_amdgcn_readlane((int)cn, 0);
            nx = nd.rec[min(cn + lane, last)];
            if (h < used) {
                uint32_t hi = node_end<SelectExits>(lkey, lbk, LB, kt, (int32_t)ch, h, rl, lo);
                if (hi > lo) {
                    cnt = hi - lo;
                    nd.set_ptr(h, hi);
                }
            }
            lane_size += cnt;
            bool cand = false;
            if (cnt) {
                const FiltKey fk = filt_key(ld, fbits);
                cand = (A.lfilt[fk.word] & fk.mask) == fk.mask;
            }
            // the filter's hits (false positives and real matches, about one
            // per two blocks): the whole wave compares each one's range, 64 entries
            // per step, and verifies the entries whose leading words match
            for (unsigned long long cm = __ballot(cand); cm; cm &= cm - 1) {
                const int k = __builtin_ctzll(cm);
                const uint32_t kh = (uint32_t)__builtin_amdgcn_readlane((int)h, k);
                const uint32_t klo = (uint32_t)__builtin_amdgcn_readlane((int)lo, k);
                const uint32_t kcnt = (uint32_t)__builtin_amdgcn_readlane((int)cnt, k);
                const uint32_t kld = (uint32_t)__builtin_amdgcn_readlane((int)ld, k);
                const uint32_t kch = (uint32_t)__builtin_amdgcn_readlane((int)ch, k);
                for (uint32_t t0 = 0; t0 < kcnt; t0 += 64) {
                    const uint32_t t = klo + t0 + lane;
                    if (t0 + lane < kcnt && ls0[t] == kld &&
                        full_zero(A, nd, code, lkey, kh, t))
                        keep_best(best, nd, lkey, kch + (lkey[t] >> kMaskBits), kh, t);
                }
            }
            c0 = cn;
        }
        {   // the wave's sum (a lane's sum is below 2^28, the wave's may not be)
            const uint32_t sl = wave_incl_scan(lane_size & 0xFFFFu);
            const uint32_t sh16 = wave_incl_scan(lane_size >> 16);
            if (lane == 63)
                sh.wband[wid] = ((unsigned long long)sh16 << 16) + sl;
        }

        // best hit of the band across the workgroup
        if (tid == 0)
            sh.hit_cost = 0xFFFFFFFFu;
        __syncthreads();
        uint64_t band_size = 0;
        for (uint32_t w = 0; w < nwv; w++)
            band_size += sh.wband[w];
        if (best.h != kNone)
            atomicMin(&sh.hit_cost, best.cost);
        __syncthreads();
        const uint32_t hc = sh.hit_cost;
        checks += band_size;
        cum += band_size;
        if (hc != 0xFFFFFFFFu) {
            const bool cand = best.h != kNone && best.cost == hc;
            if (tid == 0) {
                sh.best_tid = kNone;
                sh.ncand = 0;
                sh.acc = 0;
            }
            __syncthreads();
            if (cand) {
                atomicMin(&sh.best_tid, tid);
                atomicAdd(&sh.ncand, 1u);
            }
            __syncthreads();
            if (tid == sh.best_tid) {
                sh.best_h = best.h;
                sh.best_l = best.l;
            }
            // a tournament is needed only when several threads hold a hit
            // of the lowest cost (rare)
            const bool tie = sh.ncand > 1;
            __syncthreads();
            for (; tie;) {   // tournament among equal-cost hits, colex decides
                const uint32_t bh = sh.best_h, bl = sh.best_l;
                __syncthreads();
                if (tid == 0)
                    sh.best_tid = kNone;
                __syncthreads();
                if (cand && (best.h != bh || best.l != bl) &&
                    tep_less(nd, lkey, best.h, best.l, bh, bl))
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
            // rank: patterns with a smaller (cost, colex) key (sh.acc was
            // cleared before the barriers above)
            unsigned long long below = 0;
            for (uint32_t h = tid; h < used; h += bs) {
                int32_t ch = (int32_t)nd.cost(h);
                if (ch > (int32_t)hc)
                    continue;
                uint32_t lo = ub_bucket(lkey, lbk, kMaskBits, 1 << 19, 0, LB, (int32_t)hc - 1 - ch);
                uint32_t hi = ub_bucket(lkey, lbk, kMaskBits, 1 << 19, lo, LB, (int32_t)hc - ch);
                below += lo;
                if (hi > lo) {
                    int c = colex_cmp(nd, h, hit_h);
                    if (c < 0)
                        below += hi - lo;
                    else if (c == 0)
                        below += hit_l - lo;
                }
            }
            {   // the wave's sum, then one atomic per wave (a thread counts at
                // most 2^15 nodes of at most 2^13 entries, below 2^28, so the
                // wave sums of both halves fit in 32 bits).  An atomic of every
                // thread on the one address would run lane by lane.
                const uint32_t l16 = wave_incl_scan((uint32_t)below & 0xFFFFu);
                const uint32_t h16 = wave_incl_scan((uint32_t)(below >> 16));
                if (lane_id() == 63)
                    atomicAdd(&sh.acc, ((unsigned long long)h16 << 16) + l16);
            }
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
        if (!thr_less(kt, kmax)) {     // every pattern has been checked
            q = cum;
            abandon = true;
            break;
        }
        histC[0] = histC[1];
        histN[0] = histN[1];
        histC[1] = (float)kt.C + (float)kt.R / (float)(n + 1);
        histN[1] = (float)cum;
        kprev = kt;
        band++;
        target = min<uint64_t>(cap, cum * a.band_growth);
        if (tid == 0)
            sh.next = bs;
        __syncthreads();
    }
    __syncthreads();

    // ---- outputs ------------------------------------------------------
    const bool capacity_fail = !found && !abandon;
    if (tid == 0 && capacity_fail) {
        fail_word(a, out_slot, -5);   // GRAND_ECAPACITY
    } else if (tid == 0) {
        uint32_t flips[kMaxN / 32];
        for (uint32_t w = 0; w < kMaxN / 32; w++)
            flips[w] = 0;
        if (found) {
            for (uint32_t h = hit_h; h != 0; h = nd.par(h)) {
                uint32_t p = A.ikey[nd.rl(h) - 1] & 1023u;
                flips[p >> 5] ^= 1u << (p & 31u);
            }
            for (uint32_t msk = lkey[hit_l] & kMaskAll; msk; msk &= msk - 1) {
                uint32_t p = A.ikey[__builtin_ctz(msk)] & 1023u;
                flips[p >> 5] ^= 1u << (p & 31u);
            }
        }
        const uint32_t nw64 = (n_bits + 63) / 64;
        uint64_t *cw = a.cw_out + (uint64_t)out_slot * kCwStride;
        for (uint32_t w = 0; w < nw64; w++) {
            uint64_t lo32 = A.yhat[2 * w] ^ flips[2 * w];
            uint64_t hi32 = A.yhat[2 * w + 1] ^ flips[2 * w + 1];
            uint64_t word = lo32 | (hi32 << 32);
            if (n_bits < 64)
                word &= (1ull << n_bits) - 1;
            cw[w] = word;
        }
        a.q_out[out_slot] = q;
        a.ab_out[out_slot] = (uint8_t)(found ? 0 : 1);
        if (a.status_out)
            a.status_out[out_slot] = 0;
        if (a.checks_out)
            a.checks_out[out_slot] = checks;
    }
    return out_slot;
}

struct Workspace {
    Arr A;
    uint32_t *lkey, *ltmp, *ls0;
    Nodes nd;
};

// With BS, NI and LB given (> 0) every LDS offset is a compile-time constant.
template <uint32_t BS, uint32_t NI, uint32_t LB>
__device__ inline Workspace workspace(const KernelArgs &a, uint32_t *dyn)
{
    const LdsLayout ly = (BS && NI && LB) ? lds_layout(NI, BS, LB)
                                          : lds_layout(a.ni, blockDim.x, a.low_bits);
    Workspace w;
    w.A.yhat = dyn + ly.yhat;
    w.A.s0 = dyn + ly.s0;
    w.A.ikey = dyn + ly.ikey;
    w.A.col0 = dyn + ly.col0;
    w.A.lcol = dyn + ly.lcol;
    w.A.st = Stage{dyn + ly.foff, dyn + ly.fa, dyn + ly.fb, dyn + ly.fcost, dyn + ly.flead,
                   dyn + ly.fown};
    w.A.iidx = dyn + ly.iidx;
    w.A.lidx = dyn + ly.lidx;
    w.A.lfilt = dyn + ly.lfilt;
    w.lkey = dyn + ly.lkey;
    w.ltmp = dyn + ly.ltmp;
    w.ls0 = dyn + ly.ls0;
    w.nd.rec = (uint4 *)(a.scratch + (uint64_t)blockIdx.x * node_bytes(a.node_cap));
    return w;
}

// The persistent loop: each workgroup takes words until the batch is done.
template <uint32_t BS, uint32_t NI, uint32_t LB, bool SelectExits = false>
__device__ inline void decode_loop(const KernelArgs &a, Shared &sh)
{
    extern __shared__ __align__(16) uint32_t dyn[];
    const Workspace w = workspace<BS, NI, LB>(a, dyn);
    for (;;) {
        if (threadIdx.x == 0) {
            const unsigned long long c = atomicAdd(a.queue, 1ull) - a.qbase;
            sh.job = c < a.njobs ? (uint32_t)c : kNone;
        }
        __syncthreads();
        const uint32_t jid = sh.job;
        __syncthreads();
        if (jid == kNone)
            break;
        const uint32_t out =
            decode_one<BS, LB, SelectExits>(a, sh, w.A, w.lkey, w.ltmp, w.ls0, w.nd, jid);
        // thread 0 wrote every output of the word: publish them, then the flag
        if (a.done_out && threadIdx.x == 0)
            __hip_atomic_store(&a.done_out[out], a.done_seq, __ATOMIC_RELEASE,
                               __HIP_MEMORY_SCOPE_SYSTEM);
        __syncthreads();
    }
}

// The batch kernel for one launch shape fixed at compile time (256 threads,
// next power of two of 2L = NI, low table of 2^LB): LDS offsets and loop
// strides become immediates, which frees enough registers for 8 waves per
// SIMD (64 VGPRs) -- the most a SIMD holds.  Instantiated by the kernel
// files for the shapes they launch (SelectExits: see node_end).
template <uint32_t NI, uint32_t LB, bool SelectExits = false>
__global__ __launch_bounds__(256, 8) void grand_decode_kernel_fixed(KernelArgs a)
{
    __shared__ Shared sh;
    decode_loop<256, NI, LB, SelectExits>(a, sh);
}

}  // namespace

}  // namespace grand
