// grand_internal.h -- structures shared by the host runtime and the HIP
// kernels of the GRAND decoder (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace grand {

constexpr uint32_t kMaxN = 1024;        // block length
constexpr uint32_t kMaxItems = 1024;    // 2L <= N for M >= 4
constexpr uint32_t kMaxKW = 16;         // syndrome words (rows <= 512)
constexpr uint32_t kMaxLowBits = 13;    // low table <= 8192 entries
constexpr uint32_t kMaxBlock = 1024;   // launches of few words use 1024-thread workgroups
constexpr uint32_t kNone = 0xFFFFFFFFu;
constexpr uint32_t kCwStride = 16;      // u64 words per codeword in batch outputs

// Device-side description of one code (pointers into device memory).
struct DevCode {
    uint32_t n;          // block length N
    uint32_t rows;       // rows of H (N - K)
    uint32_t kw;         // ceil(rows / 32): 32-bit words per syndrome / column
    uint32_t row_w32;    // 32-bit words per packed row of H (2 * ceil(n / 64))
    const uint32_t *h_rows;  // rows x row_w32, row-packed H (Algorithm 1)
    const uint32_t *h_cols;  // n x kw, column-packed H: column p = H[:, p]
};

// One codeword of a launch.
struct DevJob {
    uint32_t code;       // index into the launch's DevCode array
    uint32_t M;
    uint64_t rx_off;     // float offset of the word's 2L received values
    uint64_t cap;        // query cap
    uint32_t out;        // output slot (codeword at out * kCwStride)
    uint32_t cutoff;     // Algorithm 2's cut-off S (0: the full pattern space)
};

struct KernelArgs {
    const DevCode *codes;
    const DevJob *jobs;
    uint32_t njobs;
    uint32_t low_bits;    // b: flips in the sorted low table
    uint32_t first_band;  // patterns aimed at by the first band
    uint32_t band_growth; // later bands aim at growth x the patterns checked so far
    uint32_t node_cap;    // high-subset store entries per workgroup (HBM slot)
    uint32_t ni;          // power of two >= 2L of every job of the launch
    const float *rx;
    uint64_t *cw_out;
    uint64_t *q_out;
    uint8_t *ab_out;
    int32_t *status_out;  // may be null
    uint64_t *checks_out; // may be null
    unsigned long long *queue;  // work counter; a launch takes indices from qbase on
    unsigned long long qbase;   // counter value at launch: ends at qbase + njobs + grid
    uint8_t *scratch;     // grid x node_bytes(node_cap) bytes
    uint32_t *done_out;   // may be null: per-word completion flags (by output slot),
    uint32_t done_seq;    //   set to done_seq once the word's outputs are visible
    uint32_t pad2;
};

// Bytes of one workgroup's high-subset store: a 16-byte record per node.
__host__ __device__ inline uint64_t node_bytes(uint32_t node_cap)
{
    return 16ull * node_cap;
}

constexpr uint32_t kMergePer = 8;    // low-table merge outputs per thread and level
constexpr uint32_t kBucketsPerKey = 1;  // cost buckets per sorted key

// Dynamic LDS of the decode kernel, in 32-bit words: the hard word and its
// syndrome, the ranked flips and their columns' leading words (ni each),
// the low flips' columns, per-slot staging of a block of parents in an
// expansion pass (one slot per thread; the low table is built in it before
// the bands start), bucket indexes of the ranked flips and of the low table,
// the low table (keys and leading syndrome words, 2^b each) and the Bloom
// filter of its leading words.
struct LdsLayout {
    uint32_t yhat, s0, ikey, col0, lcol, foff, fa, fb, fcost, flead, fown, iidx, lidx, lkey,
        ltmp, ls0, lfilt, words;
};

// Bits of the low table's leading-word filter: 32 per entry up to 2^11
// entries (three bits of one 32-bit word per entry, ~0.3 % false positives
// at that load), 2^16 for larger tables.
__host__ __device__ inline uint32_t filter_log2(uint32_t low_bits)
{
    return (low_bits < 11 ? low_bits : 11) + 5;
}

__host__ __device__ inline LdsLayout lds_layout(uint32_t ni, uint32_t block, uint32_t low_bits)
{
    LdsLayout L;
    uint32_t o = 0;
    L.yhat = o;  o += kMaxN / 32;
    L.s0 = o;    o += kMaxKW;
    L.ikey = o;  o += ni;
    L.col0 = o;  o += ni;
    L.lcol = o;  o += kMaxLowBits * kMaxKW;
    // per-slot staging of a block of nodes (one slot per thread); the low
    // table's build buffer (2^low_bits, then the subset tables of its two
    // halves) and the cut-off's symbol scores (at most ni) overlay it, so it
    // is at least that long
    L.ltmp = o;
    L.foff = o;  o += block;
    L.fa = o;    o += block;
    L.fb = o;    o += block;
    L.fcost = o; o += block;
    L.flead = o; o += block;
    L.fown = o;  o += block;
    {
        const uint32_t lt = (1u << low_bits) + (1u << ((low_bits + 1) / 2)) +
                            (1u << (low_bits / 2));
        const uint32_t need = lt > ni ? lt : ni;
        if (o < L.ltmp + need)
            o = L.ltmp + need;
    }
    L.iidx = o;  o += kBucketsPerKey * ni + 2;
    L.lidx = o;  o += kBucketsPerKey * (1u << low_bits) + 2;
    o = (o + 1) & ~1u;          // 8-byte alignment of the table
    L.lkey = o;  o += 1u << low_bits;
    L.ls0 = o;   o += 1u << low_bits;
    L.lfilt = o; o += 1u << (filter_log2(low_bits) - 5);
    L.words = o;
    return L;
}

// Power of two >= 2L for block length n and modulation order M.
inline uint32_t items_pow2(uint32_t n, uint32_t M)
{
    uint32_t m = 0;
    while ((1u << (2 * (m + 1))) <= M)
        m++;
    uint32_t two_l = 2 * ((n + 2 * m - 1) / (2 * m));
    uint32_t p = 1;
    while (p < two_l)
        p <<= 1;
    return p;
}

// Launch the decoder for one group of jobs sharing a tuning.  Every
// workgroup takes indices until one is past the batch, so the counter
// advances by exactly njobs + grid.
int launch_decode(const KernelArgs &a, uint32_t grid, uint32_t block, void *stream);
// The same for the N = 128 16-QAM shape (256 threads, ni = 64, low_bits = 9),
// whose kernel is built in its own file; lds = dynamic LDS bytes.
int launch_decode_n128(const KernelArgs &a, uint32_t grid, uint32_t lds, void *stream);
// Zero n 64-bit counters with a kernel (graph-safe, unlike a memset node).
int launch_zero(unsigned long long *p, uint32_t n, void *stream);

}  // namespace grand
