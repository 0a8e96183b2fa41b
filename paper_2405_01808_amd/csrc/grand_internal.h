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
constexpr uint32_t kMaxBlock = 1024;
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
    uint32_t pad;
};

struct KernelArgs {
    const DevCode *codes;
    const DevJob *jobs;
    uint32_t njobs;
    uint32_t low_bits;    // b
    uint32_t seg_len;     // S
    uint32_t first_band;  // patterns in the first band
    uint32_t node_cap;    // high-pattern store entries per workgroup
    uint32_t seg_cap;     // segment list entries per workgroup
    const float *rx;
    uint64_t *cw_out;
    uint64_t *q_out;
    uint8_t *ab_out;
    int32_t *status_out;  // may be null
    uint64_t *checks_out; // may be null
    uint32_t *queue;      // work counter, zero at launch
    uint8_t *scratch;     // per-workgroup slots
    uint64_t slot_bytes;
};

// Layout of one workgroup's scratch slot (byte offsets).
struct SlotLayout {
    uint64_t ncost, nparent, nrank, nptr, nsyn, seg, lsyn, total;
};

__host__ __device__ inline SlotLayout slot_layout(uint32_t node_cap, uint32_t seg_cap, uint32_t low_bits)
{
    SlotLayout s;
    auto al = [](uint64_t x) { return (x + 255) & ~uint64_t(255); };
    uint64_t o = 0;
    s.ncost = o;   o = al(o + 4ull * node_cap);
    s.nparent = o; o = al(o + 4ull * node_cap);
    s.nrank = o;   o = al(o + 4ull * node_cap);
    s.nptr = o;    o = al(o + 4ull * node_cap);
    s.nsyn = o;    o = al(o + 4ull * kMaxKW * node_cap);
    s.seg = o;     o = al(o + 8ull * seg_cap);
    s.lsyn = o;    o = al(o + 4ull * kMaxKW * (1ull << low_bits));
    s.total = o;
    return s;
}

// Dynamic LDS bytes for a low table of 2^b entries.
inline uint32_t dyn_lds_bytes(uint32_t low_bits)
{
    return 12u << low_bits;   // u64 sort keys + u32 leading syndrome words
}

// Launch the decoder for one group of jobs sharing a tuning.
int launch_decode(const KernelArgs &a, uint32_t grid, uint32_t block, void *stream);
int launch_reset(uint32_t *queue, void *stream);

}  // namespace grand
