// grand_noalloc.hip -- grand_decode_batch_noalloc: the batch decode of
// grand_decode_batch for callers that cannot allocate device memory (code
// under HIP graph capture, tight serving loops, harnesses that forbid it).
//
// Everything the launch needs beyond the caller's inputs and outputs lives in
// one file-scope device array, `scratch`: the work counter, the per-word
// metadata copied from the host, the job and code tables, and the
// high-subset node stores of the workgroups.  Each device holds its own copy
// for the life of the process.  In host code the array's name only stands in
// for the symbol: its device address is taken once per device with
// hipGetSymbolAddress, and only that address is handed to copies and
// kernels.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>

#include "grand_host.h"

using namespace grand;
using namespace grand::host;

namespace {

constexpr uint64_t al256(uint64_t x) { return (x + 255) & ~uint64_t(255); }

// Layout of `scratch` (byte offsets).  The node stores take what is left
// after the tables: kNoAllocNodeCap nodes per workgroup.
constexpr uint64_t kCounterOff = 0;   // one 64-bit work counter
constexpr uint64_t kCodeIdxOff = 256;
constexpr uint64_t kMOff = al256(kCodeIdxOff + 4ull * GRAND_NOALLOC_MAX_WORDS);
constexpr uint64_t kCapOff = al256(kMOff + 4ull * GRAND_NOALLOC_MAX_WORDS);
constexpr uint64_t kRxOffOff = al256(kCapOff + 8ull * GRAND_NOALLOC_MAX_WORDS);
constexpr uint64_t kJobsOff = al256(kRxOffOff + 8ull * GRAND_NOALLOC_MAX_WORDS);
constexpr uint64_t kCodesOff = al256(kJobsOff + sizeof(DevJob) * GRAND_NOALLOC_MAX_WORDS);
constexpr uint64_t kNodesOff = al256(kCodesOff + sizeof(DevCode) * GRAND_NOALLOC_MAX_CODES);
constexpr uint32_t kNoAllocNodeCap = 16384;

static_assert(kNodesOff < GRAND_NOALLOC_SCRATCH_BYTES, "scratch too small for its tables");

__device__ __align__(256) uint8_t scratch[GRAND_NOALLOC_SCRATCH_BYTES];

// Device address of `scratch` on each device (taken once, then reused).
constexpr int kMaxDevices = 64;
std::mutex g_mu;
uint8_t *g_scratch[kMaxDevices] = {};

// The code table travels as a kernel argument (at most 64 entries, 2 KiB).
struct CodeTable {
    DevCode c[GRAND_NOALLOC_MAX_CODES];
};

// Job table of a launch in the caller's order: word i writes output slot i.
__global__ void pack_jobs(const uint32_t *code_index, const uint32_t *M, const uint64_t *cap,
                          const uint64_t *rx_off, uint32_t count, uint32_t cutoff, DevJob *jobs,
                          CodeTable table, uint32_t n_codes, DevCode *codes)
{
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride)
        jobs[i] = DevJob{code_index[i], M[i], rx_off[i], cap[i], i, cutoff};
    if (blockIdx.x == 0)
        for (uint32_t c = threadIdx.x; c < n_codes; c += blockDim.x)
            codes[c] = table.c[c];
}

}  // namespace

namespace grand {
namespace host {

// Take the device address of `scratch` on the current device (once per
// device; called by grand_init and by the first no-alloc call on a device).
int noalloc_setup(int device, uint8_t **out)
{
    if (device < 0 || device >= kMaxDevices)
        return fail(GRAND_EINVAL, "device index beyond the no-alloc table");
    std::lock_guard<std::mutex> g(g_mu);
    if (!g_scratch[device]) {
        void *p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p)
            return fail(GRAND_EDEVICE, "hipGetSymbolAddress returned no address for scratch");
        g_scratch[device] = (uint8_t *)p;
    }
    if (out)
        *out = g_scratch[device];
    return GRAND_OK;
}

}  // namespace host
}  // namespace grand

extern "C" int grand_decode_batch_noalloc(const grand_batch *b, void *stream)
{
    if (!b)
        return fail(GRAND_EINVAL, "null batch");
    if (b->count == 0)
        return GRAND_OK;
    if (!b->codes || !b->code_index || !b->M || !b->query_cap || !b->noise_var ||
        !b->rx_offset || !b->rx || !b->codeword_out || !b->queries_out || !b->abandoned_out)
        return fail(GRAND_EINVAL, "null pointer in batch");
    if (b->launch_mode > GRAND_LAUNCH_BUCKETS)
        return fail(GRAND_EINVAL, "launch_mode must be GRAND_LAUNCH_AUTO, _MERGED or _BUCKETS");
    if (b->rx_count == 0)
        return fail(GRAND_EINVAL, "rx_count must give the number of floats in rx");
    if (b->count > GRAND_NOALLOC_MAX_WORDS)
        return fail(GRAND_EINVAL, "batch larger than GRAND_NOALLOC_MAX_WORDS codewords");
    if (b->n_codes == 0 || b->n_codes > GRAND_NOALLOC_MAX_CODES)
        return fail(GRAND_EINVAL, "n_codes must be 1 .. GRAND_NOALLOC_MAX_CODES");
    DeviceCtx *ctx;
    int rc = current_ctx(&ctx);
    if (rc)
        return rc;
    CodeTable table;
    for (uint32_t c = 0; c < b->n_codes; c++) {
        const grand_code *cd = b->codes[c];
        if (!cd || cd->device != ctx->device)
            return fail(GRAND_EINVAL, "null code or code on another device");
        table.c[c] = DevCode{cd->n, cd->rows, cd->kw, cd->row_w32, cd->d_rows, cd->d_cols};
    }
    // the same validation as grand_decode_batch, and the launch's LDS sizing
    uint32_t ni = 1;
    for (uint32_t i = 0; i < b->count; i++) {
        const uint32_t ci = b->code_index[i];
        if (ci >= b->n_codes)
            return fail(GRAND_EINVAL, "code index out of range");
        if (!valid_m(b->M[i]))
            return fail(GRAND_EINVAL, "invalid M");
        if (b->query_cap[i] < 1 || b->query_cap[i] > GRAND_MAX_CAP)
            return fail(GRAND_EINVAL, "query cap out of range");
        if (!std::isfinite(b->noise_var[i]) || b->noise_var[i] <= 0.0f)
            return fail(GRAND_EINVAL, "noise variance must be finite and positive");
        const uint32_t n = b->codes[ci]->n;
        const uint64_t need = 2ull * symbols(n, b->M[i]);
        if (b->rx_offset[i] > b->rx_count || b->rx_count - b->rx_offset[i] < need)
            return fail(GRAND_EINVAL, "word " + std::to_string(i) +
                                          ": received values past rx_count");
        ni = std::max(ni, items_pow2(n, b->M[i]));
    }
    uint8_t *base = nullptr;
    if ((rc = noalloc_setup(ctx->device, &base)))
        return rc;
    grand_tuning t = tuning_for(0, 0);
    t.node_cap = kNoAllocNodeCap;
    const uint64_t slot = node_bytes(t.node_cap);
    const uint64_t slots = (GRAND_NOALLOC_SCRATCH_BYTES - kNodesOff) / slot;
    uint32_t grid = std::min<uint32_t>(b->count, t.grid_per_cu * (uint32_t)ctx->cus);
    grid = (uint32_t)std::min<uint64_t>(grid, slots);
    hipStream_t st = (hipStream_t)stream;
    const size_t cnt = b->count;
    // the caller's host arrays are read during this call only: copies from
    // unpinned memory complete before they return, and the synchronisation
    // covers pinned arrays (it adds no wait after unpinned copies, which have
    // already waited for the stream's earlier work)
    HIP_TRY(hipMemcpyAsync(base + kCodeIdxOff, b->code_index, 4 * cnt, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(base + kMOff, b->M, 4 * cnt, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(base + kCapOff, b->query_cap, 8 * cnt, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(base + kRxOffOff, b->rx_offset, 8 * cnt, hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
    DevJob *jobs = (DevJob *)(base + kJobsOff);
    DevCode *codes = (DevCode *)(base + kCodesOff);
    hipLaunchKernelGGL(pack_jobs, dim3((uint32_t)std::min<size_t>((cnt + 255) / 256, 1024)),
                       dim3(256), 0, st, (const uint32_t *)(base + kCodeIdxOff),
                       (const uint32_t *)(base + kMOff), (const uint64_t *)(base + kCapOff),
                       (const uint64_t *)(base + kRxOffOff), (uint32_t)cnt, b->cutoff_symbols, jobs,
                       table, b->n_codes, codes);
    if (hipGetLastError() != hipSuccess)
        return fail(GRAND_EDEVICE, "job table kernel launch failed");
    // the work counter starts at zero for every call (a fill kernel)
    unsigned long long *counter = (unsigned long long *)(base + kCounterOff);
    if (launch_zero(counter, 1, st))
        return fail(GRAND_EDEVICE, "counter reset launch failed");
    KernelArgs a;
    a.codes = codes;
    a.jobs = jobs;
    a.njobs = (uint32_t)cnt;
    a.low_bits = t.low_bits;
    a.first_band = t.first_band;
    a.band_growth = t.band_growth;
    a.node_cap = t.node_cap;
    a.ni = ni;
    a.rx = b->rx;
    a.cw_out = b->codeword_out;
    a.q_out = b->queries_out;
    a.ab_out = b->abandoned_out;
    a.status_out = b->status_out;
    a.checks_out = b->checks_out;
    a.queue = counter;
    a.qbase = 0;
    a.scratch = base + kNodesOff;
    a.done_out = nullptr;
    a.done_seq = 0;
    a.pad2 = 0;
    if (launch_decode(a, grid, t.block, st))
        return fail(GRAND_EDEVICE, std::string("decode kernel launch failed: ") +
                                       hipGetErrorString(hipGetLastError()));
    return GRAND_OK;
}
