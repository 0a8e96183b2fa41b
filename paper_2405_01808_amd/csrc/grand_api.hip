// grand_api.hip -- host runtime behind include/grand.h: code handles, launch
// planning (bucketing by (n, M) with per-bucket tuning), staging buffers,
// argument validation and error reporting.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "grand_host.h"

using namespace grand;
using namespace grand::host;

namespace grand {
namespace host {

thread_local std::string g_last_error;

int fail(int code, const std::string &msg)
{
    g_last_error = msg;
    return code;
}

bool valid_m(uint32_t M)
{
    for (int m = 1; m <= 6; m++)
        if (M == (1u << (2 * m)))
            return true;
    return false;
}

uint32_t bits_per_axis(uint32_t M)
{
    uint32_t m = 0;
    while ((1u << (2 * (m + 1))) <= M)
        m++;
    return m;
}

uint32_t symbols(uint32_t n, uint32_t M)
{
    uint32_t m = bits_per_axis(M);
    return (n + 2 * m - 1) / (2 * m);
}

// ---------------------------------------------------------------- tuning
std::mutex g_tune_mu;
std::map<std::pair<uint32_t, uint32_t>, grand_tuning> g_tune;

grand_tuning builtin_tuning(uint32_t n, uint32_t M)
{
    grand_tuning t;
    // short words of low order mostly decode early, where a smaller low
    // table is cheaper to build; otherwise 2^9 entries (measured per bucket)
    t.low_bits = (n && n <= 64 && M && M <= 16) ? 8 : 9;
    t.block = 256;
    t.first_band = 256;
    t.band_growth = 4;
    t.node_cap = 1u << 16;
    t.grid_per_cu = 8;
    return t;
}

bool same_tuning(const grand_tuning &a, const grand_tuning &b)
{
    return a.low_bits == b.low_bits && a.block == b.block && a.first_band == b.first_band &&
           a.band_growth == b.band_growth && a.node_cap == b.node_cap &&
           a.grid_per_cu == b.grid_per_cu;
}

grand_tuning tuning_for(uint32_t n, uint32_t M)
{
    std::lock_guard<std::mutex> g(g_tune_mu);
    for (auto key : {std::make_pair(n, M), std::make_pair(n, 0u), std::make_pair(0u, M),
                     std::make_pair(0u, 0u)}) {
        auto it = g_tune.find(key);
        if (it != g_tune.end())
            return it->second;
    }
    return builtin_tuning(n, M);
}

// LDS available to one workgroup on gfx950.
constexpr uint32_t kLdsPerWorkgroup = 160u * 1024u;

bool valid_tuning(const grand_tuning &t)
{
    if (t.low_bits > kMaxLowBits || t.block < 64 || t.block > kMaxBlock || t.block % 64 ||
        t.first_band < 1 || t.band_growth < 2 || t.band_growth > 64 || t.node_cap < 64 ||
        t.node_cap > (1u << 21) || t.grid_per_cu < 1 || t.grid_per_cu > 32)
        return false;
    if ((1u << t.low_bits) > kMergePer * t.block)   // merge outputs per thread
        return false;
    // largest launch: 2L = 1024 flips
    return 4ull * lds_layout(kMaxItems, t.block, t.low_bits).words + 256 <= kLdsPerWorkgroup;
}

// ---------------------------------------------------------------- device context
std::mutex g_ctx_mu;
std::map<int, std::unique_ptr<DeviceCtx>> g_ctx;

int current_ctx(DeviceCtx **out)
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> g(g_ctx_mu);
    auto it = g_ctx.find(dev);
    if (it == g_ctx.end()) {
        auto c = std::make_unique<DeviceCtx>();
        c->device = dev;
        hipDeviceProp_t prop;
        HIP_TRY(hipGetDeviceProperties(&prop, dev));
        c->cus = prop.multiProcessorCount;
        HIP_TRY(hipStreamCreateWithFlags(&c->own_stream, hipStreamNonBlocking));
        it = g_ctx.emplace(dev, std::move(c)).first;
    }
    *out = it->second.get();
    return GRAND_OK;
}

template <typename T>
int ensure_device(T **p, size_t *cap, size_t want)
{
    if (*cap >= want && *p)
        return GRAND_OK;
    if (*p)
        HIP_TRY(hipFree(*p));
    *p = nullptr;
    *cap = 0;
    size_t n = std::max<size_t>(want, 64);
    if (hipMalloc((void **)p, n * sizeof(T)) != hipSuccess)
        return fail(GRAND_ENOMEM, "hipMalloc failed for device buffer");
    *cap = n;
    return GRAND_OK;
}

template <typename T>
int ensure_pinned(T **p, size_t *cap, size_t want)
{
    if (*cap >= want && *p)
        return GRAND_OK;
    if (*p)
        HIP_TRY(hipHostFree(*p));
    *p = nullptr;
    *cap = 0;
    size_t n = std::max<size_t>(want, 64);
    if (hipHostMalloc((void **)p, n * sizeof(T), hipHostMallocDefault) != hipSuccess)
        return fail(GRAND_ENOMEM, "hipHostMalloc failed for staging buffer");
    *cap = n;
    return GRAND_OK;
}

int init_stream_res(StreamRes &r)
{
    if (!r.queues) {
        if (hipMalloc((void **)&r.queues, 64 * sizeof(unsigned long long)) != hipSuccess)
            return fail(GRAND_ENOMEM, "hipMalloc failed for work counters");
        HIP_TRY(hipMemset(r.queues, 0, 64 * sizeof(unsigned long long)));
        HIP_TRY(hipEventCreateWithFlags(&r.staged, hipEventDisableTiming));
        if (hipMalloc((void **)&r.d_rx, 2 * kMaxItems * sizeof(float)) != hipSuccess ||
            hipMalloc((void **)&r.d_out, (kCwStride + 2) * sizeof(uint64_t)) != hipSuccess ||
            hipMalloc((void **)&r.d_ab, 64) != hipSuccess ||
            hipMalloc((void **)&r.d_status, 64) != hipSuccess)
            return fail(GRAND_ENOMEM, "hipMalloc failed for single-decode buffers");
        if (hipHostMalloc((void **)&r.h_rx, 2 * kMaxItems * sizeof(float), hipHostMallocDefault) !=
                hipSuccess ||
            hipHostMalloc((void **)&r.h_out, (kCwStride + 2) * sizeof(uint64_t),
                          hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc((void **)&r.h_ab, 64, hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc((void **)&r.h_status, 64, hipHostMallocDefault) != hipSuccess)
            return fail(GRAND_ENOMEM, "hipHostMalloc failed for single-decode buffers");
    }
    return GRAND_OK;
}

int stream_res(DeviceCtx *ctx, void *stream, StreamRes **out)
{
    StreamRes &r = ctx->res[stream];
    int rc = init_stream_res(r);
    if (rc)
        return rc;
    *out = &r;
    return GRAND_OK;
}

int ensure_scratch(StreamRes &r, size_t bytes)
{
    if (r.scratch_bytes >= bytes && r.scratch)
        return GRAND_OK;
    if (r.scratch) {
        // earlier launches on any stream may still use the old buffer
        HIP_TRY(hipDeviceSynchronize());
        HIP_TRY(hipFree(r.scratch));
    }
    r.scratch = nullptr;
    r.scratch_bytes = 0;
    if (hipMalloc((void **)&r.scratch, bytes) != hipSuccess)
        return fail(GRAND_ENOMEM, "hipMalloc failed for the high-subset stores (" +
                                      std::to_string(bytes) + " bytes)");
    r.scratch_bytes = bytes;
    return GRAND_OK;
}

struct Bucket {
    uint32_t n, M;
    grand_tuning t;
    std::vector<uint32_t> words;
    uint32_t ni = 0;   // LDS sizing: next_pow2(2L) of the bucket's largest word
};

// Where a group of launches runs: staged tables, work counters and stores.
struct LaunchTarget {
    const DevCode *codes;
    const DevJob *jobs;
    unsigned long long *queues;   // one counter per bucket (index mod 64)
    uint64_t *qnext;              // counter values at launch, or null: zero each
                                  // counter in the stream before its launch
    uint8_t *scratch;
};

// Launch shapes for buckets that keep the built-in tuning (256 threads, 8
// per CU, of which 7 are resident).  Only the shape changes, never a result.
//   - No more words than compute units leaves most of each CU idle: one
//     1024-thread workgroup (16 waves) per word.  (Measured at N = 128:
//     faster up to one word per CU, equal at 1.5, slower from 2.)
//   - Long words (n >= 256) filling at most two rounds of the resident
//     narrow slots: 512-thread workgroups, 3 per CU.  A narrow launch there
//     ends in a half-empty second round (cfg4's 2048 words: 1.71 instead of
//     2.36 ms); beyond two rounds 256 threads win again (16384 words).
// A symbol cut-off of at most 32 symbols leaves at most 64 flips per word,
// too little work for wide workgroups.
void shape_small(DeviceCtx *ctx, std::vector<Bucket> &buckets, uint32_t cutoff)
{
    if (cutoff != 0 && cutoff <= 32)
        return;
    const size_t cus = (size_t)ctx->cus;
    for (auto &bk : buckets) {
        if (!same_tuning(bk.t, builtin_tuning(bk.n, bk.M)) && bk.t.block != 256)
            continue;
        const uint32_t ni = bk.ni ? bk.ni : items_pow2(bk.n, bk.M);
        auto fits = [&](uint32_t block) {
            return 4ull * lds_layout(ni, block, bk.t.low_bits).words + 256 <= kLdsPerWorkgroup &&
                   (1u << bk.t.low_bits) <= kMergePer * block;
        };
        const size_t words = bk.words.size();
        if (words <= cus && fits(kMaxBlock)) {
            bk.t.block = kMaxBlock;
        } else if (bk.n >= 256 && words <= 14 * cus && same_tuning(bk.t, builtin_tuning(bk.n, bk.M)) &&
                   fits(512)) {
            bk.t.block = 512;
            bk.t.grid_per_cu = 3;
        }
    }
}

// Workgroups per launch of each bucket and the store bytes they need.
size_t bucket_grids(DeviceCtx *ctx, const std::vector<Bucket> &buckets, std::vector<uint32_t> &grids)
{
    grids.assign(buckets.size(), 1);
    size_t need = 0;
    for (size_t i = 0; i < buckets.size(); i++) {
        const grand_tuning &t = buckets[i].t;
        uint32_t g = std::min<uint32_t>((uint32_t)buckets[i].words.size(),
                                        t.grid_per_cu * (uint32_t)ctx->cus);
        grids[i] = std::max(1u, g);
        need = std::max<size_t>(need, (size_t)grids[i] * node_bytes(t.node_cap));
    }
    return need;
}

// Enqueue one launch per bucket; jobs/codes already staged in device memory.
int enqueue_buckets(const LaunchTarget &lt, const std::vector<Bucket> &buckets,
                    const std::vector<uint32_t> &grids, const std::vector<uint32_t> &job_base,
                    const float *rx, uint64_t *cw_out, uint64_t *q_out, uint8_t *ab_out,
                    int32_t *status_out, uint64_t *checks_out, void *stream)
{
    for (size_t i = 0; i < buckets.size(); i++) {
        const grand_tuning &t = buckets[i].t;
        KernelArgs a;
        a.codes = lt.codes;
        a.jobs = lt.jobs + job_base[i];
        a.njobs = (uint32_t)buckets[i].words.size();
        a.low_bits = t.low_bits;
        a.first_band = t.first_band;
        a.band_growth = t.band_growth;
        a.node_cap = t.node_cap;
        a.ni = buckets[i].ni ? buckets[i].ni : items_pow2(buckets[i].n, buckets[i].M);
        a.rx = rx;
        a.cw_out = cw_out;
        a.q_out = q_out;
        a.ab_out = ab_out;
        a.status_out = status_out;
        a.checks_out = checks_out;
        a.queue = lt.queues + (i % 64);
        a.qbase = lt.qnext ? lt.qnext[i % 64] : 0;
        a.scratch = lt.scratch;
        a.done_out = nullptr;
        a.done_seq = 0;
        a.pad2 = 0;
        if (!lt.qnext && launch_zero(a.queue, 1, stream))
            return fail(GRAND_EDEVICE, "counter reset launch failed");
        if (launch_decode(a, grids[i], t.block, stream))
            return fail(GRAND_EDEVICE, std::string("decode kernel launch failed: ") +
                                           hipGetErrorString(hipGetLastError()));
        if (lt.qnext)
            lt.qnext[i % 64] += a.njobs + grids[i];
    }
    return GRAND_OK;
}

// Validate a batch and group its words into launches ("buckets"), each in
// the order its workgroups should take them.
int plan_batch(DeviceCtx *ctx, const grand_batch *b, std::vector<Bucket> &buckets)
{
    if (!b)
        return fail(GRAND_EINVAL, "null batch");
    if (!b->codes || !b->code_index || !b->M || !b->query_cap || !b->noise_var ||
        !b->rx_offset || !b->rx || !b->codeword_out || !b->queries_out || !b->abandoned_out)
        return fail(GRAND_EINVAL, "null pointer in batch");
    if (b->launch_mode > GRAND_LAUNCH_BUCKETS)
        return fail(GRAND_EINVAL, "launch_mode must be GRAND_LAUNCH_AUTO, _MERGED or _BUCKETS");
    if (b->rx_count == 0)
        return fail(GRAND_EINVAL, "rx_count must give the number of floats in rx");
    if (b->n_codes == 0)
        return fail(GRAND_EINVAL, "no codes");
    for (uint32_t c = 0; c < b->n_codes; c++)
        if (!b->codes[c] || b->codes[c]->device != ctx->device)
            return fail(GRAND_EINVAL, "null code or code on another device");
    std::map<std::pair<uint32_t, uint32_t>, size_t> index;
    buckets.clear();
    std::pair<uint32_t, uint32_t> last_key{0, 0};   // words usually come in runs of one (n, M)
    size_t last = SIZE_MAX;
    for (uint32_t i = 0; i < b->count; i++) {
        uint32_t ci = b->code_index[i];
        if (ci >= b->n_codes)
            return fail(GRAND_EINVAL, "code index out of range");
        if (!valid_m(b->M[i]))
            return fail(GRAND_EINVAL, "invalid M");
        if (b->query_cap[i] < 1 || b->query_cap[i] > GRAND_MAX_CAP)
            return fail(GRAND_EINVAL, "query cap out of range");
        if (!std::isfinite(b->noise_var[i]) || b->noise_var[i] <= 0.0f)
            return fail(GRAND_EINVAL, "noise variance must be finite and positive");
        // the kernel reads 2L floats from rx_offset on: they must lie in rx
        const uint64_t need = 2ull * symbols(b->codes[ci]->n, b->M[i]);
        if (b->rx_offset[i] > b->rx_count || b->rx_count - b->rx_offset[i] < need)
            return fail(GRAND_EINVAL, "word " + std::to_string(i) +
                                          ": received values past rx_count");
        auto key = std::make_pair(b->codes[ci]->n, b->M[i]);
        if (last == SIZE_MAX || key != last_key) {
            auto it = index.find(key);
            if (it == index.end()) {
                it = index.emplace(key, buckets.size()).first;
                buckets.push_back(
                    Bucket{key.first, key.second, tuning_for(key.first, key.second), {}});
            }
            last_key = key;
            last = it->second;
        }
        buckets[last].words.push_back(i);
    }
    bool merged = false;
    int mixed = b->launch_mode == GRAND_LAUNCH_MERGED ? 1
                : b->launch_mode == GRAND_LAUNCH_BUCKETS ? 0 : -1;
    // One launch for the whole batch when asked, or when no (n, M) bucket
    // fills the device on its own: words of every size share the persistent
    // workgroups (LDS sized for the largest), heaviest first.
    if (buckets.size() > 1) {
        size_t biggest = 0;
        for (auto &bk : buckets)
            biggest = std::max(biggest, bk.words.size());
        if (mixed < 0)
            mixed = biggest < (size_t)tuning_for(0, 0).grid_per_cu * ctx->cus;
        if (mixed) {
            Bucket all{0, 0, tuning_for(0, 0), {}};
            for (auto &bk : buckets) {
                all.ni = std::max(all.ni, items_pow2(bk.n, bk.M));
                all.n = std::max(all.n, bk.n);
                all.words.insert(all.words.end(), bk.words.begin(), bk.words.end());
            }
            std::stable_sort(all.words.begin(), all.words.end(), [&](uint32_t x, uint32_t y) {
                const grand_code *cx = b->codes[b->code_index[x]], *cy = b->codes[b->code_index[y]];
                uint32_t wx = items_pow2(cx->n, b->M[x]), wy = items_pow2(cy->n, b->M[y]);
                if (wx != wy)
                    return wx > wy;
                return b->query_cap[x] > b->query_cap[y];
            });
            buckets.assign(1, all);
            merged = true;
        }
    }
    // Within a launch the workgroups take words in table order: larger caps
    // (longer decodes) start first.  Only the schedule changes, never a
    // result.  (Ordering by channel noise as well was measured slower: it
    // starts every noisy word at once.)
    if (!merged) {
        auto longer = [&](uint32_t x, uint32_t y) { return b->query_cap[x] > b->query_cap[y]; };
        for (auto &bk : buckets)
            if (!std::is_sorted(bk.words.begin(), bk.words.end(), longer))   // e.g. one cap
                std::stable_sort(bk.words.begin(), bk.words.end(), longer);
    }
    shape_small(ctx, buckets, b->cutoff_symbols);
    return GRAND_OK;
}

// Job and code tables of a planned batch, jobs in bucket order.
void fill_tables(const grand_batch *b, const std::vector<Bucket> &buckets, DevJob *jobs,
                 DevCode *codes, std::vector<uint32_t> &job_base)
{
    for (uint32_t c = 0; c < b->n_codes; c++) {
        const grand_code *cd = b->codes[c];
        codes[c] = DevCode{cd->n, cd->rows, cd->kw, cd->row_w32, cd->d_rows, cd->d_cols};
    }
    job_base.clear();
    uint32_t k = 0;
    for (auto &bk : buckets) {
        job_base.push_back(k);
        for (uint32_t i : bk.words)
            jobs[k++] = DevJob{b->code_index[i], b->M[i], b->rx_offset[i], b->query_cap[i], i,
                               b->cutoff_symbols};
    }
}

// Validate a batch, bucket it by (n, M), stage its jobs and enqueue the
// launches on `stream` using the buffers of `r`.
int decode_batch_on(DeviceCtx *ctx, StreamRes &r, const grand_batch *b, void *stream)
{
    if (b && b->count == 0)
        return GRAND_OK;
    std::vector<Bucket> buckets;
    int rc = plan_batch(ctx, b, buckets);
    if (rc)
        return rc;
    rc = init_stream_res(r);
    if (rc)
        return rc;
    if (r.staged_pending) {
        HIP_TRY(hipEventSynchronize(r.staged));
        r.staged_pending = false;
    }
    rc = ensure_device(&r.codes, &r.codes_cap, b->n_codes);
    if (!rc)
        rc = ensure_device(&r.jobs, &r.jobs_cap, b->count);
    if (!rc)
        rc = ensure_pinned(&r.h_codes, &r.h_codes_cap, b->n_codes);
    if (!rc)
        rc = ensure_pinned(&r.h_jobs, &r.h_jobs_cap, b->count);
    if (rc)
        return rc;
    std::vector<uint32_t> job_base;
    fill_tables(b, buckets, r.h_jobs, r.h_codes, job_base);
    hipStream_t st = (hipStream_t)stream;
    // The device tables of this stream still hold the last upload (launches
    // only read them), so a batch with the same tables, such as a plan
    // launched again, skips the upload and the copy kernel it costs.
    const size_t nj = b->count, nc = b->n_codes;
    const bool resident = r.up_valid && r.up_jobs.size() == nj && r.up_codes.size() == nc &&
                          !std::memcmp(r.up_jobs.data(), r.h_jobs, nj * sizeof(DevJob)) &&
                          !std::memcmp(r.up_codes.data(), r.h_codes, nc * sizeof(DevCode));
    if (!resident) {
        r.up_valid = false;
        HIP_TRY(hipMemcpyAsync(r.codes, r.h_codes, nc * sizeof(DevCode), hipMemcpyHostToDevice,
                               st));
        HIP_TRY(hipMemcpyAsync(r.jobs, r.h_jobs, nj * sizeof(DevJob), hipMemcpyHostToDevice,
                               st));
        HIP_TRY(hipEventRecord(r.staged, st));
        r.staged_pending = true;
        r.up_jobs.assign(r.h_jobs, r.h_jobs + nj);
        r.up_codes.assign(r.h_codes, r.h_codes + nc);
        r.up_valid = true;
    }
    std::vector<uint32_t> grids;
    rc = ensure_scratch(r, bucket_grids(ctx, buckets, grids));
    if (rc)
        return rc;
    const LaunchTarget lt{r.codes, r.jobs, r.queues, r.qnext, r.scratch};
    return enqueue_buckets(lt, buckets, grids, job_base, b->rx, b->codeword_out, b->queries_out,
                           b->abandoned_out, b->status_out, b->checks_out, stream);
}

}  // namespace host
}  // namespace grand

// ==================================================================== ABI

extern "C" {

const char *grand_strerror(int err)
{
    switch (err) {
    case GRAND_OK: return "success";
    case GRAND_EINVAL: return "invalid argument";
    case GRAND_ENOMEM: return "out of memory";
    case GRAND_EDEVICE: return "HIP device error";
    case GRAND_EBUSY: return "server busy (admission refused)";
    case GRAND_ECAPACITY: return "high-subset store capacity exceeded";
    case GRAND_ENOTFOUND: return "not found";
    default: return "unknown error";
    }
}

const char *grand_last_error(void) { return g_last_error.c_str(); }

int grand_init(int device)
{
    int count = 0;
    HIP_TRY(hipGetDeviceCount(&count));
    if (device < 0 || device >= count)
        return fail(GRAND_EINVAL, "no such device");
    HIP_TRY(hipSetDevice(device));
    DeviceCtx *ctx;
    int rc = current_ctx(&ctx);
    if (rc)
        return rc;
    return noalloc_setup(device, nullptr);
}

int grand_code_create(uint32_t n, uint32_t rows, const uint64_t *h_rows, grand_code **out)
{
    if (!h_rows || !out)
        return fail(GRAND_EINVAL, "null pointer");
    if (n < 2 || n > kMaxN || (n & (n - 1)))
        return fail(GRAND_EINVAL, "n must be a power of two in [2, 1024]");
    if (rows < 1 || rows >= n || rows > 32 * kMaxKW)
        return fail(GRAND_EINVAL, "rows must satisfy 1 <= rows < n and rows <= 512");
    const uint32_t w64 = (n + 63) / 64;
    for (uint32_t i = 0; i < rows; i++)
        if (n % 64 && (h_rows[(size_t)i * w64 + w64 - 1] >> (n % 64)))
            return fail(GRAND_EINVAL, "bits beyond n set in h_rows");
    DeviceCtx *ctx;
    int rc = current_ctx(&ctx);
    if (rc)
        return rc;
    auto *c = new (std::nothrow) grand_code;
    if (!c)
        return fail(GRAND_ENOMEM, "host allocation failed");
    c->n = n;
    c->rows = rows;
    c->kw = (rows + 31) / 32;
    c->row_w32 = 2 * w64;
    c->device = ctx->device;
    std::vector<uint32_t> cols((size_t)n * c->kw, 0);
    for (uint32_t i = 0; i < rows; i++)
        for (uint32_t j = 0; j < n; j++)
            if ((h_rows[(size_t)i * w64 + j / 64] >> (j % 64)) & 1ull)
                cols[(size_t)j * c->kw + i / 32] |= 1u << (i % 32);
    c->d_rows = nullptr;
    c->d_cols = nullptr;
    if (hipMalloc((void **)&c->d_rows, (size_t)rows * w64 * 8) != hipSuccess ||
        hipMalloc((void **)&c->d_cols, cols.size() * 4) != hipSuccess) {
        if (c->d_rows)
            (void)hipFree(c->d_rows);
        delete c;
        return fail(GRAND_ENOMEM, "hipMalloc failed for code");
    }
    if (hipMemcpy(c->d_rows, h_rows, (size_t)rows * w64 * 8, hipMemcpyHostToDevice) !=
            hipSuccess ||
        hipMemcpy(c->d_cols, cols.data(), cols.size() * 4, hipMemcpyHostToDevice) !=
            hipSuccess) {
        (void)hipFree(c->d_rows);
        (void)hipFree(c->d_cols);
        delete c;
        return fail(GRAND_EDEVICE, "copy of H to the device failed");
    }
    *out = c;
    return GRAND_OK;
}

void grand_code_destroy(grand_code *code)
{
    if (!code)
        return;
    (void)hipDeviceSynchronize();
    (void)hipFree(code->d_rows);
    (void)hipFree(code->d_cols);
    delete code;
}

uint32_t grand_code_n(const grand_code *code) { return code ? code->n : 0; }
uint32_t grand_code_rows(const grand_code *code) { return code ? code->rows : 0; }

int grand_tuning_get(uint32_t n, uint32_t M, grand_tuning *out)
{
    if (!out)
        return fail(GRAND_EINVAL, "null pointer");
    *out = tuning_for(n, M);
    return GRAND_OK;
}

int grand_tuning_set(uint32_t n, uint32_t M, const grand_tuning *t)
{
    if (!t || !valid_tuning(*t))
        return fail(GRAND_EINVAL, "invalid tuning");
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_tune[std::make_pair(n, M)] = *t;
    return GRAND_OK;
}

int grand_decode(const grand_code *code, const float *rx, uint32_t M, float noise_var,
                 uint64_t query_cap, uint64_t *codeword_out, uint64_t *queries_out,
                 uint8_t *abandoned_out)
{
    return grand_decode_ex(code, rx, M, noise_var, query_cap, 0, codeword_out, queries_out,
                           abandoned_out);
}

int grand_decode_ex(const grand_code *code, const float *rx, uint32_t M, float noise_var,
                    uint64_t query_cap, uint32_t cutoff_symbols, uint64_t *codeword_out,
                    uint64_t *queries_out, uint8_t *abandoned_out)
{
    if (!code || !rx || !codeword_out || !queries_out || !abandoned_out)
        return fail(GRAND_EINVAL, "null pointer");
    if (!valid_m(M))
        return fail(GRAND_EINVAL, "M must be 4, 16, 64, 256, 1024 or 4096");
    if (query_cap < 1 || query_cap > GRAND_MAX_CAP)
        return fail(GRAND_EINVAL, "query cap out of range");
    if (!std::isfinite(noise_var) || noise_var <= 0.0f)
        return fail(GRAND_EINVAL, "noise variance must be finite and positive");
    const uint32_t L = symbols(code->n, M);
    for (uint32_t i = 0; i < 2 * L; i++)
        if (!std::isfinite(rx[i]) || std::fabs(rx[i]) > 32768.0f)
            return fail(GRAND_EINVAL, "received value not finite or beyond 2^15");
    DeviceCtx *ctx;
    int rc = current_ctx(&ctx);
    if (rc)
        return rc;
    if (code->device != ctx->device)
        return fail(GRAND_EINVAL, "code was created on another device");
    std::lock_guard<std::mutex> g(ctx->mu);
    StreamRes *r;
    rc = stream_res(ctx, (void *)ctx->own_stream, &r);   // private to this path
    if (rc)
        return rc;
    hipStream_t st = ctx->own_stream;
    if (r->staged_pending) {
        HIP_TRY(hipEventSynchronize(r->staged));
        r->staged_pending = false;
    }
    rc = ensure_device(&r->codes, &r->codes_cap, 1);
    if (!rc)
        rc = ensure_device(&r->jobs, &r->jobs_cap, 1);
    if (!rc)
        rc = ensure_pinned(&r->h_codes, &r->h_codes_cap, 1);
    if (!rc)
        rc = ensure_pinned(&r->h_jobs, &r->h_jobs_cap, 1);
    if (rc)
        return rc;
    r->h_codes[0] = DevCode{code->n, code->rows, code->kw, code->row_w32, code->d_rows,
                            code->d_cols};
    r->h_jobs[0] = DevJob{0, M, 0, query_cap, 0, cutoff_symbols};
    r->up_valid = false;
    std::memcpy(r->h_rx, rx, 2 * L * sizeof(float));
    HIP_TRY(hipMemcpyAsync(r->codes, r->h_codes, sizeof(DevCode), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(r->jobs, r->h_jobs, sizeof(DevJob), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(r->d_rx, r->h_rx, 2 * L * sizeof(float), hipMemcpyHostToDevice, st));
    std::vector<Bucket> buckets{Bucket{code->n, M, tuning_for(code->n, M), {0}}};
    shape_small(ctx, buckets, cutoff_symbols);
    buckets[0].t.grid_per_cu = 1;
    std::vector<uint32_t> base{0}, grids;
    rc = ensure_scratch(*r, bucket_grids(ctx, buckets, grids));
    if (rc)
        return rc;
    const LaunchTarget lt{r->codes, r->jobs, r->queues, r->qnext, r->scratch};
    rc = enqueue_buckets(lt, buckets, grids, base, r->d_rx, r->d_out, r->d_out + kCwStride,
                         r->d_ab, r->d_status, r->d_out + kCwStride + 1, st);
    if (rc)
        return rc;
    HIP_TRY(hipMemcpyAsync(r->h_out, r->d_out, (kCwStride + 2) * sizeof(uint64_t),
                           hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(r->h_ab, r->d_ab, 1, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(r->h_status, r->d_status, 4, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (r->h_status[0] != GRAND_OK)
        return fail(r->h_status[0], "device decode failed: " +
                                        std::string(grand_strerror(r->h_status[0])));
    const uint32_t w64 = (code->n + 63) / 64;
    std::memcpy(codeword_out, r->h_out, w64 * sizeof(uint64_t));
    *queries_out = r->h_out[kCwStride];
    *abandoned_out = r->h_ab[0];
    return GRAND_OK;
}

// ---------------------------------------------------------------- graphs

struct grand_graph {
    int device = -1;
    DevJob *jobs = nullptr;
    DevCode *codes = nullptr;
    unsigned long long *queues = nullptr;
    uint8_t *scratch = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

void grand_graph_destroy(grand_graph *g)
{
    if (!g)
        return;
    if (g->exec)
        (void)hipGraphExecDestroy(g->exec);
    if (g->graph)
        (void)hipGraphDestroy(g->graph);
    (void)hipFree(g->jobs);
    (void)hipFree(g->codes);
    (void)hipFree(g->queues);
    (void)hipFree(g->scratch);
    delete g;
}

int grand_graph_create(const grand_batch *b, grand_graph **out)
{
    if (!b || !out)
        return fail(GRAND_EINVAL, "null pointer");
    if (b->count == 0)
        return fail(GRAND_EINVAL, "empty batch");
    DeviceCtx *ctx;
    int rc = current_ctx(&ctx);
    if (rc)
        return rc;
    std::vector<Bucket> buckets;
    rc = plan_batch(ctx, b, buckets);
    if (rc)
        return rc;
    std::vector<DevJob> jobs(b->count);
    std::vector<DevCode> codes(b->n_codes);
    std::vector<uint32_t> job_base, grids;
    fill_tables(b, buckets, jobs.data(), codes.data(), job_base);
    const size_t need = bucket_grids(ctx, buckets, grids);
    auto g = new grand_graph;
    g->device = ctx->device;
    hipStream_t cs = nullptr;
    auto bail = [&](int code) {
        if (cs)
            (void)hipStreamDestroy(cs);
        grand_graph_destroy(g);
        return code;
    };
    const uint32_t nq = (uint32_t)std::min<size_t>(buckets.size(), 64);
    if (hipMalloc((void **)&g->jobs, jobs.size() * sizeof(DevJob)) != hipSuccess ||
        hipMalloc((void **)&g->codes, codes.size() * sizeof(DevCode)) != hipSuccess ||
        hipMalloc((void **)&g->queues, nq * sizeof(unsigned long long)) != hipSuccess ||
        hipMalloc((void **)&g->scratch, std::max<size_t>(need, 256)) != hipSuccess)
        return bail(fail(GRAND_ENOMEM, "hipMalloc failed for a batch graph"));
    if (hipMemcpy(g->jobs, jobs.data(), jobs.size() * sizeof(DevJob), hipMemcpyHostToDevice) !=
            hipSuccess ||
        hipMemcpy(g->codes, codes.data(), codes.size() * sizeof(DevCode),
                  hipMemcpyHostToDevice) != hipSuccess ||
        hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess)
        return bail(fail(GRAND_EDEVICE, "staging a batch graph failed"));
    // every launch zeroes its counter first (a fill kernel, not a memset
    // node), so each replay starts from the same state
    const LaunchTarget lt{g->codes, g->jobs, g->queues, nullptr, g->scratch};
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed) != hipSuccess)
        return bail(fail(GRAND_EDEVICE, "hipStreamBeginCapture failed"));
    rc = enqueue_buckets(lt, buckets, grids, job_base, b->rx, b->codeword_out, b->queries_out,
                         b->abandoned_out, b->status_out, b->checks_out, cs);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(cs, &graph);
    g->graph = graph;
    if (rc)
        return bail(rc);
    if (e != hipSuccess || !graph)
        return bail(fail(GRAND_EDEVICE, std::string("hipStreamEndCapture: ") +
                                            hipGetErrorString(e)));
    if (hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0) != hipSuccess)
        return bail(fail(GRAND_EDEVICE, "hipGraphInstantiate failed"));
    (void)hipStreamDestroy(cs);
    *out = g;
    return GRAND_OK;
}

int grand_graph_launch(grand_graph *g, void *stream)
{
    if (!g)
        return fail(GRAND_EINVAL, "null graph");
    HIP_TRY(hipGraphLaunch(g->exec, (hipStream_t)stream));
    return GRAND_OK;
}

int grand_decode_batch(const grand_batch *b, void *stream)
{
    if (!b)
        return fail(GRAND_EINVAL, "null batch");
    if (b->count == 0)
        return GRAND_OK;
    if (!b->codes || !b->code_index || !b->M || !b->query_cap || !b->noise_var ||
        !b->rx_offset || !b->rx || !b->codeword_out || !b->queries_out || !b->abandoned_out ||
        b->n_codes == 0)
        return fail(GRAND_EINVAL, "null pointer or no codes in batch");
    DeviceCtx *ctx;
    int rc = current_ctx(&ctx);
    if (rc)
        return rc;
    std::lock_guard<std::mutex> g(ctx->mu);
    StreamRes *r;
    rc = stream_res(ctx, stream, &r);
    if (rc)
        return rc;
    return decode_batch_on(ctx, *r, b, stream);
}

}  // extern "C"
