// grand_host.h -- host-side runtime pieces shared by grand_api.hip and
// grand_server.hip (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "grand.h"
#include "grand_internal.h"

struct grand_code {
    uint32_t n, rows, kw, row_w32;
    int device;
    uint32_t *d_rows;   // rows x row_w32
    uint32_t *d_cols;   // n x kw
};

namespace grand {
namespace host {

// Record an error message for grand_last_error() and return `code`.
int fail(int code, const std::string &msg);

#define HIP_TRY(expr)                                                                  \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess)                                                          \
            return ::grand::host::fail(GRAND_EDEVICE,                                  \
                                       std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

// Device buffers and pinned staging of one launch stream.
struct StreamRes {
    uint8_t *scratch = nullptr;     // high-subset stores, one slot per workgroup
    size_t scratch_bytes = 0;
    unsigned long long *queues = nullptr;   // 64 work counters (never reset)
    uint64_t qnext[64] = {};        // each counter's value once queued launches end
    DevJob *jobs = nullptr;
    size_t jobs_cap = 0;
    DevCode *codes = nullptr;
    size_t codes_cap = 0;
    DevJob *h_jobs = nullptr;       // pinned staging
    size_t h_jobs_cap = 0;
    DevCode *h_codes = nullptr;
    size_t h_codes_cap = 0;
    hipEvent_t staged = nullptr;
    bool staged_pending = false;
    // host copies of the tables that `jobs` and `codes` hold: a batch whose
    // tables are identical launches on them without uploading again
    std::vector<DevJob> up_jobs;
    std::vector<DevCode> up_codes;
    bool up_valid = false;
    // single-decode buffers
    float *d_rx = nullptr;
    uint64_t *d_out = nullptr;      // 16 cw words + q + checks
    uint8_t *d_ab = nullptr;
    int32_t *d_status = nullptr;
    float *h_rx = nullptr;          // pinned
    uint64_t *h_out = nullptr;      // pinned: 16 cw words, q
    uint8_t *h_ab = nullptr;
    int32_t *h_status = nullptr;
};

struct DeviceCtx {
    int device = -1;
    int cus = 0;
    std::mutex mu;
    hipStream_t own_stream = nullptr;
    std::map<void *, StreamRes> res;
};

bool valid_m(uint32_t M);
uint32_t symbols(uint32_t n, uint32_t M);
grand_tuning tuning_for(uint32_t n, uint32_t M);
int current_ctx(DeviceCtx **out);
int init_stream_res(StreamRes &r);
// Grow r's high-subset stores to `bytes` (synchronises the device when an
// existing buffer has to be replaced).
int ensure_scratch(StreamRes &r, size_t bytes);
// Plan (b->launch_mode decides merged or per-bucket launches), stage and
// enqueue a batch on `stream` with the buffers of r.
int decode_batch_on(DeviceCtx *ctx, StreamRes &r, const grand_batch *b, void *stream);

// Device address of the no-alloc entry point's static array on `device`
// (taken with hipGetSymbolAddress the first time; *out may be null).
int noalloc_setup(int device, uint8_t **out);

}  // namespace host
}  // namespace grand
