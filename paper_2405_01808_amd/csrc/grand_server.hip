// grand_server.hip -- serving of decode requests as they arrive, and
// real-time replay of recorded arrival streams (server and plain paths).
//
// Requests are admitted within a slot count and a device-memory budget.
// Each lane is one HIP stream with its own buffers in coherent pinned
// memory.  When a lane is idle, every admitted request not yet launched is
// written into its buffers and decoded as one launch, heaviest first; the
// kernel reads the requests in place and writes each result back together
// with a per-request completion flag, so a request is returned as soon as
// its own decode ends, not when its whole launch does.  The lane's stream
// event still marks the end of the launch (every result is then final), so
// a flag that is never seen delays a result but cannot lose it.  Launches
// on different lanes overlap on the device while new requests keep being
// admitted.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "grand_host.h"

using namespace grand;
using namespace grand::host;

namespace {

double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

struct Request {
    uint64_t id;
    const grand_code *code;
    uint32_t M;
    uint64_t cap;
    float noise_var;
    std::vector<float> rx;
    double arrival_s, submit_s;
    uint64_t bytes;
};

constexpr uint32_t kSlotFloats = kMaxItems;   // 2L <= N <= 1024 received values

std::atomic<uint32_t> g_fail_launches{0};     // test hook: launches to fail

struct Lane {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    StreamRes res;                    // work counters and high-subset stores
    bool busy = false;
    uint32_t cap = 0;                 // requests per launch
    uint32_t grid = 0;                // workgroups per launch at most
    uint32_t seq = 0;                 // launch number, the value of its flags
    // coherent pinned memory used by the kernel in place (host view; d_*
    // is the device's view)
    DevJob *jobs = nullptr, *d_jobs = nullptr;
    DevCode *codes = nullptr, *d_codes = nullptr;
    float *rx = nullptr, *d_rx = nullptr;
    uint64_t *cw = nullptr, *d_cw = nullptr;
    uint64_t *q = nullptr, *d_q = nullptr;
    uint64_t *chk = nullptr, *d_chk = nullptr;
    uint8_t *ab = nullptr, *d_ab = nullptr;
    int32_t *st = nullptr, *d_st = nullptr;
    uint32_t *flag = nullptr, *d_flag = nullptr;
    std::vector<Request> reqs;        // slot i of the launch
    std::vector<uint8_t> taken;       // slot already returned
    uint32_t left = 0;                // slots not yet returned
};

}  // namespace

struct grand_server {
    grand_server_config cfg;
    DeviceCtx *ctx = nullptr;
    std::mutex mu;
    std::deque<Request> pending;      // requests for the ordinary lanes
    std::deque<Request> pending_wide; // long words, for the wide lanes (if any)
    std::vector<std::unique_ptr<Lane>> lanes;
    std::deque<grand_result> done;
    uint64_t next_id = 1;
    uint64_t inflight = 0;            // admitted and not yet returned
    uint64_t running = 0;             // launched and not yet returned
    uint64_t mem_in_use = 0;
};

namespace {

template <typename T>
int coherent_alloc(T **h, size_t count, T **d)
{
    if (hipHostMalloc((void **)h, std::max<size_t>(count, 1) * sizeof(T),
                      hipHostMallocCoherent | hipHostMallocMapped) != hipSuccess) {
        *h = nullptr;
        return fail(GRAND_ENOMEM, "hipHostMalloc failed for server lane buffers");
    }
    std::memset(*h, 0, std::max<size_t>(count, 1) * sizeof(T));
    HIP_TRY(hipHostGetDevicePointer((void **)d, *h, 0));
    return GRAND_OK;
}

int lane_init(Lane &L, uint32_t cap, uint32_t grid)
{
    HIP_TRY(hipStreamCreateWithFlags(&L.stream, hipStreamNonBlocking));
    HIP_TRY(hipEventCreateWithFlags(&L.done, hipEventDisableTiming));
    L.cap = cap;
    L.grid = grid;
    int rc;
    if ((rc = coherent_alloc(&L.jobs, cap, &L.d_jobs)) ||
        (rc = coherent_alloc(&L.codes, cap, &L.d_codes)) ||
        (rc = coherent_alloc(&L.rx, (size_t)cap * kSlotFloats, &L.d_rx)) ||
        (rc = coherent_alloc(&L.cw, (size_t)cap * kCwStride, &L.d_cw)) ||
        (rc = coherent_alloc(&L.q, cap, &L.d_q)) ||
        (rc = coherent_alloc(&L.chk, cap, &L.d_chk)) ||
        (rc = coherent_alloc(&L.ab, cap, &L.d_ab)) ||
        (rc = coherent_alloc(&L.st, cap, &L.d_st)) ||
        (rc = coherent_alloc(&L.flag, cap, &L.d_flag)))
        return rc;
    if ((rc = init_stream_res(L.res)))
        return rc;
    return ensure_scratch(L.res, (size_t)grid * node_bytes(tuning_for(0, 0).node_cap));
}

void lane_free(Lane &L)
{
    if (L.stream)
        (void)hipStreamSynchronize(L.stream);
    (void)hipHostFree(L.jobs);
    (void)hipHostFree(L.codes);
    (void)hipHostFree(L.rx);
    (void)hipHostFree(L.cw);
    (void)hipHostFree(L.q);
    (void)hipHostFree(L.chk);
    (void)hipHostFree(L.ab);
    (void)hipHostFree(L.st);
    (void)hipHostFree(L.flag);
    StreamRes &r = L.res;
    (void)hipFree(r.scratch);
    (void)hipFree(r.queues);
    (void)hipFree(r.jobs);
    (void)hipFree(r.codes);
    (void)hipHostFree(r.h_jobs);
    (void)hipHostFree(r.h_codes);
    (void)hipFree(r.d_rx);
    (void)hipFree(r.d_out);
    (void)hipFree(r.d_ab);
    (void)hipFree(r.d_status);
    (void)hipHostFree(r.h_rx);
    (void)hipHostFree(r.h_out);
    (void)hipHostFree(r.h_ab);
    (void)hipHostFree(r.h_status);
    if (r.staged)
        (void)hipEventDestroy(r.staged);
    if (L.done)
        (void)hipEventDestroy(L.done);
    if (L.stream)
        (void)hipStreamDestroy(L.stream);
}

// Return slot i of a lane's launch.
void lane_emit(grand_server *s, Lane &L, uint32_t i, double t)
{
    const Request &q = L.reqs[i];
    grand_result r;
    std::memset(&r, 0, sizeof(r));
    r.request_id = q.id;
    r.status = L.st[i];
    if (r.status == GRAND_OK) {
        std::memcpy(r.codeword, L.cw + (size_t)i * kCwStride, ((q.code->n + 63) / 64) * 8);
        r.queries = L.q[i];
        r.checks = L.chk[i];
        r.abandoned = L.ab[i];
    } else {
        r.abandoned = 1;
    }
    r.arrival_s = q.arrival_s;
    r.submit_s = q.submit_s;
    r.complete_s = t;
    s->done.push_back(r);
    s->mem_in_use -= q.bytes;
    s->inflight--;
    s->running--;
    L.taken[i] = 1;
    L.left--;
}

// Move requests of `queue` (up to the lane's capacity) onto an idle lane and
// launch them, heaviest first.  A wide lane gives every request one
// 1024-thread workgroup.
int lane_launch(grand_server *s, Lane &L, std::deque<Request> &queue, bool wide)
{
    const uint32_t B = (uint32_t)std::min<size_t>(queue.size(), L.cap);
    if (B == 0)
        return GRAND_OK;
    L.reqs.clear();
    for (uint32_t i = 0; i < B; i++) {
        L.reqs.push_back(std::move(queue.front()));
        queue.pop_front();
    }
    std::stable_sort(L.reqs.begin(), L.reqs.end(), [](const Request &x, const Request &y) {
        const uint32_t wx = items_pow2(x.code->n, x.M), wy = items_pow2(y.code->n, y.M);
        if (wx != wy)
            return wx > wy;
        return x.cap > y.cap;
    });
    uint32_t ni = 1;
    for (uint32_t i = 0; i < B; i++) {
        const Request &q = L.reqs[i];
        const grand_code *c = q.code;
        L.codes[i] = DevCode{c->n, c->rows, c->kw, c->row_w32, c->d_rows, c->d_cols};
        L.jobs[i] = DevJob{i, q.M, (uint64_t)i * kSlotFloats, q.cap, i, 0};
        std::memcpy(L.rx + (size_t)i * kSlotFloats, q.rx.data(), q.rx.size() * sizeof(float));
        ni = std::max(ni, items_pow2(c->n, q.M));
    }
    grand_tuning t = tuning_for(0, 0);
    if (wide)
        t.block = kMaxBlock;
    const uint32_t grid = std::max(1u, std::min(B, L.grid));
    L.seq = L.seq + 1 ? L.seq + 1 : 1;   // flags of this launch hold seq (never 0)
    KernelArgs a;
    a.codes = L.d_codes;
    a.jobs = L.d_jobs;
    a.njobs = B;
    a.low_bits = t.low_bits;
    a.first_band = t.first_band;
    a.band_growth = t.band_growth;
    a.node_cap = t.node_cap;
    a.ni = ni;
    a.rx = L.d_rx;
    a.cw_out = L.d_cw;
    a.q_out = L.d_q;
    a.ab_out = L.d_ab;
    a.status_out = L.d_st;
    a.checks_out = L.d_chk;
    a.queue = L.res.queues;
    a.qbase = L.res.qnext[0];
    a.scratch = L.res.scratch;
    a.done_out = L.d_flag;
    a.done_seq = L.seq;
    a.pad2 = 0;
    L.taken.assign(B, 0);
    L.left = B;
    s->running += B;
    uint32_t inject = g_fail_launches.load();
    while (inject && !g_fail_launches.compare_exchange_weak(inject, inject - 1)) {
    }
    int rc = inject ? GRAND_EDEVICE
                    : (launch_decode(a, grid, t.block, L.stream) ? GRAND_EDEVICE : GRAND_OK);
    if (rc == GRAND_OK) {
        L.res.qnext[0] += B + grid;
        if (hipEventRecord(L.done, L.stream) != hipSuccess)
            rc = GRAND_EDEVICE;
    }
    if (rc) {   // return the launch as failed requests instead of losing it
        const double now = now_s();
        for (uint32_t i = 0; i < B; i++) {
            L.st[i] = rc;
            lane_emit(s, L, i, now);
        }
        L.reqs.clear();
        return fail(rc, std::string("server lane launch failed: ") +
                            hipGetErrorString(hipGetLastError()));
    }
    L.busy = true;
    return GRAND_OK;
}

// Return the lane's finished requests; all of them once its launch ended.
int lane_poll(grand_server *s, Lane &L, double t)
{
    for (uint32_t i = 0; i < (uint32_t)L.reqs.size() && L.left; i++)
        if (!L.taken[i] && __atomic_load_n(&L.flag[i], __ATOMIC_ACQUIRE) == L.seq)
            lane_emit(s, L, i, t);
    const hipError_t e = hipEventQuery(L.done);
    if (e == hipSuccess) {
        for (uint32_t i = 0; i < (uint32_t)L.reqs.size() && L.left; i++)
            if (!L.taken[i])
                lane_emit(s, L, i, t);
        L.reqs.clear();
        L.busy = false;
    } else if (e != hipErrorNotReady) {
        return fail(GRAND_EDEVICE, std::string("server lane: ") + hipGetErrorString(e));
    }
    return GRAND_OK;
}

int validate_request(const grand_code *code, const float *rx, uint32_t M, float noise_var,
                     uint64_t cap)
{
    if (!code || !rx)
        return fail(GRAND_EINVAL, "null pointer");
    if (!valid_m(M))
        return fail(GRAND_EINVAL, "M must be 4, 16, 64, 256, 1024 or 4096");
    if (cap < 1 || cap > GRAND_MAX_CAP)
        return fail(GRAND_EINVAL, "query cap out of range");
    if (!std::isfinite(noise_var) || noise_var <= 0.0f)
        return fail(GRAND_EINVAL, "noise variance must be finite and positive");
    const uint32_t L = symbols(code->n, M);
    for (uint32_t i = 0; i < 2 * L; i++)
        if (!std::isfinite(rx[i]) || std::fabs(rx[i]) > 32768.0f)
            return fail(GRAND_EINVAL, "received value not finite or beyond 2^15");
    return GRAND_OK;
}

int submit_locked(grand_server *s, const grand_code *code, const float *rx, uint32_t M,
                  float noise_var, uint64_t cap, double arrival, uint64_t *id)
{
    int rc = validate_request(code, rx, M, noise_var, cap);
    if (rc)
        return rc;
    if (code->device != s->ctx->device)
        return fail(GRAND_EINVAL, "code was created on another device");
    const uint64_t bytes = grand_request_bytes(code->n, M);
    if (s->inflight + 1 > s->cfg.max_inflight || s->mem_in_use + bytes > s->cfg.memory_budget)
        return fail(GRAND_EBUSY, "admission refused: slots or memory budget exhausted");
    Request q;
    q.id = s->next_id++;
    q.code = code;
    q.M = M;
    q.cap = cap;
    q.noise_var = noise_var;
    q.rx.assign(rx, rx + 2 * symbols(code->n, M));
    q.submit_s = now_s();
    q.arrival_s = arrival > 0 ? arrival : q.submit_s;
    q.bytes = bytes;
    std::deque<Request> &queue =
        s->cfg.wide_lanes && 2 * symbols(code->n, M) >= GRAND_WIDE_ITEMS ? s->pending_wide
                                                                         : s->pending;
    queue.push_back(std::move(q));
    s->inflight++;
    s->mem_in_use += bytes;
    if (id)
        *id = queue.back().id;
    return GRAND_OK;
}

int drain_done(grand_server *s, grand_result *out, uint32_t max_out, uint32_t *n_out)
{
    uint32_t k = 0;
    while (k < max_out && !s->done.empty()) {
        out[k++] = s->done.front();
        s->done.pop_front();
    }
    if (n_out)
        *n_out = k;
    return GRAND_OK;
}

int poll_locked(grand_server *s, grand_result *out, uint32_t max_out, uint32_t *n_out)
{
    const double t = now_s();
    for (auto &L : s->lanes) {
        if (!L->busy)
            continue;
        int rc = lane_poll(s, *L, t);
        if (rc)
            return rc;
    }
    for (size_t k = 0; k < s->lanes.size(); k++) {
        Lane &L = *s->lanes[k];
        const bool wide = k < s->cfg.wide_lanes;
        std::deque<Request> &queue = wide ? s->pending_wide : s->pending;
        if (!L.busy && !queue.empty()) {
            int rc = lane_launch(s, L, queue, wide);
            if (rc)
                return rc;
        }
    }
    return drain_done(s, out, max_out, n_out);
}

}  // namespace

extern "C" {

void grand_debug_fail_launches(uint32_t count) { g_fail_launches.store(count); }

uint64_t grand_request_bytes(uint32_t n, uint32_t M)
{
    if (n < 2 || n > kMaxN || (n & (n - 1)) || !valid_m(M))
        return 0;
    const grand_tuning t = tuning_for(n, M);
    return 2ull * symbols(n, M) * sizeof(float) + (kCwStride + 3) * 8 +
           node_bytes(t.node_cap);
}

int grand_server_create(const grand_server_config *cfg, grand_server **out)
{
    if (!cfg || !out)
        return fail(GRAND_EINVAL, "null pointer");
    if (cfg->mode == GRAND_SERVE_PERSISTENT)
        return fail(GRAND_EINVAL, "persistent serving mode is not available");
    if (cfg->max_inflight < 1 || cfg->max_inflight > (1u << 20) || cfg->memory_budget == 0 ||
        cfg->mode != GRAND_SERVE_LANES || cfg->lanes < 1 || cfg->lanes > 32 ||
        cfg->max_batch < 1 || cfg->max_batch > 65536 || cfg->wide_lanes >= cfg->lanes ||
        cfg->pad != 0)
        return fail(GRAND_EINVAL, "invalid server configuration");
    DeviceCtx *ctx;
    int rc = current_ctx(&ctx);
    if (rc)
        return rc;
    auto s = std::make_unique<grand_server>();
    s->cfg = *cfg;
    s->ctx = ctx;
    const uint32_t per_lane = std::min(cfg->max_batch, cfg->max_inflight);
    // workgroups per launch: together the lanes may hold twice the resident
    // capacity of the device
    const grand_tuning t = tuning_for(0, 0);
    const uint32_t grid = std::max(64u, 2 * t.grid_per_cu * (uint32_t)ctx->cus / cfg->lanes);
    for (uint32_t i = 0; i < cfg->lanes; i++) {
        auto L = std::make_unique<Lane>();
        rc = lane_init(*L, per_lane, grid);
        if (rc) {
            lane_free(*L);
            for (auto &x : s->lanes)
                lane_free(*x);
            return rc;
        }
        s->lanes.push_back(std::move(L));
    }
    *out = s.release();
    return GRAND_OK;
}

void grand_server_destroy(grand_server *s)
{
    if (!s)
        return;
    for (auto &L : s->lanes)
        lane_free(*L);
    delete s;
}

int grand_server_submit(grand_server *s, const grand_code *code, const float *rx, uint32_t M,
                        float noise_var, uint64_t query_cap, uint64_t *request_id)
{
    if (!s)
        return fail(GRAND_EINVAL, "null server");
    std::lock_guard<std::mutex> g(s->mu);
    return submit_locked(s, code, rx, M, noise_var, query_cap, 0.0, request_id);
}

int grand_server_cancel(grand_server *s, uint64_t request_id)
{
    if (!s)
        return fail(GRAND_EINVAL, "null server");
    std::lock_guard<std::mutex> g(s->mu);
    for (std::deque<Request> *queue : {&s->pending, &s->pending_wide}) {
        for (auto it = queue->begin(); it != queue->end(); ++it) {
            if (it->id == request_id) {
                s->mem_in_use -= it->bytes;
                s->inflight--;
                queue->erase(it);
                return GRAND_OK;
            }
        }
    }
    return fail(GRAND_ENOTFOUND, "request not pending (unknown, launched or finished)");
}

int grand_server_poll(grand_server *s, grand_result *out, uint32_t max_out, uint32_t *n_out)
{
    if (!s || (max_out && !out))
        return fail(GRAND_EINVAL, "null pointer");
    std::lock_guard<std::mutex> g(s->mu);
    return poll_locked(s, out, max_out, n_out);
}

int grand_server_stats(grand_server *s, uint64_t *pending, uint64_t *running,
                       uint64_t *memory_in_use)
{
    if (!s)
        return fail(GRAND_EINVAL, "null server");
    std::lock_guard<std::mutex> g(s->mu);
    if (pending)
        *pending = s->pending.size() + s->pending_wide.size();
    if (running)
        *running = s->running;
    if (memory_in_use)
        *memory_in_use = s->mem_in_use;
    return GRAND_OK;
}

// Every request of a trace names a code and reads 2L floats inside rx.
static int check_trace(const grand_code *const *codes, uint32_t n_codes,
                       const grand_trace_req *reqs, uint32_t count, uint64_t rx_count)
{
    for (uint32_t i = 0; i < count; i++) {
        const grand_trace_req &r = reqs[i];
        if (r.code_index >= n_codes || !codes[r.code_index])
            return fail(GRAND_EINVAL, "trace request with a bad code index");
        if (!valid_m(r.M))
            return fail(GRAND_EINVAL, "trace request with an invalid M");
        const uint64_t need = 2ull * symbols(codes[r.code_index]->n, r.M);
        if (r.rx_offset > rx_count || rx_count - r.rx_offset < need)
            return fail(GRAND_EINVAL, "trace request " + std::to_string(i) +
                                          ": received values past rx_count");
    }
    return GRAND_OK;
}

int grand_server_run_trace(grand_server *s, const grand_code *const *codes, uint32_t n_codes,
                           const grand_trace_req *reqs, uint32_t count, const float *rx,
                           uint64_t rx_count, grand_result *results, double *wall_s)
{
    if (!s || !codes || !reqs || !rx || !results || n_codes == 0)
        return fail(GRAND_EINVAL, "null pointer");
    if (int rc = check_trace(codes, n_codes, reqs, count, rx_count))
        return rc;
    std::unordered_map<uint64_t, uint32_t> slot_of;
    std::vector<grand_result> buf(1024);
    const double t0 = now_s();
    uint32_t next = 0, completed = 0;
    std::lock_guard<std::mutex> g(s->mu);
    while (completed < count) {
        const double t = now_s() - t0;
        while (next < count && reqs[next].arrival_s <= t) {
            const grand_trace_req &r = reqs[next];
            uint64_t id = 0;
            int rc = submit_locked(s, codes[r.code_index], rx + r.rx_offset, r.M, r.noise_var,
                                   r.query_cap, t0 + r.arrival_s, &id);
            if (rc == GRAND_EBUSY)
                break;           // retried once completions free room
            if (rc)
                return rc;
            slot_of[id] = next++;
        }
        uint32_t got = 0;
        int rc = poll_locked(s, buf.data(), (uint32_t)buf.size(), &got);
        if (rc)
            return rc;
        for (uint32_t k = 0; k < got; k++) {
            auto it = slot_of.find(buf[k].request_id);
            if (it == slot_of.end())
                continue;        // a request submitted outside this replay
            results[it->second] = buf[k];
            slot_of.erase(it);
            completed++;
        }
    }
    if (wall_s)
        *wall_s = now_s() - t0;
    return GRAND_OK;
}

int grand_plain_run_trace(const grand_code *const *codes, uint32_t n_codes,
                          const grand_trace_req *reqs, uint32_t count, const float *rx,
                          uint64_t rx_count, grand_result *results, double *wall_s)
{
    if (!codes || !reqs || !rx || !results || n_codes == 0)
        return fail(GRAND_EINVAL, "null pointer");
    if (int rc = check_trace(codes, n_codes, reqs, count, rx_count))
        return rc;
    const double t0 = now_s();
    for (uint32_t i = 0; i < count; i++) {
        const grand_trace_req &r = reqs[i];
        if (r.code_index >= n_codes || !codes[r.code_index])
            return fail(GRAND_EINVAL, "trace request with a bad code index");
        while (now_s() - t0 < r.arrival_s) {
        }
        grand_result &o = results[i];
        std::memset(&o, 0, sizeof(o));
        o.request_id = i + 1;
        o.arrival_s = t0 + r.arrival_s;
        o.submit_s = now_s();
        int rc = grand_decode(codes[r.code_index], rx + r.rx_offset, r.M, r.noise_var,
                              r.query_cap, o.codeword, &o.queries, &o.abandoned);
        if (rc)
            return rc;
        o.checks = 0;
        o.status = GRAND_OK;
        o.complete_s = now_s();
    }
    if (wall_s)
        *wall_s = now_s() - t0;
    return GRAND_OK;
}

}  // extern "C"
