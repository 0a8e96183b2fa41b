// Host sanitizer run of the C ABI's host-side paths (argument validation,
// error strings, sizes).  No GPU is needed: every call here is rejected
// before it reaches the device, or reports GRAND_EDEVICE without one.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "grand.h"

static int fails = 0;
#define EXPECT(cond)                                                     \
    do {                                                                 \
        if (!(cond)) {                                                   \
            std::printf("failed: %s (line %d)\n", #cond, __LINE__);      \
            fails++;                                                     \
        }                                                                \
    } while (0)

int main()
{
    for (int e = 0; e >= -10; e--)
        EXPECT(grand_strerror(e) != nullptr && std::strlen(grand_strerror(e)) > 0);
    EXPECT(grand_last_error() != nullptr);

    grand_code *code = nullptr;
    std::vector<uint64_t> h(4, 0x5ull);
    EXPECT(grand_code_create(8, 4, nullptr, &code) == GRAND_EINVAL);
    EXPECT(grand_code_create(8, 4, h.data(), nullptr) == GRAND_EINVAL);
    EXPECT(grand_code_create(12, 4, h.data(), &code) == GRAND_EINVAL);    // n not a power of two
    EXPECT(grand_code_create(8, 8, h.data(), &code) == GRAND_EINVAL);     // rows >= n
    EXPECT(grand_code_create(2048, 4, h.data(), &code) == GRAND_EINVAL);  // n too large
    grand_code_destroy(nullptr);

    float rx[64] = {0};
    uint64_t cw[16], q;
    uint8_t ab;
    EXPECT(grand_decode(nullptr, rx, 4, 1.0f, 10, cw, &q, &ab) == GRAND_EINVAL);
    EXPECT(grand_decode_ex(nullptr, rx, 4, 1.0f, 10, 8, cw, &q, &ab) == GRAND_EINVAL);
    EXPECT(grand_probe_xor_rate(0, nullptr, nullptr) == GRAND_EINVAL);

    grand_batch b;
    std::memset(&b, 0, sizeof(b));
    EXPECT(grand_decode_batch(nullptr, nullptr) == GRAND_EINVAL);
    b.count = 1;
    EXPECT(grand_decode_batch(&b, nullptr) == GRAND_EINVAL);
    b.count = 0;
    EXPECT(grand_decode_batch(&b, nullptr) == GRAND_OK);   // empty batch: nothing to do
    EXPECT(grand_decode_batch_noalloc(nullptr, nullptr) == GRAND_EINVAL);
    EXPECT(grand_decode_batch_noalloc(&b, nullptr) == GRAND_OK);
    b.count = 1;
    EXPECT(grand_decode_batch_noalloc(&b, nullptr) == GRAND_EINVAL);   // null arrays
    b.count = 0;

    grand_trace_req tr;
    std::memset(&tr, 0, sizeof(tr));
    grand_result res;
    double wall = 0;
    const grand_code *const no_codes[1] = {nullptr};
    EXPECT(grand_plain_run_trace(no_codes, 1, &tr, 1, rx, 64, &res, &wall) == GRAND_EINVAL);
    EXPECT(grand_plain_run_trace(nullptr, 1, &tr, 1, rx, 64, &res, &wall) == GRAND_EINVAL);

    grand_tuning t;
    std::memset(&t, 0, sizeof(t));
    EXPECT(grand_tuning_get(128, 16, nullptr) == GRAND_EINVAL);
    EXPECT(grand_tuning_get(128, 16, &t) == GRAND_OK);
    grand_tuning bad = t;
    bad.block = 100;
    EXPECT(grand_tuning_set(128, 16, &bad) == GRAND_EINVAL);
    bad = t;
    bad.low_bits = 14;
    EXPECT(grand_tuning_set(128, 16, &bad) == GRAND_EINVAL);
    EXPECT(grand_tuning_set(128, 16, nullptr) == GRAND_EINVAL);

    EXPECT(grand_request_bytes(128, 16) > 0);
    EXPECT(grand_request_bytes(48, 16) == 0);
    EXPECT(grand_request_bytes(128, 8) == 0);

    grand_server *srv = nullptr;
    grand_server_config cfg;
    std::memset(&cfg, 0, sizeof(cfg));
    EXPECT(grand_server_create(&cfg, &srv) == GRAND_EINVAL);
    cfg.max_inflight = 4;
    cfg.lanes = 1;
    cfg.max_batch = 1;
    cfg.memory_budget = 1 << 20;
    cfg.mode = GRAND_SERVE_PERSISTENT;
    EXPECT(grand_server_create(&cfg, &srv) == GRAND_EINVAL);
    EXPECT(grand_server_submit(nullptr, nullptr, rx, 4, 1.0f, 1, nullptr) == GRAND_EINVAL);
    EXPECT(grand_server_poll(nullptr, nullptr, 0, nullptr) == GRAND_EINVAL);
    EXPECT(grand_server_cancel(nullptr, 1) == GRAND_EINVAL);
    grand_server_destroy(nullptr);

    grand_graph *g = nullptr;
    EXPECT(grand_graph_create(nullptr, &g) == GRAND_EINVAL);
    EXPECT(grand_graph_create(&b, &g) == GRAND_EINVAL);    // empty batch
    EXPECT(grand_graph_launch(nullptr, nullptr) == GRAND_EINVAL);
    grand_graph_destroy(nullptr);

    std::printf("abi sanitizer run: %d failures\n", fails);
    return fails != 0;
}
