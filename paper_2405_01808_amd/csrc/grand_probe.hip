// grand_probe.hip -- measured 32-bit bitwise throughput of the device, the
// peak against which the decode kernel's roofline is quoted.
//
// Every lane runs eight rotating XOR chains, written one instruction per
// XOR, over a grid that fills every compute unit several times over.  One step
// is eight v_xor_b32 per lane; gfx950 has no three-input XOR, so a column
// XOR of the incremental syndrome costs exactly one such instruction.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "grand.h"

namespace {

constexpr uint32_t kProbeBlock = 256;
constexpr uint32_t kProbeUnroll = 8;

__global__ __launch_bounds__(256) void xor_rate_kernel(uint32_t steps, uint32_t seed, uint32_t *out)
{
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t a = seed ^ t, b = a * 3u + 1u, c = a * 5u + 7u, d = a * 9u + 3u;
    uint32_t e = a * 17u + 5u, f = a * 33u + 11u, g = a * 65u + 13u, h = a * 129u + 17u;
    for (uint32_t i = 0; i < steps; i += kProbeUnroll) {
#pragma unroll
        for (uint32_t u = 0; u < kProbeUnroll; u++) {
            // one instruction per XOR: the compiler may not re-associate
            // the network (it would fold most of it away)
            asm volatile("v_xor_b32 %0, %0, %1" : "+v"(a) : "v"(b));
            asm volatile("v_xor_b32 %0, %0, %1" : "+v"(b) : "v"(c));
            asm volatile("v_xor_b32 %0, %0, %1" : "+v"(c) : "v"(d));
            asm volatile("v_xor_b32 %0, %0, %1" : "+v"(d) : "v"(e));
            asm volatile("v_xor_b32 %0, %0, %1" : "+v"(e) : "v"(f));
            asm volatile("v_xor_b32 %0, %0, %1" : "+v"(f) : "v"(g));
            asm volatile("v_xor_b32 %0, %0, %1" : "+v"(g) : "v"(h));
            asm volatile("v_xor_b32 %0, %0, %1" : "+v"(h) : "v"(a));
        }
    }
    out[t] = a + b + c + d + e + f + g + h;
}

}  // namespace

extern "C" int grand_probe_xor_rate(uint32_t steps, double *lane_ops_per_s, double *seconds)
{
    if (!lane_ops_per_s || steps == 0 || steps % kProbeUnroll)
        return GRAND_EINVAL;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus <= 0)
        return GRAND_EDEVICE;
    const uint32_t grid = (uint32_t)cus * 8u;
    const size_t threads = (size_t)grid * kProbeBlock;
    uint32_t *out = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = GRAND_EDEVICE;
    float ms = 0.0f;
    if (hipMalloc(&out, threads * sizeof(uint32_t)) != hipSuccess)
        return GRAND_ENOMEM;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        goto done;
    // one warm-up launch, then the timed one
    hipLaunchKernelGGL(xor_rate_kernel, dim3(grid), dim3(kProbeBlock), 0, 0, kProbeUnroll, 1u, out);
    if (hipEventRecord(e0, 0) != hipSuccess)
        goto done;
    hipLaunchKernelGGL(xor_rate_kernel, dim3(grid), dim3(kProbeBlock), 0, 0, steps, 2u, out);
    if (hipGetLastError() != hipSuccess || hipEventRecord(e1, 0) != hipSuccess ||
        hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess ||
        ms <= 0.0f)
        goto done;
    *lane_ops_per_s = (double)threads * (double)steps * 8.0 / (ms * 1e-3);
    if (seconds)
        *seconds = ms * 1e-3;
    rc = 0;
done:
    if (e0)
        (void)hipEventDestroy(e0);
    if (e1)
        (void)hipEventDestroy(e1);
    (void)hipFree(out);
    return rc;
}
