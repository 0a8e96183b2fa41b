// grand_probe.hip -- measured 32-bit bitwise throughput of the device, the
// peak against which the decode kernel's roofline is quoted.
//
// Every lane runs eight rotating XOR chains, written one instruction per
// XOR, over a grid that fills every compute unit several times over.  One step
// is eight v_xor_b32 per lane; gfx950 has no three-input XOR, so a column
// XOR of the incremental syndrome costs exactly one such instruction.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "grand.h"
#include "grand_host.h"

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

// Baseline for the incremental syndrome: Algorithm 1 run in full for every
// pattern, as in Algorithm 2's Step 5 (one pMult per test error pattern).
// Check g of the launch takes word g / patterns and pattern g % patterns:
// the word is a hash-generated hard decision, the pattern flips the bits of
// the pattern index at 16 positions spread over the word.  s = H (yhat + e)
// is formed row by row from the bit-packed rows in LDS (AND, XOR-fold of the
// row's words, parity), and zero syndromes are counted.  N is a template
// parameter, so the word stays in registers and the flip positions fold.
__device__ inline uint32_t probe_hash(uint32_t a, uint32_t b)
{
    uint32_t h = a * 0x9E3779B1u ^ (b + 0x7F4A7C15u) * 0x85EBCA77u;
    h ^= h >> 15;
    h *= 0x2C1B3C6Du;
    h ^= h >> 12;
    return h;
}

template <uint32_t N>
__global__ __launch_bounds__(256) void dense_pmult_kernel(const uint32_t *h_rows, uint32_t rows,
                                                          uint64_t checks, uint32_t patterns,
                                                          const uint32_t *words,
                                                          unsigned long long *zeros)
{
    constexpr uint32_t W = N <= 64 ? 2u : N / 32u;   // 32-bit words per packed row
    extern __shared__ uint32_t hs[];
    for (uint32_t i = threadIdx.x; i < rows * W; i += blockDim.x)
        hs[i] = h_rows[i];
    __syncthreads();
    unsigned long long found = 0;
    for (uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; g < checks;
         g += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t wi = (uint32_t)(g / patterns), p = (uint32_t)(g % patterns);
        uint32_t x[W];
#pragma unroll
        for (uint32_t k = 0; k < W; k++) {
            const uint32_t valid = N >= 32 * (k + 1) ? 0xFFFFFFFFu
                                   : (N <= 32 * k ? 0u : (1u << (N - 32 * k)) - 1u);
            // the caller's hard words (W 32-bit words each), or hashed ones
            x[k] = (words ? words[(uint64_t)wi * W + k] : probe_hash(wi, k)) & valid;
        }
#pragma unroll
        for (uint32_t j = 0; j < 16; j++) {
            const uint32_t pos = j * N / 16;
            x[pos >> 5] ^= ((p >> j) & 1u) << (pos & 31u);
        }
        uint32_t any = 0;
        for (uint32_t r = 0; r < rows; r++) {
            uint32_t acc = 0;
#pragma unroll
            for (uint32_t k = 0; k < W; k++)
                acc ^= hs[r * W + k] & x[k];
            any |= __popc(acc) & 1u;
        }
        found += any == 0;
    }
    if (found)
        atomicAdd(zeros, found);
}

template <uint32_t N>
int launch_dense(const grand_code *c, uint32_t grid, uint64_t checks, uint32_t patterns,
                 const uint32_t *words, unsigned long long *zeros)
{
    const uint32_t lds = c->rows * c->row_w32 * 4u;
    if (hipFuncSetAttribute((const void *)dense_pmult_kernel<N>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
        return GRAND_EDEVICE;
    hipLaunchKernelGGL(dense_pmult_kernel<N>, dim3(grid), dim3(256), lds, 0, c->d_rows, c->rows,
                       checks, patterns, words, zeros);
    return hipGetLastError() == hipSuccess ? 0 : GRAND_EDEVICE;
}

int launch_dense_any(const grand_code *c, uint32_t grid, uint64_t checks, uint32_t patterns,
                     const uint32_t *words, unsigned long long *zeros)
{
    switch (c->n) {
    case 2: return launch_dense<2>(c, grid, checks, patterns, words, zeros);
    case 4: return launch_dense<4>(c, grid, checks, patterns, words, zeros);
    case 8: return launch_dense<8>(c, grid, checks, patterns, words, zeros);
    case 16: return launch_dense<16>(c, grid, checks, patterns, words, zeros);
    case 32: return launch_dense<32>(c, grid, checks, patterns, words, zeros);
    case 64: return launch_dense<64>(c, grid, checks, patterns, words, zeros);
    case 128: return launch_dense<128>(c, grid, checks, patterns, words, zeros);
    case 256: return launch_dense<256>(c, grid, checks, patterns, words, zeros);
    case 512: return launch_dense<512>(c, grid, checks, patterns, words, zeros);
    case 1024: return launch_dense<1024>(c, grid, checks, patterns, words, zeros);
    default: return GRAND_EINVAL;
    }
}

// Algorithm 1 for a batch of vectors: thread i forms s = H x_i^T row by row
// from the packed rows in LDS (the AND of row and vector, the XOR fold of
// the products' words, the parity of the fold: the Theorem's log2 addition
// tree over the row's support) and writes the syndrome bit-packed.
__global__ __launch_bounds__(256) void pmult_batch_kernel(const uint32_t *h_rows, uint32_t rows,
                                                          uint32_t w32, const uint64_t *x,
                                                          uint32_t count, uint64_t *syn)
{
    extern __shared__ uint32_t hs[];
    for (uint32_t i = threadIdx.x; i < rows * w32; i += blockDim.x)
        hs[i] = h_rows[i];
    __syncthreads();
    const uint32_t w64 = w32 / 2, s64 = (rows + 63) / 64;
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < count;
         v += gridDim.x * blockDim.x) {
        const uint32_t *xv = (const uint32_t *)(x + (uint64_t)v * w64);
        uint64_t *out = syn + (uint64_t)v * s64;
        for (uint32_t o = 0; o < s64; o++) {
            uint64_t bits = 0;
            for (uint32_t r = 64 * o; r < rows && r < 64 * (o + 1); r++) {
                uint32_t acc = 0;
                for (uint32_t k = 0; k < w32; k++)
                    acc ^= hs[r * w32 + k] & xv[k];
                bits |= (uint64_t)(__popc(acc) & 1u) << (r - 64 * o);
            }
            out[o] = bits;
        }
    }
}

}  // namespace

extern "C" int grand_pmult(const grand_code *code, const uint64_t *x, uint32_t count,
                           uint64_t *syndromes, void *stream)
{
    if (!code || (count && (!x || !syndromes)))
        return GRAND_EINVAL;
    if (count == 0)
        return GRAND_OK;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev != code->device ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus <= 0)
        return GRAND_EDEVICE;
    const uint32_t lds = code->rows * code->row_w32 * 4u;
    if (hipFuncSetAttribute((const void *)pmult_batch_kernel,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
        return GRAND_EDEVICE;
    const uint32_t grid = std::min<uint32_t>((count + 255) / 256, (uint32_t)cus * 8u);
    hipLaunchKernelGGL(pmult_batch_kernel, dim3(grid), dim3(256), lds, (hipStream_t)stream,
                       code->d_rows, code->rows, code->row_w32, x, count, syndromes);
    return hipGetLastError() == hipSuccess ? GRAND_OK : GRAND_EDEVICE;
}

extern "C" int grand_probe_dense_pmult(const grand_code *code, const uint64_t *words_dev,
                                       uint32_t words, uint32_t patterns, double *checks_per_s,
                                       uint64_t *zero_syndromes)
{
    if (!code || !checks_per_s || words == 0 || patterns == 0 || patterns > 65536 ||
        (uint64_t)words * patterns > (1ull << 32))
        return GRAND_EINVAL;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev != code->device ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus <= 0)
        return GRAND_EDEVICE;
    const uint64_t checks = (uint64_t)words * patterns;
    const uint32_t grid = (uint32_t)cus * 8u;
    unsigned long long *zeros = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = GRAND_EDEVICE;
    float ms = 0.0f;
    unsigned long long hz = 0;
    if (hipMalloc((void **)&zeros, sizeof(unsigned long long)) != hipSuccess)
        return GRAND_ENOMEM;
    if (hipMemset(zeros, 0, sizeof(unsigned long long)) != hipSuccess ||
        hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        goto done;
    // warm-up on the first word's patterns, then the timed launch
    rc = launch_dense_any(code, grid, patterns, patterns, (const uint32_t *)words_dev, zeros);
    if (rc)
        goto done;
    rc = GRAND_EDEVICE;
    if (hipDeviceSynchronize() != hipSuccess ||
        hipMemset(zeros, 0, sizeof(unsigned long long)) != hipSuccess ||
        hipEventRecord(e0, 0) != hipSuccess)
        goto done;
    rc = launch_dense_any(code, grid, checks, patterns, (const uint32_t *)words_dev, zeros);
    if (rc)
        goto done;
    rc = GRAND_EDEVICE;
    if (hipEventRecord(e1, 0) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&ms, e0, e1) != hipSuccess || ms <= 0.0f ||
        hipMemcpy(&hz, zeros, sizeof(hz), hipMemcpyDeviceToHost) != hipSuccess)
        goto done;
    *checks_per_s = (double)checks / (ms * 1e-3);
    if (zero_syndromes)
        *zero_syndromes = hz;
    rc = 0;
done:
    if (e0)
        (void)hipEventDestroy(e0);
    if (e1)
        (void)hipEventDestroy(e1);
    (void)hipFree(zeros);
    return rc;
}

extern "C" int grand_probe_xor_rate(uint32_t steps, double *lane_ops_per_s, double *seconds)
{
    if (!lane_ops_per_s || steps == 0 || steps % kProbeUnroll || steps > (1u << 20))
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
