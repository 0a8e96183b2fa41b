// grand_kernels.hip -- the GRAND decoder's kernels for the generic, merged-
// batch and wide launch shapes, and the launchers that pick a kernel for a
// launch (the device code itself is in grand_decode.h).

#include "grand_decode.h"

namespace grand {

namespace {

// Batches: 256 threads and at most 72 VGPRs (7 waves per SIMD); the kernel
// is bound by LDS and memory latency, so more resident waves beat the few
// registers spilled.
__global__ __launch_bounds__(256, 7) void grand_decode_kernel(KernelArgs a)
{
    __shared__ Shared sh;
    decode_loop<0, 0, 0>(a, sh);
}

// Launches of few words: 1024 threads (16 waves) per word, so a word has a
// whole compute unit's SIMDs; at most 128 VGPRs.
__global__ __launch_bounds__(1024, 4) void grand_decode_kernel_wide(KernelArgs a)
{
    __shared__ Shared sh;
    decode_loop<0, 0, 0>(a, sh);
}

__global__ void zero_kernel(unsigned long long *p, uint32_t n)
{
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x)
        p[i] = 0;
}

}  // namespace

int launch_zero(unsigned long long *p, uint32_t n, void *stream)
{
    hipLaunchKernelGGL(zero_kernel, dim3(1), dim3(64), 0, (hipStream_t)stream, p, n);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

int launch_decode(const KernelArgs &a, uint32_t grid, uint32_t block, void *stream)
{
    if (block > kMaxBlock || block % 64 || block == 0)
        return -1;
    const uint32_t lds = 4u * lds_layout(a.ni, block, a.low_bits).words;
    void (*fn)(KernelArgs) = grand_decode_kernel;
    if (block > 256)
        fn = grand_decode_kernel_wide;
    else if (block == 256 && a.low_bits == 9 && a.ni == 64)     // N = 128, 16-QAM
        return launch_decode_n128(a, grid, lds, stream);
    else if (block == 256 && a.low_bits == 9 && a.ni == 512)    // merged batches up to N = 512
        fn = grand_decode_kernel_fixed<512, 9>;
    else if (block == 256 && a.low_bits == 9 && a.ni == 1024)   // merged batches up to N = 1024
        fn = grand_decode_kernel_fixed<1024, 9>;
    if (hipFuncSetAttribute((const void *)fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds) != hipSuccess)
        return -3;
    hipLaunchKernelGGL(fn, dim3(grid), dim3(block), lds, (hipStream_t)stream, a);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

}  // namespace grand
