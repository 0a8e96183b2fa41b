// grand_kernels_n128.hip -- the decode kernel for the launch shape of N = 128
// 16-QAM batches (256 threads, 2L = 64 flips, a 2^9-entry low table) and its
// launcher.  This file is compiled on its own, without the compiler's atomic
// optimizer (the flag is in build.py): the optimizer wraps each single-lane
// LDS claim in lane-counting code, and this shape ran 4.7 % faster without
// it, with identical results, while the N = 1024 shape ran 6 % slower, so
// the other shapes keep the default.  The kernel also takes the range end's
// early exits as selects (node_end's SelectExits, 2 % faster here and no
// faster in the other shapes).

#include "grand_decode.h"

namespace grand {

int launch_decode_n128(const KernelArgs &a, uint32_t grid, uint32_t lds, void *stream)
{
    void (*fn)(KernelArgs) = grand_decode_kernel_fixed<64, 9, true>;   // node_end's exits as selects
    if (hipFuncSetAttribute((const void *)fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds) != hipSuccess)
        return -3;
    hipLaunchKernelGGL(fn, dim3(grid), dim3(256), lds, (hipStream_t)stream, a);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

}  // namespace grand
