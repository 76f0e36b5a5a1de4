// batch_kern.hip -- the persistent batched kernel for one precision
// (-DMIFFT_REAL=float|double); exports its launcher and LDS sizing.
#include "batch_kernels.hpp"

#ifndef MIFFT_REAL
#error "MIFFT_REAL must be float or double"
#endif

#define MIFFT_CAT2(a, b) a##b
#define MIFFT_CAT(a, b) MIFFT_CAT2(a, b)

extern "C" hipError_t MIFFT_CAT(mifft_batch_launch_, MIFFT_REAL)(const void* args, unsigned grid, size_t lds,
                                                                  int* counters, int ncounters,
                                                                  hipStream_t s)
{
    using namespace mifft;
    const BatchArgs<MIFFT_REAL>& a = *static_cast<const BatchArgs<MIFFT_REAL>*>(args);
    hipLaunchKernelGGL(k_batch_reset<MIFFT_REAL>, dim3(1), dim3(256), 0, s, counters, ncounters);
    if (lds > 65536)
        (void)hipFuncSetAttribute((const void*)&k_batch<MIFFT_REAL>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k_batch<MIFFT_REAL>, dim3(grid), dim3(kBatchBlock), lds, s, a);
    return hipGetLastError();
}

extern "C" int MIFFT_CAT(mifft_batch_blocks_per_cu_, MIFFT_REAL)(size_t lds)
{
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, mifft::k_batch<MIFFT_REAL>, mifft::kBatchBlock, lds) !=
        hipSuccess)
        return 1;
    return n > 0 ? n : 1;
}
