// BF16-input instantiations of the block product.
#include "bgemm_impl.h"
#include "bgemm_launch.h"

namespace mlfft {

template<int BP, int TAG>
static hipError_t launch_b16_cfg(const GemmTask& t0, const GemmTask* td, int n, int grid, int waves, hipStream_t s) {
    const size_t lds = (size_t)kNT * (2 * BP + 8) * sizeof(unsigned short);
    auto k = bgemm_bf16_kernel<BP, kNT, TAG>;
    (void)hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k, dim3(grid), dim3(64 * waves), lds, s, t0, td, n);
    return hipGetLastError();
}

hipError_t launch_bgemm_bf16(int bp, GemmShape sh, int tag, const GemmTask& t0, const GemmTask* td, int n, int grid,
                             hipStream_t s) {
    switch (bp) {
#define C16(B) case B: return tag ? launch_b16_cfg<B, 1>(t0, td, n, grid, sh.waves, s) \
                                  : launch_b16_cfg<B, 0>(t0, td, n, grid, sh.waves, s);
        MLFFT_BP16(C16)
#undef C16
        default: return hipErrorInvalidValue;
    }
}

}  // namespace mlfft
