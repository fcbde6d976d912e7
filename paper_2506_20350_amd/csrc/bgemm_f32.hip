// FP32 instantiations of the block product (four- and three-product forms).
#include "bgemm_impl.h"
#include "bgemm_launch.h"

namespace mlfft {

template<typename T, int BP, int NT, int WAVES, int TAG>
static hipError_t launch_real_cfg(const GemmTask& t0, const GemmTask* td, int n, int grid, hipStream_t s) {
    const size_t lds = (size_t)NT * (2 * BP + 2) * sizeof(T);
    auto k = bgemm_real_kernel<T, BP, NT, WAVES, TAG>;
    (void)hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k, dim3(grid), dim3(64 * WAVES), lds, s, t0, td, n);
    return hipGetLastError();
}

// tag 1 (preconditioner) always uses one fixed shape, so its kernel symbol differs
// from every shape the MLFFT product can take
template<typename T, int BP>
static hipError_t launch_real(GemmShape sh, int tag, const GemmTask& t0, const GemmTask* td, int n, int grid,
                              hipStream_t s) {
    constexpr int NS = sizeof(T) == 8 ? 16 : 32;
    if (tag) return launch_real_cfg<T, BP, NS, 8, 1>(t0, td, n, grid, s);
    const bool big = sh.nt == 2 * NS;
    if (sh.waves == 4)
        return big ? launch_real_cfg<T, BP, 2 * NS, 4, 0>(t0, td, n, grid, s)
                   : launch_real_cfg<T, BP, NS, 4, 0>(t0, td, n, grid, s);
    return big ? launch_real_cfg<T, BP, 2 * NS, 8, 0>(t0, td, n, grid, s)
               : launch_real_cfg<T, BP, NS, 8, 0>(t0, td, n, grid, s);
}

template<int BP, int NT, int WAVES, int TAG = 0>
static hipError_t launch_3m_cfg(const GemmTask& t0, const GemmTask* td, int n, int grid, hipStream_t s) {
    const size_t lds = (size_t)NT * (2 * BP + 2) * sizeof(float);
    auto k = bgemm_f32_3m_kernel<BP, NT, WAVES, TAG>;
    (void)hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k, dim3(grid), dim3(64 * WAVES), lds, s, t0, td, n);
    return hipGetLastError();
}

template<int BP, int NT, int TAG = 0, int DB = 0, int WAVES = 8>
static hipError_t launch_3m_flat_cfg(const GemmTask& t0, const GemmTask* td, int n, int grid, hipStream_t s) {
    const size_t lds = (size_t)(DB ? 4 : 2) * NT * (2 * BP + 2) * sizeof(float);
    auto k = bgemm_f32_3m_flat_kernel<BP, NT, TAG, DB, WAVES>;
    (void)hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k, dim3(grid), dim3(64 * WAVES), lds, s, t0, td, n);
    return hipGetLastError();
}

template<int BP, int TAG>
static hipError_t launch_direct_cfg(const GemmTask& t0, const GemmTask* td, int n, int grid, hipStream_t s) {
    if constexpr (BP >= 104) {
        const size_t lds = (size_t)4 * 16 * f32_direct_rs(BP) * sizeof(float2);
        auto k = bgemm_f32_3m_direct_kernel<BP, TAG>;
        (void)hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL(k, dim3(grid), dim3(512), lds, s, t0, td, n);
        return hipGetLastError();
    } else {
        return hipErrorInvalidValue;     // the flat kernels need ceil(b / 16) >= 7
    }
}

template<int BP>
static hipError_t launch_f32(GemmShape sh, int tag, const GemmTask& t0, const GemmTask* td, int n, int grid,
                             hipStream_t s) {
    constexpr int B16 = (BP + 15) / 16 * 16;
    if (sh.m3 == 4)       // flat, direct-to-LDS tiles (even b)
        return tag ? launch_direct_cfg<BP, 1>(t0, td, n, grid, s) : launch_direct_cfg<BP, 0>(t0, td, n, grid, s);
    // the flat kernels slice rows at run time and only need the reduction
    // length padded to a multiple of 8 (b = 200: 50 reduction steps, not 52)
    if (tag)      // preconditioner: fixed shape (flat unless some b is below 97)
        return sh.m3 == 2 ? (sh.nt == 16 ? launch_3m_flat_cfg<BP, 16, 1, 1>(t0, td, n, grid, s)
                                         : launch_3m_flat_cfg<BP, 32, 1>(t0, td, n, grid, s))
                          : launch_3m_cfg<B16, 32, 8, 1>(t0, td, n, grid, s);
    if (sh.m3 == 2) {
        if (sh.waves == 4) return launch_3m_flat_cfg<BP, 16, 0, 0, 4>(t0, td, n, grid, s);
        return sh.nt == 16 ? launch_3m_flat_cfg<BP, 16, 0, 1>(t0, td, n, grid, s) : launch_3m_flat_cfg<BP, 32>(t0, td, n, grid, s);
    }
    if (sh.m3) {
        if (sh.waves == 4)
            return sh.nt == 64 ? launch_3m_cfg<B16, 64, 4>(t0, td, n, grid, s) : launch_3m_cfg<B16, 32, 4>(t0, td, n, grid, s);
        return sh.nt == 64 ? launch_3m_cfg<B16, 64, 8>(t0, td, n, grid, s) : launch_3m_cfg<B16, 32, 8>(t0, td, n, grid, s);
    }
    return launch_real<float, BP>(sh, tag, t0, td, n, grid, s);
}

hipError_t launch_bgemm_f32(int bp, GemmShape sh, int tag, const GemmTask& t0, const GemmTask* td, int n, int grid,
                            hipStream_t s) {
    switch (bp) {
#define C32(B) case B: return launch_f32<B>(sh, tag, t0, td, n, grid, s);
        MLFFT_BP8(C32)
#undef C32
        default: return hipErrorInvalidValue;
    }
}

}  // namespace mlfft
