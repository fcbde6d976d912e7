// FP64 instantiations of the block product.
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

template<int BP, int NT, int TAG = 0>
static hipError_t launch_3m_flat_cfg(const GemmTask& t0, const GemmTask* td, int n, int grid, hipStream_t s) {
    const size_t lds = (size_t)2 * NT * (2 * BP + 2) * sizeof(double);
    auto k = bgemm_f64_3m_flat_kernel<BP, NT, TAG>;
    (void)hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k, dim3(grid), dim3(256), lds, s, t0, td, n);
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

template<int BP, int TAG>
static hipError_t launch_direct_cfg(const GemmTask& t0, const GemmTask* td, int n, int grid, hipStream_t s) {
    if constexpr (BP >= 40) {
        const size_t lds = (size_t)4 * 16 * f64_direct_rs(BP) * sizeof(double2);
        auto k = bgemm_f64_3m_direct_kernel<BP, TAG>;
        (void)hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL(k, dim3(grid), dim3(256), lds, s, t0, td, n);
        return hipGetLastError();
    } else {
        return hipErrorInvalidValue;     // four waves of one slice each need ceil(b / 16) >= 3
    }
}

template<int BP>
static hipError_t launch_f64(GemmShape sh, int tag, const GemmTask& t0, const GemmTask* td, int n, int grid,
                             hipStream_t s) {
    if (sh.m3 == 4)       // flat, direct-to-LDS half-reduction tiles
        return tag ? launch_direct_cfg<BP, 1>(t0, td, n, grid, s) : launch_direct_cfg<BP, 0>(t0, td, n, grid, s);
    // the flat kernel slices rows at run time and only needs the reduction length
    // padded to a multiple of 8
    if (sh.m3 == 2)
        return tag ? launch_3m_flat_cfg<BP, 16, 1>(t0, td, n, grid, s) : launch_3m_flat_cfg<BP, 16>(t0, td, n, grid, s);
    return launch_real<double, BP>(sh, tag, t0, td, n, grid, s);
}

hipError_t launch_bgemm_f64(int bp, GemmShape sh, int tag, const GemmTask& t0, const GemmTask* td, int n, int grid,
                            hipStream_t s) {
    switch (bp) {
#define C64(B) case B: return launch_f64<B>(sh, tag, t0, td, n, grid, s);
        MLFFT_BP8(C64)
#undef C64
        default: return hipErrorInvalidValue;
    }
}

}  // namespace mlfft
