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

template<int BP, int TAG, int NT, int WAVES>
static hipError_t launch_b16_flat_cfg(const GemmTask& t0, const GemmTask* td, int n, int grid, hipStream_t s) {
    const size_t lds = (size_t)4 * NT * (BP + 4) * sizeof(uint32_t);
    auto k = bgemm_bf16_flat_kernel<BP, NT, TAG, WAVES>;
    (void)hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k, dim3(grid), dim3(64 * WAVES), lds, s, t0, td, n);
    return hipGetLastError();
}

template<int BP, int TAG, int RANGE, int PAIRS = 0, int XB = 0>
static hipError_t launch_b16_freq(const GemmTask& t0, const GemmTask* td, int n, int grid, hipStream_t s) {
    constexpr int BP32 = (BP + 31) / 32 * 32;
    const size_t lds = (size_t)4 * 32 * (BP32 + 8) * sizeof(unsigned short);
    auto k = bgemm_bf16_freq_kernel<BP, 32, TAG, RANGE, PAIRS, XB>;
    (void)hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k, dim3(grid), dim3(512), lds, s, t0, td, n);
    return hipGetLastError();
}

template<int BP, int TAG>
static hipError_t launch_b16_flat(GemmShape sh, const GemmTask& t0, const GemmTask* td, int n, int grid,
                                  hipStream_t s) {
    if (sh.waves == 8 && sh.nt == 32) return launch_b16_flat_cfg<BP, TAG, 32, 8>(t0, td, n, grid, s);
    if (sh.waves == 4 && sh.nt == 16) return launch_b16_flat_cfg<BP, TAG, 16, 4>(t0, td, n, grid, s);
    return hipErrorInvalidValue;
}

// the eight-wave flat kernel needs ceil(b/16) >= 7 (b >= 97), the four-wave one
// ceil(b/16) >= 3 (b >= 33); reduction lengths from 48 up
#define MLFFT_BP16_FLAT(X) X(48) X(64) X(80) X(96) X(112) X(128) X(144) X(160) X(176) X(192) X(208) X(224) \
    X(240) X(256)

#define MLFFT_BP16_FREQ(X) X(16) X(32) X(48) X(64) X(80) X(96) X(112) X(128) X(144) X(160) X(176) X(192) X(208)

hipError_t launch_bgemm_bf16(int bp, GemmShape sh, int tag, const GemmTask& t0, const GemmTask* td, int n, int grid,
                             hipStream_t s) {
    if (sh.m3 == 3 || sh.m3 == 5) {
        // form 5 moves pairs of complex values when every task has even b and 16-byte
        // aligned spectra
        const bool pairs = sh.m3 == 5 && sh.pairs;
        if (sh.x16 && !(pairs && tag)) return hipErrorInvalidValue;
        switch (bp) {
#define Q16(B) case B: return sh.m3 == 5 ? (pairs ? (tag ? (sh.x16 ? launch_b16_freq<B, 1, 1, 1, 1>(t0, td, n, grid, s) \
                                                                   : launch_b16_freq<B, 1, 1, 1>(t0, td, n, grid, s))   \
                                                          : launch_b16_freq<B, 0, 1, 1>(t0, td, n, grid, s))  \
                                                  : (tag ? launch_b16_freq<B, 1, 1>(t0, td, n, grid, s)      \
                                                         : launch_b16_freq<B, 0, 1>(t0, td, n, grid, s)))    \
                                         : (tag ? launch_b16_freq<B, 1, 0>(t0, td, n, grid, s)          \
                                                : launch_b16_freq<B, 0, 0>(t0, td, n, grid, s));
            MLFFT_BP16_FREQ(Q16)
#undef Q16
            default: return hipErrorInvalidValue;
        }
    }
    if (sh.m3 == 2) {
        switch (bp) {
#define F16(B) case B: return tag ? launch_b16_flat<B, 1>(sh, t0, td, n, grid, s) \
                                  : launch_b16_flat<B, 0>(sh, t0, td, n, grid, s);
            MLFFT_BP16_FLAT(F16)
#undef F16
            default: return hipErrorInvalidValue;
        }
    }
    switch (bp) {
#define C16(B) case B: return tag ? launch_b16_cfg<B, 1>(t0, td, n, grid, sh.waves, s) \
                                  : launch_b16_cfg<B, 0>(t0, td, n, grid, sh.waves, s);
        MLFFT_BP16(C16)
#undef C16
        default: return hipErrorInvalidValue;
    }
}

}  // namespace mlfft
