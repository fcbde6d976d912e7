// Launch entry points of the block-product kernels, one per precision.
#pragma once
#include "internal.h"

namespace mlfft {

struct GemmShape {
    int waves;      // waves per workgroup
    int nt;         // columns per LDS tile
    int m3;         // FP32 only: 1 = three real products per complex product
    int pairs = 0;  // bf16 form 5: every b even and every spectrum 16-byte aligned
    int x16 = 0;    // bf16 form 5 with pairs: X in bf16 (re, im) pairs (GemmTask::x16 of every task)
};

GemmShape gemm_shape(int prec, int bp, int tag);

#define MLFFT_BP8(X) X(8) X(16) X(24) X(32) X(40) X(48) X(56) X(64) X(72) X(80) X(88) X(96) X(104) \
    X(112) X(120) X(128) X(136) X(144) X(152) X(160) X(168) X(176) X(184) X(192) X(200) X(208) \
    X(216) X(224) X(232) X(240) X(248) X(256)
#define MLFFT_BP16(X) X(16) X(32) X(48) X(64) X(80) X(96) X(112) X(128) X(144) X(160) X(176) X(192) \
    X(208) X(224) X(240) X(256)

hipError_t launch_bgemm_f32(int bp, GemmShape sh, int tag, const GemmTask& t0, const GemmTask* td, int n, int grid,
                            hipStream_t s);
hipError_t launch_bgemm_f64(int bp, GemmShape sh, int tag, const GemmTask& t0, const GemmTask* td, int n, int grid,
                            hipStream_t s);
hipError_t launch_bgemm_bf16(int bp, GemmShape sh, int tag, const GemmTask& t0, const GemmTask* td, int n, int grid,
                             hipStream_t s);

}  // namespace mlfft
