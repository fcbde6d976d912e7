// Per-frequency block product of the MLFFT matvec (eq. multL: the block-diagonal
// diag_{N0}(F^[2] C_1^[2]) applied to the transformed vectors), batched over all
// right-hand sides:  Y[k][w][:] = G[k] X[k][w][:]  for every frequency k.
//
// With W right-hand sides each frequency is a complex (b x b) * (b x W) GEMM,
// run on the MFMA units.  A complex product is one real GEMM of twice the size:
// real row 2m+p (p = 0 real, 1 imaginary part of row m), real column 2n+c, with
// the 2x2 block [[gr, -gi], [gi, gr]] of G(m, n); the interleaved complex
// vectors X[k][w][:] are already the real operand in that order.
//
// Scheme (A stationary): a wave owns 16 real rows (8 complex rows) of G[k] and
// keeps their MFMA A fragments for the whole reduction in registers, loaded once.
// The workgroup streams the X columns of the frequency through LDS in tiles of
// NT columns and every wave multiplies the tile by its rows.  Each workgroup
// works on one frequency, so G[k] is read once per row group, and the row
// groups of one frequency are placed on the same XCD so that they share the X
// stream through that XCD's L2.
//
// Precisions: FP64 (v_mfma_f64_16x16x4f64), FP32 (v_mfma_f32_16x16x4f32) and
// BF16 inputs with FP32 accumulation (v_mfma_f32_16x16x32_bf16, gfx950), where
// G is stored as bf16 pairs and X is rounded to bf16 while it is staged in LDS.
#include "internal.h"

namespace mlfft {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short ushortx8 __attribute__((ext_vector_type(8)));

constexpr int kNT = 64;          // columns per LDS tile
constexpr int kXcd = 8;          // XCDs on MI355X; workgroups are dealt round robin

__device__ __forceinline__ const GemmTask* find_gemm_task(const GemmTask* tasks, int ntasks) {
    int lo = 0, hi = ntasks - 1;
    const int bid = blockIdx.x;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (tasks[mid].block_begin <= bid) lo = mid; else hi = mid - 1;
    }
    return tasks + lo;
}

// XCD-aware decode of the workgroup index into (frequency, row group).
__device__ __forceinline__ bool decode_block(const GemmTask& t, int* k, int* mg) {
    const int local = blockIdx.x - t.block_begin;
    const int xcd = local % kXcd;
    const int r = local / kXcd;
    *mg = r % t.mgroups;
    *k = (r / t.mgroups) * kXcd + xcd;
    return *k < t.K;
}

// ------------------------------------------------------------------ FP32 / FP64

template<typename T> struct MfmaReal;
// The accumulator layout of the two instructions differs: lane l, register r
// holds output row 4*(l/16) + r for f32 and row 4*r + l/16 for f64.  A-fragment
// row i is therefore mapped to the (complex row, part) that makes every lane
// end up with (Re m, Im m, Re m+1, Im m+1), m = 2*(l/16), in both cases.
template<> struct MfmaReal<float> {
    typedef floatx4 acc_t;
    typedef float2 c_t;
    static __device__ __forceinline__ int row_cplx(int i) { return i >> 1; }
    static __device__ __forceinline__ int row_part(int i) { return i & 1; }
    static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};
template<> struct MfmaReal<double> {
    typedef doublex4 acc_t;
    typedef double2 c_t;
    static __device__ __forceinline__ int row_cplx(int i) { return 2 * (i & 3) + (i >> 3); }
    static __device__ __forceinline__ int row_part(int i) { return (i >> 2) & 1; }
    static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
};

template<typename T, int BP, int NT, int TAG>
__global__ void __launch_bounds__(512) bgemm_real_kernel(GemmTask t0, const GemmTask* tasks, int ntasks) {
    typedef MfmaReal<T> M;
    typedef typename M::c_t C;
    typedef typename M::acc_t acc_t;
    extern __shared__ unsigned char smem_raw[];
    T* xs = reinterpret_cast<T*>(smem_raw);
    const GemmTask t = ntasks > 0 ? *find_gemm_task(tasks, ntasks) : t0;
    int k, mg;
    if (!decode_block(t, &k, &mg)) return;
    const int b = t.b, W = t.W;
    const int nw = blockDim.x >> 6;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int slice = mg * nw + wave;
    const int nslices = (b + 7) >> 3;
    const bool active = slice < nslices;
    const int m_base = slice * 8;
    const int ldx = 2 * BP + 2;

    // A fragments for all BP/2 reduction steps (4 real columns each)
    T a[BP / 2];
    {
        const C* __restrict__ Gk = static_cast<const C*>(t.G) + (size_t)k * t.gstride;
        const int i = lane & 15, kk = lane >> 4;
        const int m = m_base + M::row_cplx(i), pr = M::row_part(i), pc = kk & 1;
#pragma unroll
        for (int s = 0; s < BP / 2; ++s) {
            const int n = 2 * s + (kk >> 1);
            T v = 0;
            if (active && m < b && n < b) {
                const C g = Gk[(size_t)m * b + n];
                v = pr == 0 ? (pc == 0 ? g.x : -g.y) : (pc == 0 ? g.y : g.x);
            }
            a[s] = v;
        }
    }
    // zero the padded reduction columns n in [b, BP) once; tiles never write them
    const int padn = BP - b;
    for (int e = threadIdx.x; e < NT * padn; e += blockDim.x) {
        const int w = e / padn, n = b + (e - w * padn);
        xs[w * ldx + 2 * n] = 0;
        xs[w * ldx + 2 * n + 1] = 0;
    }
    const C* __restrict__ Xk = static_cast<const C*>(t.X) + (size_t)k * W * b;
    C* __restrict__ Yk = static_cast<C*>(t.Y) + (size_t)k * W * b;
    const int j = lane & 15, q = lane >> 4;
    for (int w0 = 0; w0 < W; w0 += NT) {
        const int ncols = min(NT, W - w0);
        __syncthreads();
        const C* __restrict__ src = Xk + (size_t)w0 * b;
        const int tot = NT * b, have = ncols * b;
        for (int e = threadIdx.x; e < tot; e += blockDim.x) {
            const int w = e / b, n = e - w * b;
            C v = e < have ? src[e] : czero<C>();
            *reinterpret_cast<C*>(&xs[w * ldx + 2 * n]) = v;
        }
        __syncthreads();
        if (active) {
            acc_t acc[NT / 16];
#pragma unroll
            for (int cg = 0; cg < NT / 16; ++cg) acc[cg] = acc_t{0, 0, 0, 0};
#pragma unroll
            for (int s = 0; s < BP / 2; ++s) {
#pragma unroll
                for (int cg = 0; cg < NT / 16; ++cg) {
                    const T bv = xs[(cg * 16 + j) * ldx + 4 * s + q];
                    acc[cg] = M::mma(a[s], bv, acc[cg]);
                }
            }
            const int m = m_base + 2 * q;
#pragma unroll
            for (int cg = 0; cg < NT / 16; ++cg) {
                const int w = w0 + cg * 16 + j;
                if (w < W) {
                    if (m < b) Yk[(size_t)w * b + m] = cmake<C>(acc[cg][0], acc[cg][1]);
                    if (m + 1 < b) Yk[(size_t)w * b + m + 1] = cmake<C>(acc[cg][2], acc[cg][3]);
                }
            }
        }
    }
}

// ------------------------------------------------------------------ BF16

__device__ __forceinline__ unsigned short bf16_rne(float f) { return f32_to_bf16_bits(f); }

template<int BP, int NT, int TAG>
__global__ void __launch_bounds__(512) bgemm_bf16_kernel(GemmTask t0, const GemmTask* tasks, int ntasks) {
    extern __shared__ unsigned char smem_raw[];
    unsigned short* xs = reinterpret_cast<unsigned short*>(smem_raw);
    const GemmTask t = ntasks > 0 ? *find_gemm_task(tasks, ntasks) : t0;
    int k, mg;
    if (!decode_block(t, &k, &mg)) return;
    const int b = t.b, W = t.W;
    const int nw = blockDim.x >> 6;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int slice = mg * nw + wave;
    const int nslices = (b + 7) >> 3;
    const bool active = slice < nslices;
    const int m_base = slice * 8;
    const int ldx = 2 * BP + 8;               // bf16 elements per LDS row (16-byte skew)

    // A fragments: BP/16 steps of 32 real columns; lane holds 8 consecutive real columns
    ushortx8 a[BP / 16];
    {
        const uint32_t* __restrict__ Gk = static_cast<const uint32_t*>(t.G) + (size_t)k * t.gstride;
        const int i = lane & 15, q = lane >> 4;
        const int m = m_base + (i >> 1), pr = i & 1;
#pragma unroll
        for (int s = 0; s < BP / 16; ++s) {
            ushortx8 v;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int n = 16 * s + 4 * q + e;
                uint32_t g = 0;
                if (active && m < b && n < b) g = Gk[(size_t)m * b + n];
                const unsigned short gr = (unsigned short)(g & 0xffffu), gi = (unsigned short)(g >> 16);
                if (pr == 0) { v[2 * e] = gr; v[2 * e + 1] = (unsigned short)(gi ^ 0x8000u); }
                else         { v[2 * e] = gi; v[2 * e + 1] = gr; }
            }
            a[s] = v;
        }
    }
    const int padn = BP - b;
    for (int e = threadIdx.x; e < NT * padn; e += blockDim.x) {
        const int w = e / padn, n = b + (e - w * padn);
        *reinterpret_cast<uint32_t*>(&xs[w * ldx + 2 * n]) = 0u;
    }
    const float2* __restrict__ Xk = static_cast<const float2*>(t.X) + (size_t)k * W * b;
    float2* __restrict__ Yk = static_cast<float2*>(t.Y) + (size_t)k * W * b;
    const int j = lane & 15, q = lane >> 4;
    for (int w0 = 0; w0 < W; w0 += NT) {
        const int ncols = min(NT, W - w0);
        __syncthreads();
        const float2* __restrict__ src = Xk + (size_t)w0 * b;
        const int tot = NT * b, have = ncols * b;
        for (int e = threadIdx.x; e < tot; e += blockDim.x) {
            const int w = e / b, n = e - w * b;
            const float2 v = e < have ? src[e] : make_float2(0.f, 0.f);
            const uint32_t packed = (uint32_t)bf16_rne(v.x) | ((uint32_t)bf16_rne(v.y) << 16);
            *reinterpret_cast<uint32_t*>(&xs[w * ldx + 2 * n]) = packed;
        }
        __syncthreads();
        if (active) {
            floatx4 acc[NT / 16];
#pragma unroll
            for (int cg = 0; cg < NT / 16; ++cg) acc[cg] = floatx4{0, 0, 0, 0};
#pragma unroll
            for (int s = 0; s < BP / 16; ++s) {
#pragma unroll
                for (int cg = 0; cg < NT / 16; ++cg) {
                    const ushortx8 bv = *reinterpret_cast<const ushortx8*>(&xs[(cg * 16 + j) * ldx + 32 * s + 8 * q]);
                    acc[cg] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                        __builtin_bit_cast(bf16x8, a[s]), __builtin_bit_cast(bf16x8, bv), acc[cg], 0, 0, 0);
                }
            }
            const int m = m_base + 2 * q;
#pragma unroll
            for (int cg = 0; cg < NT / 16; ++cg) {
                const int w = w0 + cg * 16 + j;
                if (w < W) {
                    if (m < b) Yk[(size_t)w * b + m] = make_float2(acc[cg][0], acc[cg][1]);
                    if (m + 1 < b) Yk[(size_t)w * b + m + 1] = make_float2(acc[cg][2], acc[cg][3]);
                }
            }
        }
    }
}

// ------------------------------------------------------------------ host side

int gemm_bp(int prec, int b) {
    // padded reduction size: a multiple of 8 (FP32/FP64) or 16 (BF16), from the
    // instantiated list below
    const int q = prec == PBF16 ? 16 : 8;
    int bp = (b + q - 1) / q * q;
    if (bp < q) bp = q;
    return bp;
}

static int waves_for(int nslices) {
    const int groups = (nslices + 7) / 8;
    return (nslices + groups - 1) / groups;
}

void plan_gemm_tasks(int prec, GemmTask* tasks, int ntasks, int* grid, int* bp_max) {
    int g = 0, bpm = 0, wmax = 1;
    for (int i = 0; i < ntasks; ++i) {
        GemmTask& t = tasks[i];
        const int nslices = (t.b + 7) / 8;
        const int bp = gemm_bp(prec, t.b);
        if (bp > bpm) bpm = bp;
        const int wv = waves_for(nslices);
        if (wv > wmax) wmax = wv;
    }
    for (int i = 0; i < ntasks; ++i) {
        GemmTask& t = tasks[i];
        const int nslices = (t.b + 7) / 8;
        t.mgroups = (nslices + wmax - 1) / wmax;
        t.block_begin = g;
        g += ((t.K + kXcd - 1) / kXcd) * kXcd * t.mgroups;
    }
    *grid = g;
    *bp_max = bpm;
}

template<typename T, int BP, int NT>
static hipError_t launch_real_nt(const GemmTask* th, const GemmTask* td, int ntasks, int grid, int waves, int tag,
                                 hipStream_t s) {
    const size_t lds = (size_t)NT * (2 * BP + 2) * sizeof(T);
    auto k = tag ? bgemm_real_kernel<T, BP, NT, 1> : bgemm_real_kernel<T, BP, NT, 0>;
    (void)hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k, dim3(grid), dim3(64 * waves), lds, s, th[0], ntasks > 1 ? td : nullptr,
                       ntasks > 1 ? ntasks : 0);
    return hipGetLastError();
}

// 64-column tiles when they fit the 160 KB of LDS, 32-column tiles otherwise (FP64, b > 160)
template<typename T, int BP>
static hipError_t launch_real(const GemmTask* th, const GemmTask* td, int ntasks, int grid, int waves, int tag,
                              hipStream_t s) {
    if ((size_t)kNT * (2 * BP + 2) * sizeof(T) <= 160 * 1024)
        return launch_real_nt<T, BP, kNT>(th, td, ntasks, grid, waves, tag, s);
    return launch_real_nt<T, BP, kNT / 2>(th, td, ntasks, grid, waves, tag, s);
}

template<int BP>
static hipError_t launch_b16(const GemmTask* th, const GemmTask* td, int ntasks, int grid, int waves, int tag,
                             hipStream_t s) {
    const size_t lds = (size_t)kNT * (2 * BP + 8) * sizeof(unsigned short);
    auto k = tag ? bgemm_bf16_kernel<BP, kNT, 1> : bgemm_bf16_kernel<BP, kNT, 0>;
    (void)hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k, dim3(grid), dim3(64 * waves), lds, s, th[0], ntasks > 1 ? td : nullptr,
                       ntasks > 1 ? ntasks : 0);
    return hipGetLastError();
}

#define MLFFT_BP8(X) X(8) X(16) X(24) X(32) X(40) X(48) X(56) X(64) X(72) X(80) X(88) X(96) X(104) \
    X(112) X(120) X(128) X(136) X(144) X(152) X(160) X(168) X(176) X(184) X(192) X(200) X(208) \
    X(216) X(224) X(232) X(240) X(248) X(256)
#define MLFFT_BP16(X) X(16) X(32) X(48) X(64) X(80) X(96) X(112) X(128) X(144) X(160) X(176) X(192) \
    X(208) X(224) X(240) X(256)

hipError_t launch_bgemm(int prec, const GemmTask* th, const GemmTask* td, int ntasks, int tag, hipStream_t s) {
    if (ntasks <= 0) return hipSuccess;
    int grid = 0, bpm = 0, wmax = 1;
    for (int i = 0; i < ntasks; ++i) {
        const int bp = gemm_bp(prec, th[i].b);
        if (bp > bpm) bpm = bp;
        const int wv = waves_for((th[i].b + 7) / 8);
        if (wv > wmax) wmax = wv;
        const int end = th[i].block_begin + ((th[i].K + kXcd - 1) / kXcd) * kXcd * th[i].mgroups;
        if (end > grid) grid = end;
    }
    if (grid == 0) return hipSuccess;
    if (prec == P64) {
        switch (bpm) {
#define C64(B) case B: return launch_real<double, B>(th, td, ntasks, grid, wmax, tag, s);
            MLFFT_BP8(C64)
#undef C64
            default: return hipErrorInvalidValue;
        }
    } else if (prec == P32) {
        switch (bpm) {
#define C32(B) case B: return launch_real<float, B>(th, td, ntasks, grid, wmax, tag, s);
            MLFFT_BP8(C32)
#undef C32
            default: return hipErrorInvalidValue;
        }
    } else {
        switch (bpm) {
#define C16(B) case B: return launch_b16<B>(th, td, ntasks, grid, wmax, tag, s);
            MLFFT_BP16(C16)
#undef C16
            default: return hipErrorInvalidValue;
        }
    }
}

}  // namespace mlfft
