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
#pragma once
#include "internal.h"

#include <algorithm>

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

template<typename T, int BP, int NT, int WAVES, int TAG>
__global__ void __launch_bounds__(64 * WAVES) bgemm_real_kernel(GemmTask t0, const GemmTask* tasks, int ntasks) {
    typedef MfmaReal<T> M;
    typedef typename M::c_t C;
    typedef typename M::acc_t acc_t;
    // complex elements of the next X tile each thread keeps in registers
    constexpr int PF = (NT * BP + 64 * WAVES - 1) / (64 * WAVES);
    extern __shared__ unsigned char smem_raw[];
    T* xs = reinterpret_cast<T*>(smem_raw);
    const GemmTask t = ntasks > 0 ? *find_gemm_task(tasks, ntasks) : t0;
    int k, mg;
    if (!decode_block(t, &k, &mg)) return;
    const int b = t.b, W = t.W;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int slice = mg * WAVES + wave;
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
                const C g = gload(Gk + (size_t)m * b + n);
                v = pr == 0 ? (pc == 0 ? g.x : -g.y) : (pc == 0 ? g.y : g.x);
            }
            a[s] = v;
        }
    }
    // zero the padded reduction columns n in [b, BP) once; tiles never write them
    const int padn = BP - b;
    for (int e = threadIdx.x; e < NT * padn; e += 64 * WAVES) {
        const int w = e / padn, n = b + (e - w * padn);
        xs[w * ldx + 2 * n] = 0;
        xs[w * ldx + 2 * n + 1] = 0;
    }
    const C* __restrict__ Xk = static_cast<const C*>(t.X) + (size_t)k * W * b;
    C* __restrict__ Yk = static_cast<C*>(t.Y) + (size_t)k * W * b;
    const int j = lane & 15, q = lane >> 4;
    // the tile of NT columns is NT*b consecutive complex values; thread tid owns
    // elements tid + i * 64 * WAVES of it
    C pre[PF];
    auto fetch = [&](int w0) {
        const int have = min(NT, W - w0) * b;
        const C* __restrict__ src = Xk + (size_t)w0 * b;
#pragma unroll
        for (int i = 0; i < PF; ++i) {
            const int e = threadIdx.x + i * 64 * WAVES;
            pre[i] = e < have ? gload(src + e) : czero<C>();
        }
    };
    fetch(0);
    for (int w0 = 0; w0 < W; w0 += NT) {
        __syncthreads();
#pragma unroll
        for (int i = 0; i < PF; ++i) {
            const int e = threadIdx.x + i * 64 * WAVES;
            if (e < NT * b) {
                const int w = e / b, n = e - w * b;
                *reinterpret_cast<C*>(&xs[w * ldx + 2 * n]) = pre[i];
            }
        }
        __syncthreads();
        if (w0 + NT < W) fetch(w0 + NT);      // next tile in flight while this one is multiplied
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
                    if (m < b) gstore(Yk + (size_t)w * b + m, cmake<C>(acc[cg][0], acc[cg][1]));
                    if (m + 1 < b) gstore(Yk + (size_t)w * b + m + 1, cmake<C>(acc[cg][2], acc[cg][3]));
                }
            }
        }
    }
}

// ------------------------------------------------------------------ FP32, three real products

// Complex product with three real products per complex multiply-add (the
// Gauss / "3M" form): T1 = Gr Ur, T2 = Gi Ui, T3 = (Gr + Gi)(Ur + Ui), then
// Re = T1 - T2, Im = T3 - T1 - T2.  A wave owns 16 complex rows; its A
// fragments (Gr, Gi, Gr + Gi for all BP/4 reduction steps) stay in registers;
// B fragments are the real and imaginary parts of 4 consecutive basis
// functions of 16 columns, read from the LDS tile as one 8-byte pair.  The
// MFMA work is 6 b^2 W flops instead of 8 b^2 W; the rounding error of Im grows
// by at most a factor ~2 (|T3| <= 2 |G| |U|).
template<int BP, int NT, int WAVES, int TAG>
__global__ void __launch_bounds__(64 * WAVES) bgemm_f32_3m_kernel(GemmTask t0, const GemmTask* tasks, int ntasks) {
    constexpr int PF = (NT * BP + 64 * WAVES - 1) / (64 * WAVES);
    extern __shared__ unsigned char smem_raw[];
    float* xs = reinterpret_cast<float*>(smem_raw);
    const GemmTask t = ntasks > 0 ? *find_gemm_task(tasks, ntasks) : t0;
    int k, mg;
    if (!decode_block(t, &k, &mg)) return;
    const int b = t.b, W = t.W;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int slice = mg * WAVES + wave;
    const int nslices = (b + 15) >> 4;
    const bool active = slice < nslices;
    const int m_base = slice * 16;
    const int ldx = 2 * BP + 2;
    float ar[BP / 4], ai[BP / 4], as[BP / 4];
    {
        const float2* __restrict__ Gk = static_cast<const float2*>(t.G) + (size_t)k * t.gstride;
        const int m = m_base + (lane & 15), kk = lane >> 4;
#pragma unroll
        for (int s = 0; s < BP / 4; ++s) {
            const int n = 4 * s + kk;
            float2 g = make_float2(0.f, 0.f);
            if (active && m < b && n < b) g = gload(Gk + (size_t)m * b + n);
            ar[s] = g.x;
            ai[s] = g.y;
            as[s] = g.x + g.y;
        }
    }
    const int padn = BP - b;
    for (int e = threadIdx.x; e < NT * padn; e += 64 * WAVES) {
        const int w = e / padn, n = b + (e - w * padn);
        xs[w * ldx + 2 * n] = 0.f;
        xs[w * ldx + 2 * n + 1] = 0.f;
    }
    const float2* __restrict__ Xk = static_cast<const float2*>(t.X) + (size_t)k * W * b;
    float2* __restrict__ Yk = static_cast<float2*>(t.Y) + (size_t)k * W * b;
    const int j = lane & 15, q = lane >> 4;
    float2 pre[PF];
    auto fetch = [&](int w0) {
        const int have = min(NT, W - w0) * b;
        const float2* __restrict__ src = Xk + (size_t)w0 * b;
#pragma unroll
        for (int i = 0; i < PF; ++i) {
            const int e = threadIdx.x + i * 64 * WAVES;
            pre[i] = e < have ? gload(src + e) : make_float2(0.f, 0.f);
        }
    };
    fetch(0);
    for (int w0 = 0; w0 < W; w0 += NT) {
        __syncthreads();
#pragma unroll
        for (int i = 0; i < PF; ++i) {
            const int e = threadIdx.x + i * 64 * WAVES;
            if (e < NT * b) {
                const int w = e / b, n = e - w * b;
                *reinterpret_cast<float2*>(&xs[w * ldx + 2 * n]) = pre[i];
            }
        }
        __syncthreads();
        if (w0 + NT < W) fetch(w0 + NT);
        if (active) {
            floatx4 t1[NT / 16], t2[NT / 16], t3[NT / 16];
#pragma unroll
            for (int cg = 0; cg < NT / 16; ++cg) {
                t1[cg] = floatx4{0, 0, 0, 0};
                t2[cg] = floatx4{0, 0, 0, 0};
                t3[cg] = floatx4{0, 0, 0, 0};
            }
#pragma unroll
            for (int s = 0; s < BP / 4; ++s) {
#pragma unroll
                for (int cg = 0; cg < NT / 16; ++cg) {
                    const float2 u = *reinterpret_cast<const float2*>(&xs[(cg * 16 + j) * ldx + 2 * (4 * s + q)]);
                    t1[cg] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[s], u.x, t1[cg], 0, 0, 0);
                    t2[cg] = __builtin_amdgcn_mfma_f32_16x16x4f32(ai[s], u.y, t2[cg], 0, 0, 0);
                    t3[cg] = __builtin_amdgcn_mfma_f32_16x16x4f32(as[s], u.x + u.y, t3[cg], 0, 0, 0);
                }
            }
            // lane holds complex rows m_base + 4q + r (r = 0..3) of column j
#pragma unroll
            for (int cg = 0; cg < NT / 16; ++cg) {
                const int w = w0 + cg * 16 + j;
                if (w < W) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int m = m_base + 4 * q + r;
                        if (m < b) {
                            const float re = t1[cg][r] - t2[cg][r];
                            const float im = t3[cg][r] - t1[cg][r] - t2[cg][r];
                            gstore(Yk + (size_t)w * b + m, make_float2(re, im));
                        }
                    }
                }
            }
        }
    }
}

typedef float mlfft_f4v __attribute__((ext_vector_type(4)));
// two consecutive complex values with one 16-byte global store (p 16-byte aligned)
__device__ __forceinline__ void gstore2(float2* p, float2 a, float2 b) {
    *(MLFFT_GLOBAL mlfft_f4v*)p = mlfft_f4v{a.x, a.y, b.x, b.y};
}

// Three-product form with a flat assignment of work to waves.  The K * ns
// (frequency, 16-row slice) items of a task, ns = ceil(b / 16), are dealt to
// the waves of consecutive workgroups, WAVES (eight or four) per workgroup, so
// that no wave is idle whatever ns is (with one workgroup per frequency row
// group, b = 200 has 13 slices for 16 wave slots).  A workgroup then spans at
// most two frequencies and stages the X tiles of both; Gr + Gi is formed from
// the register-resident Gr, Gi fragments at each reduction step.  Eight waves
// fill a CU with one workgroup; four waves with 16-column tiles leave room for
// two, so one's tile staging overlaps the other's products.
template<int BP, int NT, int TAG, int DB, int WAVES = 8>
__global__ void __launch_bounds__(64 * WAVES, 2) bgemm_f32_3m_flat_kernel(GemmTask t0, const GemmTask* tasks, int ntasks) {
    constexpr int NTH = 64 * WAVES;
    constexpr int PF = (NT * BP + NTH - 1) / NTH;      // prefetched complex values per thread and panel
    extern __shared__ unsigned char smem_raw[];
    float* xs = reinterpret_cast<float*>(smem_raw);     // [buffer][panel][NT][ldx]
    const GemmTask t = ntasks > 0 ? *find_gemm_task(tasks, ntasks) : t0;
    const int b = t.b, W = t.W, K = t.K;
    const int ns = (b + 15) >> 4;
    const int total = K * ns;
    const int nwg = (total + WAVES - 1) / WAVES;
    const int local = blockIdx.x - t.block_begin;
    // consecutive slice groups on one XCD, so the workgroups sharing a frequency share its L2
    const int per = nwg >> 3;
    const int grp = local < per * 8 ? (local & 7) * per + (local >> 3) : local;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int gs0 = grp * WAVES;
    const int kA = gs0 / ns;
    const int kB = min((gs0 + WAVES - 1) / ns, K - 1);
    const int npan = kB != kA ? 2 : 1;
    const int gs = gs0 + wave;
    const bool active = gs < total;
    const int kw = active ? gs / ns : kA;
    const int m_base = (gs - kw * ns) * 16;
    const int pan = kw - kA;
    // every row of the wave's slice exists and rows of an even b keep 16-byte alignment
    const bool full16 = m_base + 16 <= b && (b & 1) == 0;
    const int ldx = 2 * BP + 2;
    float ar[BP / 4], ai[BP / 4];
    {
        const float2* __restrict__ Gk = static_cast<const float2*>(t.G) + (size_t)kw * t.gstride;
        const int m = m_base + (lane & 15), kk = lane >> 4;
#pragma unroll
        for (int s = 0; s < BP / 4; ++s) {
            const int n = 4 * s + kk;
            float2 g = make_float2(0.f, 0.f);
            if (active && m < b && n < b) g = gload(Gk + (size_t)m * b + n);
            ar[s] = g.x;
            ai[s] = g.y;
        }
    }
    const int padn = BP - b;
    for (int e = threadIdx.x; e < (DB ? 4 : 2) * NT * padn; e += NTH) {
        const int pw = e / padn, n = b + (e - pw * padn);
        xs[pw * ldx + 2 * n] = 0.f;
        xs[pw * ldx + 2 * n + 1] = 0.f;
    }
    const int tile = NT * b;
    const float2* __restrict__ Xa = static_cast<const float2*>(t.X) + (size_t)kA * W * b;
    const float2* __restrict__ Xb = static_cast<const float2*>(t.X) + (size_t)kB * W * b;
    float2* __restrict__ Yk = static_cast<float2*>(t.Y) + (size_t)kw * W * b;
    const int j = lane & 15, q = lane >> 4;
    float2 pre[2 * PF];
    auto fetch = [&](int w0) {
        const int have = min(NT, W - w0) * b;
#pragma unroll
        for (int i = 0; i < 2 * PF; ++i) {
            const int e = threadIdx.x + (i % PF) * NTH;
            const int p = i / PF;
            const float2* __restrict__ src = (p ? Xb : Xa) + (size_t)w0 * b;
            pre[i] = (p < npan && e < have) ? gload(src + e) : make_float2(0.f, 0.f);
        }
    };
    auto stage = [&](float* buf) {
#pragma unroll
        for (int i = 0; i < 2 * PF; ++i) {
            const int e = threadIdx.x + (i % PF) * NTH;
            const int p = i / PF;
            if (p < npan && e < tile) {
                const int w = e / b, n = e - w * b;
                *reinterpret_cast<float2*>(&buf[(p * NT + w) * ldx + 2 * n]) = pre[i];
            }
        }
    };
    const int bufsz = 2 * NT * ldx;
    fetch(0);
    if (DB) {
        // double buffering: tile t+1 is stored into the other buffer while tile t is
        // multiplied, one barrier per tile
        __syncthreads();                      // padding zeroed
        stage(xs);
        if (NT < W) fetch(NT);
        __syncthreads();
    }
    for (int w0 = 0, it = 0; w0 < W; w0 += NT, ++it) {
        const float* cur = xs + (DB ? (it & 1) * bufsz : 0);
        if (!DB) {
            __syncthreads();
            stage(xs);
            __syncthreads();
            if (w0 + NT < W) fetch(w0 + NT);
        }
        if (active) {
            const float* __restrict__ xp = cur + pan * NT * ldx;
            floatx4 t1[NT / 16], t2[NT / 16], t3[NT / 16];
#pragma unroll
            for (int cg = 0; cg < NT / 16; ++cg) {
                t1[cg] = floatx4{0, 0, 0, 0};
                t2[cg] = floatx4{0, 0, 0, 0};
                t3[cg] = floatx4{0, 0, 0, 0};
            }
#pragma unroll
            for (int s = 0; s < BP / 4; ++s) {
                const float as = ar[s] + ai[s];
#pragma unroll
                for (int cg = 0; cg < NT / 16; ++cg) {
                    const float2 u = *reinterpret_cast<const float2*>(&xp[(cg * 16 + j) * ldx + 2 * (4 * s + q)]);
                    t1[cg] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[s], u.x, t1[cg], 0, 0, 0);
                    t2[cg] = __builtin_amdgcn_mfma_f32_16x16x4f32(ai[s], u.y, t2[cg], 0, 0, 0);
                    t3[cg] = __builtin_amdgcn_mfma_f32_16x16x4f32(as, u.x + u.y, t3[cg], 0, 0, 0);
                }
            }
#pragma unroll
            for (int cg = 0; cg < NT / 16; ++cg) {
                const int w = w0 + cg * 16 + j;
                if (w < W) {
                    float2 o[4];
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        o[r] = make_float2(t1[cg][r] - t2[cg][r], t3[cg][r] - t1[cg][r] - t2[cg][r]);
                    const int m0 = m_base + 4 * q;
                    float2* dst = Yk + (size_t)w * b + m0;
                    if (full16) {
                        // the lane's four rows are 32 contiguous bytes: two 16-byte stores
                        gstore2(dst, o[0], o[1]);
                        gstore2(dst + 2, o[2], o[3]);
                    } else {
#pragma unroll
                        for (int r = 0; r < 4; ++r)
                            if (m0 + r < b) gstore(dst + r, o[r]);
                    }
                }
            }
        }
        if (DB) {
            if (w0 + NT < W) {
                stage(xs + ((it + 1) & 1) * bufsz);
                if (w0 + 2 * NT < W) fetch(w0 + 2 * NT);
            }
            __syncthreads();
        }
    }
}

// The FP32 three-product flat kernel with the X tiles loaded straight into LDS
// (global_load_lds_dwordx4, gfx950): no staging registers and no LDS stores, so
// the next tile's loads run under the current tile's products with one barrier per
// tile.  Eight waves, 16-column tiles, double-buffered, even b only (a lane moves
// two consecutive complex values, which must not cross a column).
//  - LDS rows hold RS = BP + 2 complex values; RS / 2 is odd, so the 16-byte B
//    fragment reads of eight consecutive lanes fall on distinct banks.
//  - The reduction runs in pair steps: sub-step e of pair step s2 takes n = 8 s2 +
//    2 q + e in lane group q, so one 16-byte read feeds two sub-steps (six MFMAs).
//  - A lane's 16-byte slots in a tile are fixed, so their source offsets are
//    computed once; pairs past b / 2 of a row are never loaded and stay zero.
//  - The products of a tile leave after the barrier that ends the tile, and the
//    wait before that barrier (one counter covers loads and stores) then covers
//    stores issued a whole tile earlier.
// LDS row length (complex values) of the direct-tile kernel
__host__ __device__ constexpr int f32_direct_rs(int bp) { return bp + 2; }

template<int BP, int TAG>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2, 2))) bgemm_f32_3m_direct_kernel(GemmTask t0, const GemmTask* tasks, int ntasks) {
    constexpr int WAVES = 8, NTH = 512, NT = 16;
    constexpr int RS = f32_direct_rs(BP);               // complex values per LDS row
    constexpr int HP = RS / 2;                          // 16-byte pairs per row
    constexpr int TILE = NT * RS;                       // complex values per (buffer, panel)
    constexpr int CHUNKS = (NT * HP + 63) / 64;         // 64-pair chunks per tile
    constexpr int CPW = (CHUNKS + WAVES - 1) / WAVES;   // chunks per wave and tile
    static_assert(HP % 2 == 1, "row pairs must be odd");
    extern __shared__ unsigned char smem_raw[];
    float2* xs = reinterpret_cast<float2*>(smem_raw);   // [buffer][panel][NT][RS]
    const GemmTask t = ntasks > 0 ? *find_gemm_task(tasks, ntasks) : t0;
    const int b = t.b, W = t.W, K = t.K;
    const int ns = (b + 15) >> 4;
    const int total = K * ns;
    const int nwg = (total + WAVES - 1) / WAVES;
    const int local = blockIdx.x - t.block_begin;
    const int per = nwg >> 3;
    const int grp = local < per * 8 ? (local & 7) * per + (local >> 3) : local;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int gs0 = grp * WAVES;
    const int kA = gs0 / ns;
    const int kB = min((gs0 + WAVES - 1) / ns, K - 1);
    const int npan = kB != kA ? 2 : 1;
    const int gs = gs0 + wave;
    const bool active = gs < total;
    const int kw = active ? gs / ns : kA;
    const int m_base = (gs - kw * ns) * 16;
    const int pan = kw - kA;
    const bool full16 = m_base + 16 <= b;
    const int j = lane & 15, q = lane >> 4;
    // stationary fragments: Re G, Im G and Re G + Im G (the third product's operand)
    float ar[BP / 4], ai[BP / 4], as[BP / 4];
    {
        const float2* __restrict__ Gk = static_cast<const float2*>(t.G) + (size_t)kw * t.gstride;
        const int m = m_base + j;
#pragma unroll
        for (int s2 = 0; s2 < BP / 8; ++s2) {
            const int n = 8 * s2 + 2 * q;
            mlfft_f4v g = mlfft_f4v{0.f, 0.f, 0.f, 0.f};
            if (active && m < b && n < b) g = *(const MLFFT_GLOBAL mlfft_f4v*)(Gk + (size_t)m * b + n);
            ar[2 * s2] = g[0];
            ai[2 * s2] = g[1];
            ar[2 * s2 + 1] = g[2];
            ai[2 * s2 + 1] = g[3];
        }
#pragma unroll
        for (int s = 0; s < BP / 4; ++s) as[s] = ar[s] + ai[s];
    }
    // both buffers and panels zeroed once: the pairs past b / 2 of every row are padding
    {
        mlfft_f4v* z = reinterpret_cast<mlfft_f4v*>(xs);
        for (int e = threadIdx.x; e < 2 * TILE; e += NTH) z[e] = mlfft_f4v{0.f, 0.f, 0.f, 0.f};
    }
    // source offsets (complex values from the tile's first column) of this lane's slots
    int soff[CPW];
#pragma unroll
    for (int c = 0; c < CPW; ++c) {
        const int ch = wave + WAVES * c;
        const int slot = ch * 64 + lane;
        const int row = slot / HP, p = slot - row * HP;
        soff[c] = (ch < CHUNKS && row < NT && 2 * p < b) ? row * b + 2 * p : -1;
    }
    const float2* __restrict__ Xa = static_cast<const float2*>(t.X) + (size_t)kA * W * b;
    const float2* __restrict__ Xb = static_cast<const float2*>(t.X) + (size_t)kB * W * b;
    float2* __restrict__ Yk = static_cast<float2*>(t.Y) + (size_t)kw * W * b;
    auto load_tile = [&](int w0, int buf) {
        const int lim = min(NT, W - w0) * b;             // the columns of a last, partial tile
#pragma unroll
        for (int pn = 0; pn < 2; ++pn) {
            if (pn >= npan) break;
            const float2* __restrict__ src = (pn ? Xb : Xa) + (size_t)w0 * b;
            float2* dst = xs + (buf * 2 + pn) * TILE;
#pragma unroll
            for (int c = 0; c < CPW; ++c) {
                const int ch = wave + WAVES * c;
                if (ch < CHUNKS && soff[c] >= 0 && soff[c] < lim)
                    __builtin_amdgcn_global_load_lds(
                        (const void*)(src + soff[c]),
                        (__attribute__((address_space(3))) void*)(dst + ch * 128), 16, 0, 0);
            }
        }
    };
    float2 o[4];
    auto store = [&](int w0) {
        const int w = w0 + j;
        if (w < W) {
            const int m0 = m_base + 4 * q;
            float2* dst = Yk + (size_t)w * b + m0;
            if (full16) {
                gstore2(dst, o[0], o[1]);
                gstore2(dst + 2, o[2], o[3]);
            } else {
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    if (m0 + r < b) gstore(dst + r, o[r]);
            }
        }
    };
    __syncthreads();                                     // zeroing done before any tile lands
    load_tile(0, 0);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    for (int w0 = 0, it = 0; w0 < W; w0 += NT, ++it) {
        // the next tile's loads are issued after the first pair step, so the MFMA pipes
        // already have work while the wave issues them
        auto next = [&]() { if (w0 + NT < W) load_tile(w0 + NT, (it + 1) & 1); };
        if (!active) next();
        if (active) {
            const float2* __restrict__ xp = xs + ((it & 1) * 2 + pan) * TILE + j * RS + 2 * q;
            floatx4 t1 = floatx4{0, 0, 0, 0}, t2 = floatx4{0, 0, 0, 0}, t3 = floatx4{0, 0, 0, 0};
            // B fragments read two pair steps ahead of their products
            mlfft_f4v u0 = *reinterpret_cast<const mlfft_f4v*>(xp);
            mlfft_f4v u1 = *reinterpret_cast<const mlfft_f4v*>(xp + 8);
#pragma unroll
            for (int s2 = 0; s2 < BP / 8; ++s2) {
                const mlfft_f4v u = u0;
                u0 = u1;
                if (s2 + 2 < BP / 8) u1 = *reinterpret_cast<const mlfft_f4v*>(xp + 8 * (s2 + 2));
                if (s2 == 1) next();
                t1 = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[2 * s2], u[0], t1, 0, 0, 0);
                t2 = __builtin_amdgcn_mfma_f32_16x16x4f32(ai[2 * s2], u[1], t2, 0, 0, 0);
                t3 = __builtin_amdgcn_mfma_f32_16x16x4f32(as[2 * s2], u[0] + u[1], t3, 0, 0, 0);
                t1 = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[2 * s2 + 1], u[2], t1, 0, 0, 0);
                t2 = __builtin_amdgcn_mfma_f32_16x16x4f32(ai[2 * s2 + 1], u[3], t2, 0, 0, 0);
                t3 = __builtin_amdgcn_mfma_f32_16x16x4f32(as[2 * s2 + 1], u[2] + u[3], t3, 0, 0, 0);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) o[r] = make_float2(t1[r] - t2[r], t3[r] - t1[r] - t2[r]);
        }
        __builtin_amdgcn_s_waitcnt(0);                   // the next tile has landed
        __syncthreads();
        if (active) store(w0);
    }
}

// FP64 three-product form with the flat assignment, four waves per workgroup.
// Same scheme as the FP32 kernel above with v_mfma_f64_16x16x4f64, whose
// accumulator holds row 4r + l/16 of column l%16 in register r.  Four waves of
// one slice each keep Gr and Gi (BP/2 doubles per lane) in registers, one wave
// per SIMD; four consecutive slices span at most two frequencies when
// ceil(b/16) >= 3.
template<int BP, int NT, int TAG>
__global__ void __launch_bounds__(256) bgemm_f64_3m_flat_kernel(GemmTask t0, const GemmTask* tasks, int ntasks) {
    constexpr int WAVES = 4, NTH = 64 * WAVES;
    constexpr int PF = (NT * BP + NTH - 1) / NTH;
    extern __shared__ unsigned char smem_raw[];
    double* xs = reinterpret_cast<double*>(smem_raw);     // [panel][NT][ldx]
    const GemmTask t = ntasks > 0 ? *find_gemm_task(tasks, ntasks) : t0;
    const int b = t.b, W = t.W, K = t.K;
    const int ns = (b + 15) >> 4;
    const int total = K * ns;
    const int nwg = (total + WAVES - 1) / WAVES;
    const int local = blockIdx.x - t.block_begin;
    const int per = nwg >> 3;
    const int grp = local < per * 8 ? (local & 7) * per + (local >> 3) : local;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int gs0 = grp * WAVES;
    const int kA = gs0 / ns;
    const int kB = min((gs0 + WAVES - 1) / ns, K - 1);
    const int npan = kB != kA ? 2 : 1;
    const int gs = gs0 + wave;
    const bool active = gs < total;
    const int kw = active ? gs / ns : kA;
    const int m_base = (gs - kw * ns) * 16;
    const int pan = kw - kA;
    const int ldx = 2 * BP + 2;
    double ar[BP / 4], ai[BP / 4];
    {
        const double2* __restrict__ Gk = static_cast<const double2*>(t.G) + (size_t)kw * t.gstride;
        const int m = m_base + (lane & 15), kk = lane >> 4;
#pragma unroll
        for (int s = 0; s < BP / 4; ++s) {
            const int n = 4 * s + kk;
            double2 g = make_double2(0.0, 0.0);
            if (active && m < b && n < b) g = gload(Gk + (size_t)m * b + n);
            ar[s] = g.x;
            ai[s] = g.y;
        }
    }
    const int padn = BP - b;
    for (int e = threadIdx.x; e < 2 * NT * padn; e += NTH) {
        const int pw = e / padn, n = b + (e - pw * padn);
        xs[pw * ldx + 2 * n] = 0.0;
        xs[pw * ldx + 2 * n + 1] = 0.0;
    }
    const int tile = NT * b;
    const double2* __restrict__ Xa = static_cast<const double2*>(t.X) + (size_t)kA * W * b;
    const double2* __restrict__ Xb = static_cast<const double2*>(t.X) + (size_t)kB * W * b;
    double2* __restrict__ Yk = static_cast<double2*>(t.Y) + (size_t)kw * W * b;
    const int j = lane & 15, q = lane >> 4;
    double2 pre[2 * PF];
    auto fetch = [&](int w0) {
        const int have = min(NT, W - w0) * b;
#pragma unroll
        for (int i = 0; i < 2 * PF; ++i) {
            const int e = threadIdx.x + (i % PF) * NTH;
            const int p = i / PF;
            const double2* __restrict__ src = (p ? Xb : Xa) + (size_t)w0 * b;
            pre[i] = (p < npan && e < have) ? gload(src + e) : make_double2(0.0, 0.0);
        }
    };
    // The products of a tile are stored one step late, after the loads of the
    // next tile's prefetch have been issued: the wait for that prefetch (one
    // counter covers loads and stores) then finds these stores long complete
    // instead of waiting for stores issued just before it.
    doublex4 t1[NT / 16], t2[NT / 16], t3[NT / 16];
    int wdone = -1;
    auto store = [&]() {
#pragma unroll
        for (int cg = 0; cg < NT / 16; ++cg) {
            const int w = wdone + cg * 16 + j;
            if (w < W) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int m = m_base + 4 * r + q;
                    if (m < b) {
                        const double re = t1[cg][r] - t2[cg][r];
                        const double im = t3[cg][r] - t1[cg][r] - t2[cg][r];
                        gstore(Yk + (size_t)w * b + m, make_double2(re, im));
                    }
                }
            }
        }
        wdone = -1;
    };
    fetch(0);
    // Everything loaded so far (the stationary G fragments and the first tile) is
    // waited for here, once: otherwise the compiler's wait before the first use
    // of a G fragment inside the loop covers the loads of the next tile too, and
    // the prefetch never overlaps the products.
    __builtin_amdgcn_s_waitcnt(0);
    for (int w0 = 0; w0 < W; w0 += NT) {
        __syncthreads();
#pragma unroll
        for (int i = 0; i < 2 * PF; ++i) {
            const int e = threadIdx.x + (i % PF) * NTH;
            const int p = i / PF;
            if (p < npan && e < tile) {
                const int w = e / b, n = e - w * b;
                *reinterpret_cast<double2*>(&xs[(p * NT + w) * ldx + 2 * n]) = pre[i];
            }
        }
        __syncthreads();
        if (w0 + NT < W) fetch(w0 + NT);
        if (active) {
            if (wdone >= 0) store();
            const double* __restrict__ xp = xs + pan * NT * ldx;
#pragma unroll
            for (int cg = 0; cg < NT / 16; ++cg) {
                t1[cg] = doublex4{0, 0, 0, 0};
                t2[cg] = doublex4{0, 0, 0, 0};
                t3[cg] = doublex4{0, 0, 0, 0};
            }
#pragma unroll
            for (int s = 0; s < BP / 4; ++s) {
                const double as = ar[s] + ai[s];
#pragma unroll
                for (int cg = 0; cg < NT / 16; ++cg) {
                    const double2 u = *reinterpret_cast<const double2*>(&xp[(cg * 16 + j) * ldx + 2 * (4 * s + q)]);
                    t1[cg] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[s], u.x, t1[cg], 0, 0, 0);
                    t2[cg] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[s], u.y, t2[cg], 0, 0, 0);
                    t3[cg] = __builtin_amdgcn_mfma_f64_16x16x4f64(as, u.x + u.y, t3[cg], 0, 0, 0);
                }
            }
            wdone = w0;
        }
    }
    if (active && wdone >= 0) store();
}

// LDS row length (complex values) of a half-reduction tile of the FP64 direct-tile
// kernel: odd, so the 16-byte B-fragment reads of eight lanes fall on distinct banks
__host__ __device__ constexpr int f64_direct_rs(int bp) { return bp / 2 + 1; }

// The FP64 three-product flat kernel with X tiles loaded straight into LDS
// (global_load_lds_dwordx4, one complex value per lane), four waves (one per SIMD,
// so that Gr and Gi of a 16-row slice, 2 b' doubles per lane, stay in registers)
// of one 16-row slice each.  A 16-column tile of two panels would not fit in LDS
// twice, so each tile is split into the two halves of the reduction, which take
// turns in the two buffers: the loads of one half run under the products of the
// other, with one wait and one barrier per half.  The products of a tile leave
// after the barrier that ends it (covered by the next wait, a half-tile later).
template<int BP, int TAG>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1))) bgemm_f64_3m_direct_kernel(GemmTask t0, const GemmTask* tasks, int ntasks) {
    constexpr int WAVES = 4, NT = 16;
    constexpr int HB = BP / 2;                          // reduction length of a half
    constexpr int RS = f64_direct_rs(BP);               // complex values per LDS row
    constexpr int TILE = NT * RS;                       // complex values per (buffer, panel)
    constexpr int CHUNKS = (TILE + 63) / 64;            // 64-value chunks per half tile
    constexpr int CPW = (CHUNKS + WAVES - 1) / WAVES;   // chunks per wave
    constexpr int SH = HB / 4;                          // reduction steps per half
    static_assert(HB % 4 == 0 && RS % 2 == 1, "half tiles of whole steps, odd rows");
    extern __shared__ unsigned char smem_raw[];
    double2* xs = reinterpret_cast<double2*>(smem_raw);  // [buffer = half][panel][NT][RS]
    const GemmTask t = ntasks > 0 ? *find_gemm_task(tasks, ntasks) : t0;
    const int b = t.b, W = t.W, K = t.K;
    const int ns = (b + 15) >> 4;
    const int total = K * ns;
    const int nwg = (total + WAVES - 1) / WAVES;
    const int local = blockIdx.x - t.block_begin;
    const int per = nwg >> 3;
    const int grp = local < per * 8 ? (local & 7) * per + (local >> 3) : local;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int gs0 = grp * WAVES;
    const int kA = gs0 / ns;
    const int kB = min((gs0 + WAVES - 1) / ns, K - 1);
    const int npan = kB != kA ? 2 : 1;
    const int gs = gs0 + wave;
    const bool active = gs < total;
    const int kw = active ? gs / ns : kA;
    const int m_base = (gs - kw * ns) * 16;
    const int pan = kw - kA;
    const int j = lane & 15, q = lane >> 4;
    double ar[BP / 4], ai[BP / 4];
    {
        const double2* __restrict__ Gk = static_cast<const double2*>(t.G) + (size_t)kw * t.gstride;
        const int m = m_base + j;
#pragma unroll
        for (int s = 0; s < BP / 4; ++s) {
            const int n = 4 * s + q;
            double2 g = make_double2(0.0, 0.0);
            if (active && m < b && n < b) g = gload(Gk + (size_t)m * b + n);
            ar[s] = g.x;
            ai[s] = g.y;
        }
    }
    {
        mlfft_d2v* z = reinterpret_cast<mlfft_d2v*>(xs);
        for (int e = threadIdx.x; e < 4 * TILE; e += WAVES * 64) z[e] = mlfft_d2v{0.0, 0.0};
    }
    // source offsets (from the half's first value in the tile's first column) of this
    // lane's slots, and which slots hold reduction indices below b in each half
    const int nv0 = min(HB, b), nv1 = max(0, b - HB);
    int soff[CPW];
    unsigned vm0 = 0, vm1 = 0;
#pragma unroll
    for (int c = 0; c < CPW; ++c) {
        const int ch = wave + WAVES * c;
        const int slot = ch * 64 + lane;
        const int row = slot / RS, p = slot - row * RS;
        const bool ok = ch < CHUNKS && row < NT && p < HB;
        soff[c] = ok ? row * b + p : -1;
        vm0 |= (ok && p < nv0 ? 1u : 0u) << c;
        vm1 |= (ok && p < nv1 ? 1u : 0u) << c;
    }
    const double2* __restrict__ Xa = static_cast<const double2*>(t.X) + (size_t)kA * W * b;
    const double2* __restrict__ Xb = static_cast<const double2*>(t.X) + (size_t)kB * W * b;
    double2* __restrict__ Yk = static_cast<double2*>(t.Y) + (size_t)kw * W * b;
    auto load_half = [&](int w0, int h) {
        const int lim = min(NT, W - w0) * b;
        const unsigned vm = h ? vm1 : vm0;
#pragma unroll
        for (int pn = 0; pn < 2; ++pn) {
            if (pn >= npan) break;
            const double2* __restrict__ src = (pn ? Xb : Xa) + (size_t)w0 * b + h * HB;
            double2* dst = xs + (h * 2 + pn) * TILE;
#pragma unroll
            for (int c = 0; c < CPW; ++c) {
                const int ch = wave + WAVES * c;
                if (ch < CHUNKS && ((vm >> c) & 1u) && soff[c] < lim)
                    __builtin_amdgcn_global_load_lds(
                        (const void*)(src + soff[c]),
                        (__attribute__((address_space(3))) void*)(dst + ch * 64), 16, 0, 0);
            }
        }
    };
    doublex4 t1, t2, t3;
    // the products of one half; the other buffer's loads are issued after the first two
    // steps, so the MFMA pipes already have work while the wave issues them
    auto products = [&](int h, auto issue) {
        const double2* xp = xs + (h * 2 + pan) * TILE + j * RS + q;
        // B fragments read two steps ahead: with one wave per SIMD nothing else hides
        // the LDS latency behind the three products of a step
        mlfft_d2v u0 = *reinterpret_cast<const mlfft_d2v*>(xp);
        mlfft_d2v u1 = *reinterpret_cast<const mlfft_d2v*>(xp + 4);
#pragma unroll
        for (int s2 = 0; s2 < SH; ++s2) {
            const int s = (h ? SH : 0) + s2;
            const mlfft_d2v u = u0;
            u0 = u1;
            if (s2 + 2 < SH) u1 = *reinterpret_cast<const mlfft_d2v*>(xp + 4 * (s2 + 2));
            t1 = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[s], u[0], t1, 0, 0, 0);
            t2 = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[s], u[1], t2, 0, 0, 0);
            t3 = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[s] + ai[s], u[0] + u[1], t3, 0, 0, 0);
            if (s2 == (SH > 2 ? 1 : 0)) issue();
        }
    };
    double2 o[4];
    auto store = [&](int w0) {
        const int w = w0 + j;
        if (w < W) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = m_base + 4 * r + q;
                if (m < b) gstore(Yk + (size_t)w * b + m, o[r]);
            }
        }
    };
    __syncthreads();                                     // zeroing done before any tile lands
    load_half(0, 0);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    for (int w0 = 0; w0 < W; w0 += NT) {
        auto next1 = [&]() { load_half(w0, 1); };
        auto next0 = [&]() { if (w0 + NT < W) load_half(w0 + NT, 0); };
        if (active) {
            t1 = doublex4{0, 0, 0, 0};
            t2 = doublex4{0, 0, 0, 0};
            t3 = doublex4{0, 0, 0, 0};
            products(0, next1);
        } else {
            next1();
        }
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (active) {
            products(1, next0);
#pragma unroll
            for (int r = 0; r < 4; ++r) o[r] = make_double2(t1[r] - t2[r], t3[r] - t1[r] - t2[r]);
        } else {
            next0();
        }
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (active) store(w0);
    }
}

// ------------------------------------------------------------------ BF16

typedef unsigned int mlfft_u2v __attribute__((ext_vector_type(2)));

// p (wave-uniform) through an empty asm statement: the compiler can neither hoist nor
// precompute addresses derived from the result
template<typename T>
__device__ __forceinline__ const T* opaque_uniform(const T* p) {
    const uint64_t v = reinterpret_cast<uint64_t>(p);
    uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    asm volatile("" : "+s"(lo), "+s"(hi));
    return reinterpret_cast<const T*>(((uint64_t)hi << 32) | lo);
}

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
                if (active && m < b && n < b) g = gload(Gk + (size_t)m * b + n);
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
            const float2 v = e < have ? gload(src + e) : make_float2(0.f, 0.f);
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
                    if (m < b) gstore(Yk + (size_t)w * b + m, make_float2(acc[cg][0], acc[cg][1]));
                    if (m + 1 < b) gstore(Yk + (size_t)w * b + m + 1, make_float2(acc[cg][2], acc[cg][3]));
                }
            }
        }
    }
}


// BF16 inputs, FP32 accumulation, with the flat assignment of the FP32
// three-product kernel: K * ceil(b/16) (frequency, 16-row slice) items dealt to
// the WAVES waves of a workgroup (eight with 32-column tiles, or four with
// 16-column tiles so that two workgroups share a CU), at most two frequencies
// per workgroup, X tiles double-buffered
// through LDS with the next tile prefetched in registers.  The complex product
// runs as a real one of twice the size: A row 2i is (Re G[m], -Im G[m]) and row
// 2i+1 is (Im G[m], Re G[m]) over the interleaved (Re X, Im X) reduction, so a
// 16-row MFMA tile covers eight complex rows and a wave's slice is two such
// halves, both kept in registers.  X is rounded to bf16 as it is staged (one
// packed (re, im) word per complex value), and each B fragment read from LDS
// feeds the products of both halves.  The lane's outputs of one half are rows
// m and m+1 (re, im, re, im) of one column: a single 16-byte store.
template<int BP, int NT, int TAG, int WAVES = 8>
__global__ void __launch_bounds__(64 * WAVES) bgemm_bf16_flat_kernel(GemmTask t0, const GemmTask* tasks, int ntasks) {
    constexpr int NTH = 64 * WAVES;
    constexpr int PF = (NT * BP + NTH - 1) / NTH;      // prefetched complex values per thread and panel
    constexpr int LDX = BP + 4;                        // packed words per LDS row (16-byte skew)
    extern __shared__ unsigned char smem_raw[];
    uint32_t* xs = reinterpret_cast<uint32_t*>(smem_raw);     // [buffer][panel][NT][LDX]
    const GemmTask t = ntasks > 0 ? *find_gemm_task(tasks, ntasks) : t0;
    const int b = t.b, W = t.W, K = t.K;
    const int ns = (b + 15) >> 4;
    const int total = K * ns;
    const int nwg = (total + WAVES - 1) / WAVES;
    const int local = blockIdx.x - t.block_begin;
    // consecutive slice groups on one XCD, so the workgroups sharing a frequency share its L2
    const int per = nwg >> 3;
    const int grp = local < per * 8 ? (local & 7) * per + (local >> 3) : local;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int gs0 = grp * WAVES;
    const int kA = gs0 / ns;
    const int kB = min((gs0 + WAVES - 1) / ns, K - 1);
    const int npan = kB != kA ? 2 : 1;
    const int gs = gs0 + wave;
    const bool active = gs < total;
    const int kw = active ? gs / ns : kA;
    const int m_base = (gs - kw * ns) * 16;
    const int pan = kw - kA;
    const int j = lane & 15, q = lane >> 4;
    // A fragments of the two 8-row halves for all BP/16 reduction steps (16 complex columns each)
    ushortx8 a0[BP / 16], a1[BP / 16];
    {
        const uint32_t* __restrict__ Gk = static_cast<const uint32_t*>(t.G) + (size_t)kw * t.gstride;
        const int pr = j & 1;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int m = m_base + 8 * h + (j >> 1);
#pragma unroll
            for (int s = 0; s < BP / 16; ++s) {
                ushortx8 v;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int n = 16 * s + 4 * q + e;
                    uint32_t g = 0;
                    if (active && m < b && n < b) g = gload(Gk + (size_t)m * b + n);
                    const unsigned short gr = (unsigned short)(g & 0xffffu), gi = (unsigned short)(g >> 16);
                    if (pr == 0) { v[2 * e] = gr; v[2 * e + 1] = (unsigned short)(gi ^ 0x8000u); }
                    else         { v[2 * e] = gi; v[2 * e + 1] = gr; }
                }
                if (h == 0) a0[s] = v; else a1[s] = v;
            }
        }
    }
    // reduction padding n in [b, BP) of every row of both buffers and panels
    const int padn = BP - b;
    for (int e = threadIdx.x; e < 4 * NT * padn; e += NTH) {
        const int pw = e / padn, n = b + (e - pw * padn);
        xs[pw * LDX + n] = 0u;
    }
    const int tile = NT * b;
    const float2* __restrict__ Xa = static_cast<const float2*>(t.X) + (size_t)kA * W * b;
    const float2* __restrict__ Xb = static_cast<const float2*>(t.X) + (size_t)kB * W * b;
    float2* __restrict__ Yk = static_cast<float2*>(t.Y) + (size_t)kw * W * b;
    float2 pre[2 * PF];
    auto fetch = [&](int w0) {
        const int have = min(NT, W - w0) * b;
#pragma unroll
        for (int i = 0; i < 2 * PF; ++i) {
            const int e = threadIdx.x + (i % PF) * NTH;
            const int p = i / PF;
            const float2* __restrict__ src = (p ? Xb : Xa) + (size_t)w0 * b;
            pre[i] = (p < npan && e < have) ? gload(src + e) : make_float2(0.f, 0.f);
        }
    };
    auto stage = [&](uint32_t* buf) {
#pragma unroll
        for (int i = 0; i < 2 * PF; ++i) {
            const int e = threadIdx.x + (i % PF) * NTH;
            const int p = i / PF;
            if (p < npan && e < tile) {
                const int w = e / b, n = e - w * b;
                buf[(p * NT + w) * LDX + n] =
                    (uint32_t)f32_to_bf16_bits(pre[i].x) | ((uint32_t)f32_to_bf16_bits(pre[i].y) << 16);
            }
        }
    };
    const int bufsz = 2 * NT * LDX;
    const bool even_b = (b & 1) == 0;
    fetch(0);
    __syncthreads();                      // padding zeroed
    stage(xs);
    if (NT < W) fetch(NT);
    __syncthreads();
    for (int w0 = 0, it = 0; w0 < W; w0 += NT, ++it) {
        const uint32_t* cur = xs + (it & 1) * bufsz;
        if (active) {
            const uint32_t* __restrict__ xp = cur + pan * NT * LDX;
            floatx4 c0[NT / 16], c1[NT / 16];
#pragma unroll
            for (int cg = 0; cg < NT / 16; ++cg) {
                c0[cg] = floatx4{0, 0, 0, 0};
                c1[cg] = floatx4{0, 0, 0, 0};
            }
#pragma unroll
            for (int s = 0; s < BP / 16; ++s) {
#pragma unroll
                for (int cg = 0; cg < NT / 16; ++cg) {
                    const ushortx8 bv = *reinterpret_cast<const ushortx8*>(&xp[(cg * 16 + j) * LDX + 16 * s + 4 * q]);
                    c0[cg] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                        __builtin_bit_cast(bf16x8, a0[s]), __builtin_bit_cast(bf16x8, bv), c0[cg], 0, 0, 0);
                    c1[cg] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                        __builtin_bit_cast(bf16x8, a1[s]), __builtin_bit_cast(bf16x8, bv), c1[cg], 0, 0, 0);
                }
            }
#pragma unroll
            for (int cg = 0; cg < NT / 16; ++cg) {
                const int w = w0 + cg * 16 + j;
                if (w < W) {
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const floatx4 acc = h ? c1[cg] : c0[cg];
                        const int m = m_base + 8 * h + 2 * q;
                        float2* dst = Yk + (size_t)w * b + m;
                        const float2 y0 = make_float2(acc[0], acc[1]), y1 = make_float2(acc[2], acc[3]);
                        if (even_b && m + 1 < b) {
                            gstore2(dst, y0, y1);
                        } else {
                            if (m < b) gstore(dst, y0);
                            if (m + 1 < b) gstore(dst + 1, y1);
                        }
                    }
                }
            }
        }
        if (w0 + NT < W) {
            stage(xs + ((it + 1) & 1) * bufsz);
            if (w0 + 2 * NT < W) fetch(w0 + 2 * NT);
        }
        __syncthreads();
    }
}

// BF16 inputs, FP32 accumulation, one frequency per workgroup: the product of the
// preconditioner, which is bound by HBM (a bf16 ridge of 315 flop/B), so each X tile
// of a frequency is staged into LDS once and serves all ceil(b/16) row slices of
// that frequency.  The eight waves take slices w and w + 8; each keeps the two slices'
// A fragments in registers as separate real and imaginary planes (Re G, Im G: half the
// registers of the real-expanded form, which is what lets a wave hold two slices), and
// the tile is staged as Re X and -Im X planes (bf16 rounding is symmetric, so -Im X
// rounds to minus the rounded Im X).  A complex product is four MFMAs into two
// accumulators: Re Y = Re G Re X + Im G (-Im X), Im Y = Im G Re X + (-Re G)(-Im X),
// with -Re G formed by flipping sign bits.  The reduction runs over b padded to 32.
// Work items are (frequency, 32-column tile) pairs, item i being tile i % ntile of
// frequency i / ntile; a workgroup runs a contiguous range of items, one segment per
// frequency the range touches (the segment loads that frequency's fragments).
// RANGE == 0: the range is one of mgroups column chunks of one frequency (K * mgroups
// workgroups).  RANGE == 1: all K * ntile items are split evenly over mgroups
// workgroups, about one per CU, so that no partial last round of workgroups leaves CUs
// idle (30x30, b = 200: 900 frequencies of 29 tiles were 3.5 rounds of one-frequency
// workgroups).  X tiles are double-buffered with the next tile prefetched into
// registers; a lane's four output rows leave as two 16-byte stores.  PAIRS (every b
// even, spectra 16-byte aligned): a lane moves two consecutive values of a column.
// XB (with PAIRS): X holds bf16 (re, im) pairs already rounded by the transform that
// wrote it, so a value is 4 bytes read and nothing is converted.
template<int BP, int NT, int TAG, int RANGE, int PAIRS, int XB = 0>
__global__ void __launch_bounds__(512) bgemm_bf16_freq_kernel(GemmTask t0, const GemmTask* tasks, int ntasks) {
    constexpr int NTH = 512;
    constexpr int BP32 = (BP + 31) / 32 * 32;
    constexpr int S = BP32 / 32;                      // reduction steps of 32
    constexpr int LDX = BP32 + 8;                     // bf16 elements per LDS row (16-byte skew)
    constexpr int PF = (NT * BP + NTH - 1) / NTH;      // prefetched complex values per thread
    constexpr int PF2 = (NT * BP / 2 + NTH - 1) / NTH; // prefetched pairs per thread (even b)
    constexpr int PFA = PAIRS ? 2 * PF2 : PF;
    extern __shared__ unsigned char smem_raw[];
    unsigned short* xs = reinterpret_cast<unsigned short*>(smem_raw);   // [buffer][plane][NT][LDX]
    const GemmTask t = ntasks > 0 ? *find_gemm_task(tasks, ntasks) : t0;
    const int b = t.b, W = t.W, K = t.K;
    const int ntile = (W + NT - 1) / NT;
    const int local = blockIdx.x - t.block_begin;
    const int nwg = RANGE ? t.mgroups : K * t.mgroups;
    const int per = nwg >> 3;
    const int grp = local < per * 8 ? (local & 7) * per + (local >> 3) : local;
    // this workgroup's items [i0, i1): item i is column tile i % ntile of frequency i / ntile
    int i0, i1;
    if (RANGE) {
        const long long T = (long long)K * ntile;
        i0 = (int)(T * grp / nwg);
        i1 = (int)(T * (grp + 1) / nwg);
    } else {
        const int ncs = t.mgroups;
        const int k = grp / ncs, chunk = grp - k * ncs;
        const int tpc = (ntile + ncs - 1) / ncs;      // tiles per column chunk
        i0 = k * ntile + min(ntile, chunk * tpc);
        i1 = k * ntile + min(ntile, (chunk + 1) * tpc);
    }
    if (i0 >= i1) return;                             // uniform over the workgroup
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int j = lane & 15, q = lane >> 4;
    const int ns = (b + 15) >> 4;
    bool act[2];
    int mb[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        act[h] = wave + 8 * h < ns;
        mb[h] = (wave + 8 * h) * 16;
    }
    // reduction padding n in [b, BP32) of every row, both planes, both buffers
    const int padn = BP32 - b;
    for (int e = threadIdx.x; e < 4 * NT * padn; e += NTH) {
        const int row = e / padn, n = b + (e - row * padn);
        xs[row * LDX + n] = 0;
    }
    // one segment per frequency the range touches: its fragments, then its tiles
    for (int k = i0 / ntile; k * ntile < i1; ++k) {
    // b made opaque per segment: nothing derived from it (bounds tests, LDS offsets) is
    // hoisted out of the segment loop, where it would be live during the fragment loads
    int bk = __builtin_amdgcn_readfirstlane(b);
    asm volatile("" : "+s"(bk));
    const int wbeg = (max(i0, k * ntile) - k * ntile) * NT;
    const int wend = min(W, (min(i1, (k + 1) * ntile) - k * ntile) * NT);
    ushortx8 gr[2][S], gi[2][S];
    {
        // G's base made opaque, so that the bounds tests and addresses below are formed
        // per segment rather than hoisted out of the segment loop
        const uint32_t* __restrict__ Gk = opaque_uniform(static_cast<const uint32_t*>(t.G) + (size_t)k * t.gstride);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int m = mb[h] + j;
#pragma unroll
            for (int st = 0; st < S; ++st) {
                ushortx8 vr, vi;
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const int n = 32 * st + 8 * q + e;
                    uint32_t g = 0;
                    if (act[h] && m < bk && n < bk) g = gload(Gk + (size_t)m * bk + n);
                    vr[e] = (unsigned short)(g & 0xffffu);
                    vi[e] = (unsigned short)(g >> 16);
                }
                gr[h][st] = vr;
                gi[h][st] = vi;
            }
        }
    }
    const float2* __restrict__ Xk = static_cast<const float2*>(t.X) + (size_t)k * W * bk;
    float2* __restrict__ Yk = static_cast<float2*>(t.Y) + (size_t)k * W * bk;
    const int plane = NT * LDX, bufsz = 2 * plane;
    const bool even_b = (bk & 1) == 0;
    // PAIRS (every b even, spectra 16-byte aligned): a lane moves two consecutive complex
    // values of one column (one 16-byte load, one 4-byte LDS store per plane); otherwise
    // one value
    constexpr bool pairs = PAIRS != 0;
    float2 pre[PFA];
    auto fetch = [&](int w0) {
        const int have = min(NT, wend - w0) * bk;
        // the tile's base made opaque, so that the per-load addresses are formed at each
        // fetch rather than hoisted out of the tile loop into registers of their own
        const float2* __restrict__ src = opaque_uniform(Xk + (size_t)w0 * bk);
        if constexpr (XB != 0) {
            // X already in bf16 (re, im) pairs: a lane loads two values as two 32-bit words,
            // kept bit for bit in a prefetch slot
            const mlfft_u2v* __restrict__ s16 = opaque_uniform(static_cast<const mlfft_u2v*>(t.X) +
                                                               (((size_t)k * W + w0) * bk >> 1));
#pragma unroll
            for (int i = 0; i < PF2; ++i) {
                const int e = 2 * (threadIdx.x + i * NTH);
                mlfft_u2v v = mlfft_u2v{0u, 0u};
                if (e < have) v = *(const MLFFT_GLOBAL mlfft_u2v*)(s16 + (e >> 1));
                // elements copied to scalars first: a bit cast of a vector element reads element 0
                const unsigned int a0 = v[0], a1 = v[1];
                pre[2 * i] = make_float2(__uint_as_float(a0), __uint_as_float(a1));
            }
        } else if constexpr (pairs) {
#pragma unroll
            for (int i = 0; i < PF2; ++i) {
                const int e = 2 * (threadIdx.x + i * NTH);
                mlfft_f4v v = mlfft_f4v{0.f, 0.f, 0.f, 0.f};
                if (e < have) v = *(const MLFFT_GLOBAL mlfft_f4v*)(src + e);
                pre[2 * i] = make_float2(v[0], v[1]);
                pre[2 * i + 1] = make_float2(v[2], v[3]);
            }
        } else {
#pragma unroll
            for (int i = 0; i < PF; ++i) {
                const int e = threadIdx.x + i * NTH;
                pre[i] = e < have ? gload(src + e) : make_float2(0.f, 0.f);
            }
        }
    };
    auto stage = [&](unsigned short* buf) {
        if constexpr (XB != 0) {
#pragma unroll
            for (int i = 0; i < PF2; ++i) {
                const int e = 2 * (threadIdx.x + i * NTH);
                if (e < NT * bk) {
                    const int w = e / bk, n = e - w * bk;
                    const float f0 = pre[2 * i].x, f1 = pre[2 * i].y;
                    const uint32_t w0v = __float_as_uint(f0), w1v = __float_as_uint(f1);
                    // Re X of both values; -Im X by flipping the sign bits (bf16 rounding is
                    // symmetric, so this is the rounded -Im X)
                    const uint32_t re = (w0v & 0xffffu) | (w1v << 16);
                    const uint32_t im = ((w0v >> 16) | (w1v & 0xffff0000u)) ^ 0x80008000u;
                    *reinterpret_cast<uint32_t*>(&buf[w * LDX + n]) = re;
                    *reinterpret_cast<uint32_t*>(&buf[plane + w * LDX + n]) = im;
                }
            }
        } else if constexpr (pairs) {
#pragma unroll
            for (int i = 0; i < PF2; ++i) {
                const int e = 2 * (threadIdx.x + i * NTH);
                if (e < NT * bk) {
                    const int w = e / bk, n = e - w * bk;
                    const uint32_t re = (uint32_t)f32_to_bf16_bits(pre[2 * i].x) |
                                        ((uint32_t)f32_to_bf16_bits(pre[2 * i + 1].x) << 16);
                    const uint32_t im = (uint32_t)f32_to_bf16_bits(-pre[2 * i].y) |
                                        ((uint32_t)f32_to_bf16_bits(-pre[2 * i + 1].y) << 16);
                    *reinterpret_cast<uint32_t*>(&buf[w * LDX + n]) = re;
                    *reinterpret_cast<uint32_t*>(&buf[plane + w * LDX + n]) = im;
                }
            }
        } else {
#pragma unroll
            for (int i = 0; i < PF; ++i) {
                const int e = threadIdx.x + i * NTH;
                if (e < NT * bk) {
                    const int w = e / bk, n = e - w * bk;
                    buf[w * LDX + n] = f32_to_bf16_bits(pre[i].x);
                    buf[plane + w * LDX + n] = f32_to_bf16_bits(-pre[i].y);
                }
            }
        }
    };
    fetch(wbeg);
    __syncthreads();                      // padding zeroed; the previous segment's tiles read
    stage(xs);
    if (wbeg + NT < wend) fetch(wbeg + NT);
    __syncthreads();
    for (int w0 = wbeg, it = 0; w0 < wend; w0 += NT, ++it) {
        const unsigned short* xr = xs + (it & 1) * bufsz;
        const unsigned short* xn = xr + plane;            // -Im X
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            if (!act[h]) continue;
            floatx4 cr[NT / 16], ci[NT / 16];
#pragma unroll
            for (int cg = 0; cg < NT / 16; ++cg) {
                cr[cg] = floatx4{0, 0, 0, 0};
                ci[cg] = floatx4{0, 0, 0, 0};
            }
#pragma unroll
            for (int st = 0; st < S; ++st) {
                const bf16x8 ar = __builtin_bit_cast(bf16x8, gr[h][st]);
                const bf16x8 ai = __builtin_bit_cast(bf16x8, gi[h][st]);
                const bf16x8 an = __builtin_bit_cast(bf16x8, gr[h][st] ^ (unsigned short)0x8000u);   // -Re G
#pragma unroll
                for (int cg = 0; cg < NT / 16; ++cg) {
                    const int off = (cg * 16 + j) * LDX + 32 * st + 8 * q;
                    const bf16x8 br = __builtin_bit_cast(bf16x8, *reinterpret_cast<const ushortx8*>(&xr[off]));
                    const bf16x8 bn = __builtin_bit_cast(bf16x8, *reinterpret_cast<const ushortx8*>(&xn[off]));
                    // Re Y = Re G Re X + Im G (-Im X),  Im Y = Im G Re X + (-Re G)(-Im X)
                    cr[cg] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ar, br, cr[cg], 0, 0, 0);
                    cr[cg] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ai, bn, cr[cg], 0, 0, 0);
                    ci[cg] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ai, br, ci[cg], 0, 0, 0);
                    ci[cg] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(an, bn, ci[cg], 0, 0, 0);
                }
            }
#pragma unroll
            for (int cg = 0; cg < NT / 16; ++cg) {
                const int w = w0 + cg * 16 + j;
                if (w < wend) {
                    float2 o[4];
#pragma unroll
                    for (int r = 0; r < 4; ++r) o[r] = make_float2(cr[cg][r], ci[cg][r]);
                    const int m0 = mb[h] + 4 * q;
                    float2* dst = Yk + (size_t)w * bk + m0;
                    if (even_b && m0 + 4 <= bk) {
                        gstore2(dst, o[0], o[1]);
                        gstore2(dst + 2, o[2], o[3]);
                    } else {
#pragma unroll
                        for (int r = 0; r < 4; ++r)
                            if (m0 + r < bk) gstore(dst + r, o[r]);
                    }
                }
            }
        }
        if (w0 + NT < wend) {
            stage(xs + ((it + 1) & 1) * bufsz);
            if (w0 + 2 * NT < wend) fetch(w0 + 2 * NT);
        }
        __syncthreads();
    }
    }
}

}  // namespace mlfft
