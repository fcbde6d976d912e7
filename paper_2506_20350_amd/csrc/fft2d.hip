// Two-level blockwise FFT kernels of the MLFFT product and of the block-circulant
// preconditioner (Sec. III-A, eq. multL with L = 2; eq. xc2 for the padding and
// the extraction of v from v^[2]).
//
// A column w holds Ny x Nx cells of b basis functions, in[w][iy][ix][m].  The
// blockwise 2-level DFT is the 2-D DFT over (iy, ix) of each of the b*W series
// (F^[2] = F_Ny (x) F_Nx (x) I_b, eq. F2).  One workgroup transforms one column
// for a chunk of cm consecutive basis functions, so every global access reads
// or writes cm contiguous complex values:
//   forward : phase 1 (threads over ix, m) loads the Ny values of its series,
//             transforms along y in registers and writes a [Py][Nx][cm] LDS
//             tile; phase 2 (threads over ky, m) transforms along x and writes
//             the spectrum out[k][w][m], k = ky*Px + kx.
//   inverse : the same two phases in the opposite order, keeping only the
//             Ny x Nx cells of the result.
// With pad = 1 the grid is 2Ny x 2Nx.  Only the first N inputs of a length-2N
// transform are non-zero, so its even outputs are the length-N DFT of x and its
// odd outputs the length-N DFT of x[n] exp(-i pi n/N); the cropped inverse is
// the mirror image.  Every transform therefore runs as length-N codelets.
#include "internal.h"
#include "fft_codelets.h"

#include <algorithm>
#include <map>
#include <tuple>

namespace mlfft {

// Transform lengths are grouped in classes, one kernel instantiation per class,
// so that the register allocation of a kernel is set by the largest codelet of
// its own class only: class 0 = 1..16, class 1 = the composite lengths 17..32,
// class 2 = the primes 17..31 (direct DFTs with the most live values).
#define MLFFT_CASES0(X) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16)
#define MLFFT_CASES1(X) X(18) X(20) X(21) X(22) X(24) X(25) X(26) X(27) X(28) X(30) X(32)
#define MLFFT_CASES2(X) X(17) X(19) X(23) X(29) X(31)

__host__ __device__ constexpr int len_class(int n) {
    return n <= 16 ? 0 : (n == 17 || n == 19 || n == 23 || n == 29 || n == 31) ? 2 : 1;
}

template<template<typename, int> class F, typename C, int CLS, typename... A>
__device__ __forceinline__ void dispatch_n(int n, A... a) {
    switch (n) {
#define MLFFT_CASE(N) case N: F<C, N>::run(a...); break;
        MLFFT_CASES0(MLFFT_CASE)
#undef MLFFT_CASE
        default: break;
    }
    if (CLS >= 1) {
        switch (n) {
#define MLFFT_CASE(N) case N: F<C, N>::run(a...); break;
            MLFFT_CASES1(MLFFT_CASE)
#undef MLFFT_CASE
            default: break;
        }
    }
    if (CLS >= 2) {
        switch (n) {
#define MLFFT_CASE(N) case N: F<C, N>::run(a...); break;
            MLFFT_CASES2(MLFFT_CASE)
#undef MLFFT_CASE
            default: break;
        }
    }
}

struct Work {
    int w, m0, mlen;
};

// XCD-aware order of the work items.  Workgroups are dealt to the 8 XCDs round
// robin, so consecutive workgroup indices land on different XCDs (and L2s).
// Consecutive work items are the neighbouring basis-function chunks of one
// column, whose global segments share 128-byte lines when a chunk is 64 bytes;
// giving each XCD a contiguous range of work items lets the two halves of a line
// meet in the same L2 instead of being fetched twice.
__device__ __forceinline__ int work_index() {
    const int bid = blockIdx.x, G = gridDim.x;
    const int per = G >> 3;
    if (bid >= per * 8) return bid;
    return (bid & 7) * per + (bid >> 3);
}

__device__ __forceinline__ const FftTask* find_task(const FftTask* tasks, int ntasks, int bid) {
    int lo = 0, hi = ntasks - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (tasks[mid].block_begin <= bid) lo = mid; else hi = mid - 1;
    }
    return tasks + lo;
}

// ---------------------------------------------------------------- forward

template<typename C, int NY>
struct FwdY {
    // The column is read from HBM once: with pad = 1 it is parked in the odd rows
    // of this thread's own tile column while the even half is transformed, then
    // read back, twiddled and transformed into those odd rows.
    static __device__ __forceinline__ void run(const FftTask& tt, Work wk, C* tile) {
        const FftTask* t = &tt;
        const int Nx = t->Nx, cm = t->cm, b = t->b;
        const int tid = threadIdx.x;
        if (tid >= Nx * cm) return;
        const int ix = tid / cm, mi = tid - ix * cm;
        if (mi >= wk.mlen) return;
        const C* __restrict__ src = static_cast<const C*>(t->in)
            + (size_t)wk.w * ((size_t)NY * Nx * b + t->colpad) + (size_t)ix * b + wk.m0 + mi;
        const size_t ys = (size_t)Nx * b;
        C* col = tile + ix * cm + mi;
        const int rs = t->rs;
        C v[NY];
#pragma unroll
        for (int iy = 0; iy < NY; ++iy) v[iy] = src[iy * ys];
        if (t->pad) {
#pragma unroll
            for (int j = 0; j < NY; ++j) col[(2 * j + 1) * rs] = v[j];
            Fft<C, NY, -1>::run(v);
#pragma unroll
            for (int j = 0; j < NY; ++j) col[2 * j * rs] = v[j];
#pragma unroll
            for (int j = 0; j < NY; ++j) v[j] = col[(2 * j + 1) * rs];
            Fft<C, NY, -1>::tw2(v);
            Fft<C, NY, -1>::run(v);
#pragma unroll
            for (int j = 0; j < NY; ++j) col[(2 * j + 1) * rs] = v[j];
        } else {
            Fft<C, NY, -1>::run(v);
#pragma unroll
            for (int j = 0; j < NY; ++j) col[j * rs] = v[j];
        }
    }
};

template<typename C, int NX>
struct FwdX {
    static __device__ __forceinline__ void run(const FftTask& tt, Work wk, const C* tile) {
        const FftTask* t = &tt;
        const int cm = t->cm, b = t->b, W = t->W;
        const int H = t->pad ? 2 : 1;
        const int Py = H * t->Ny, Px = H * NX;
        const int tid = threadIdx.x;
        if (tid >= Py * cm) return;
        const int ky = tid / cm, mi = tid - ky * cm;
        if (mi >= wk.mlen) return;
        const size_t base = (size_t)wk.w * b + wk.m0 + mi;
        C* __restrict__ dst = static_cast<C*>(t->out) + base;
        const size_t ks = (size_t)W * b;
        for (int g = 0; g < H; ++g) {
            C v[NX];
#pragma unroll
            for (int ix = 0; ix < NX; ++ix) v[ix] = tile[ky * t->rs + ix * cm + mi];
            if (g) Fft<C, NX, -1>::tw2(v);
            Fft<C, NX, -1>::run(v);
            if constexpr (std::is_same<C, float2>::value) {
                if (t->out16) {
                    // bf16 spectrum for the bf16 block product: (re, im) rounded to nearest even
                    uint32_t* __restrict__ d16 = static_cast<uint32_t*>(t->out) + base;
#pragma unroll
                    for (int i = 0; i < NX; ++i) {
                        const int kx = t->pad ? 2 * i + g : i;
                        d16[(size_t)(ky * Px + kx) * ks] =
                            (uint32_t)f32_to_bf16_bits(v[i].x) | ((uint32_t)f32_to_bf16_bits(v[i].y) << 16);
                    }
                    continue;
                }
            }
#pragma unroll
            for (int i = 0; i < NX; ++i) {
                const int kx = t->pad ? 2 * i + g : i;
                dst[(size_t)(ky * Px + kx) * ks] = v[i];
            }
        }
    }
};

template<typename C, int CLS, int PAD>
__global__ void __launch_bounds__(512) fft_fwd_kernel(FftTask t0, const FftTask* tasks, int ntasks) {
    extern __shared__ unsigned char smem_raw[];
    C* tile = reinterpret_cast<C*>(smem_raw);
    const int bid = work_index();
    FftTask tl = ntasks > 0 ? *find_task(tasks, ntasks, bid) : t0;
    tl.pad = PAD;
    const FftTask* t = &tl;
    const int local = bid - t->block_begin;
    Work wk;
    wk.w = local / t->nmc;
    const int mc = local - wk.w * t->nmc;
    wk.m0 = mc * t->cm;
    wk.mlen = min(t->cm, t->b - wk.m0);
    dispatch_n<FwdY, C, CLS>(t->Ny, tl, wk, tile);
    __syncthreads();
    dispatch_n<FwdX, C, CLS>(t->Nx, tl, wk, (const C*)tile);
}

// ---------------------------------------------------------------- forward, half-height tile

// The padded forward in two halves: the even-ky rows (the length-Ny DFT of each
// column) are written to a tile of Ny rows and transformed along x; then the
// odd-ky rows (the DFT of the twiddled column) go through the same tile.  Each
// thread keeps its input column in registers between the halves, so the column
// is read from HBM once.  The tile is half as tall as the one-pass kernel's,
// which admits twice the m-chunk (longer contiguous runs in the spectrum) or two
// workgroups per CU.
template<typename C, int NY>
struct FwdYHalf {
    static __device__ __forceinline__ void run(const FftTask& tt, Work wk, C* tile, C* xin, int par) {
        const FftTask* t = &tt;
        const int Nx = t->Nx, cm = t->cm, b = t->b;
        const int tid = threadIdx.x;
        if (tid >= Nx * cm) return;
        const int ix = tid / cm, mi = tid - ix * cm;
        if (mi >= wk.mlen) return;
        C v[NY];
        if (par == 0) {
            const C* __restrict__ src = static_cast<const C*>(t->in)
                + (size_t)wk.w * ((size_t)NY * Nx * b + t->colpad) + (size_t)ix * b + wk.m0 + mi;
            const size_t ys = (size_t)Nx * b;
#pragma unroll
            for (int iy = 0; iy < NY; ++iy) v[iy] = src[iy * ys];
#pragma unroll
            for (int iy = 0; iy < NY; ++iy) xin[iy] = v[iy];
        } else {
#pragma unroll
            for (int iy = 0; iy < NY; ++iy) v[iy] = xin[iy];
            Fft<C, NY, -1>::tw2(v);
        }
        Fft<C, NY, -1>::run(v);
        C* col = tile + ix * cm + mi;
#pragma unroll
        for (int j = 0; j < NY; ++j) col[j * t->rs] = v[j];
    }
};

template<typename C, int NX>
struct FwdXHalf {
    static __device__ __forceinline__ void run(const FftTask& tt, Work wk, const C* tile, int par) {
        const FftTask* t = &tt;
        const int cm = t->cm, b = t->b, W = t->W;
        const int Px = 2 * NX;
        const int tid = threadIdx.x;
        if (tid >= t->Ny * cm) return;
        const int a = tid / cm, mi = tid - a * cm;
        if (mi >= wk.mlen) return;
        const int ky = 2 * a + par;
        C* __restrict__ dst = static_cast<C*>(t->out) + (size_t)wk.w * b + wk.m0 + mi;
        const size_t ks = (size_t)W * b;
        for (int g = 0; g < 2; ++g) {
            C v[NX];
#pragma unroll
            for (int ix = 0; ix < NX; ++ix) v[ix] = tile[a * t->rs + ix * cm + mi];
            if (g) Fft<C, NX, -1>::tw2(v);
            Fft<C, NX, -1>::run(v);
#pragma unroll
            for (int i = 0; i < NX; ++i) dst[(size_t)(ky * Px + 2 * i + g) * ks] = v[i];
        }
    }
};

template<typename C, int CLS, int LB>
__global__ void __launch_bounds__(LB) fft_fwd_half_kernel(FftTask t0, const FftTask* tasks, int ntasks) {
    extern __shared__ unsigned char smem_raw[];
    C* tile = reinterpret_cast<C*>(smem_raw);
    const int bid = work_index();
    FftTask tl = ntasks > 0 ? *find_task(tasks, ntasks, bid) : t0;
    tl.pad = 1;
    const FftTask* t = &tl;
    const int local = bid - t->block_begin;
    Work wk;
    wk.w = local / t->nmc;
    const int mc = local - wk.w * t->nmc;
    wk.m0 = mc * t->cm;
    wk.mlen = min(t->cm, t->b - wk.m0);
    C xin[32];
    dispatch_n<FwdYHalf, C, CLS>(t->Ny, tl, wk, tile, xin, 0);
    __syncthreads();
    dispatch_n<FwdXHalf, C, CLS>(t->Nx, tl, wk, (const C*)tile, 0);
    __syncthreads();
    dispatch_n<FwdYHalf, C, CLS>(t->Ny, tl, wk, tile, xin, 1);
    __syncthreads();
    dispatch_n<FwdXHalf, C, CLS>(t->Nx, tl, wk, (const C*)tile, 1);
}

// ---------------------------------------------------------------- inverse

template<typename C, int NX>
struct InvX {
    // The even-kx half is written to the LDS tile and the odd half added to it,
    // so only one length-NX vector is live in registers.
    static __device__ __forceinline__ void run(const FftTask& tt, Work wk, C* tile) {
        const FftTask* t = &tt;
        const int cm = t->cm, b = t->b, W = t->W;
        const int H = t->pad ? 2 : 1;
        const int Py = H * t->Ny, Px = H * NX;
        const int tid = threadIdx.x;
        if (tid >= Py * cm) return;
        const int ky = tid / cm, mi = tid - ky * cm;
        if (mi >= wk.mlen) return;
        const C* __restrict__ src = static_cast<const C*>(t->in) + (size_t)wk.w * b + wk.m0 + mi;
        const size_t ks = (size_t)W * b;
        C* row = tile + ky * t->rs + mi;
        for (int g = 0; g < H; ++g) {
            C v[NX];
#pragma unroll
            for (int i = 0; i < NX; ++i) {
                const int kx = t->pad ? 2 * i + g : i;
                v[i] = src[(size_t)(ky * Px + kx) * ks];
            }
            Fft<C, NX, 1>::run(v);
            if (g) {
                Fft<C, NX, 1>::tw2(v);
#pragma unroll
                for (int ix = 0; ix < NX; ++ix) row[ix * cm] = cadd(row[ix * cm], v[ix]);
            } else {
#pragma unroll
                for (int ix = 0; ix < NX; ++ix) row[ix * cm] = v[ix];
            }
        }
    }
};

template<typename C, int NY>
struct InvY {
    // Each thread owns the tile column (ix, mi): the even-ky half's transform is
    // parked in the even rows of that column while the odd half is transformed.
    static __device__ __forceinline__ void run(const FftTask& tt, Work wk, C* tile) {
        const FftTask* t = &tt;
        typedef typename CTraits<C>::real R;
        const int Nx = t->Nx, cm = t->cm, b = t->b;
        const int H = t->pad ? 2 : 1;
        const int tid = threadIdx.x;
        if (tid >= Nx * cm) return;
        const int ix = tid / cm, mi = tid - ix * cm;
        if (mi >= wk.mlen) return;
        C* col = tile + ix * cm + mi;
        const int rs = t->rs;
        C v[NY];
#pragma unroll
        for (int j = 0; j < NY; ++j) v[j] = col[(t->pad ? 2 * j : j) * rs];
        Fft<C, NY, 1>::run(v);
        if (H == 2) {
#pragma unroll
            for (int j = 0; j < NY; ++j) col[2 * j * rs] = v[j];
#pragma unroll
            for (int j = 0; j < NY; ++j) v[j] = col[(2 * j + 1) * rs];
            Fft<C, NY, 1>::run(v);
            Fft<C, NY, 1>::tw2(v);
#pragma unroll
            for (int iy = 0; iy < NY; ++iy) v[iy] = cadd(v[iy], col[2 * iy * rs]);
        }
        const size_t off = (size_t)wk.w * ((size_t)NY * Nx * b + t->colpad) + (size_t)ix * b + wk.m0 + mi;
        const size_t ys = (size_t)Nx * b;
        C* __restrict__ dst = static_cast<C*>(t->out) + off;
        const R alpha = (R)t->alpha;
        if (t->addend) {
            const C* __restrict__ add = static_cast<const C*>(t->addend) + off;
            const R beta = (R)t->beta;
#pragma unroll
            for (int iy = 0; iy < NY; ++iy) {
                const C a = add[iy * ys];
                dst[iy * ys] = cmake<C>(v[iy].x * alpha + a.x * beta, v[iy].y * alpha + a.y * beta);
            }
        } else {
#pragma unroll
            for (int iy = 0; iy < NY; ++iy) dst[iy * ys] = cscale(v[iy], alpha);
        }
    }
};

template<typename C, int CLS, int PAD>
__global__ void __launch_bounds__(512) fft_inv_kernel(FftTask t0, const FftTask* tasks, int ntasks) {
    extern __shared__ unsigned char smem_raw[];
    C* tile = reinterpret_cast<C*>(smem_raw);
    const int bid = work_index();
    FftTask tl = ntasks > 0 ? *find_task(tasks, ntasks, bid) : t0;
    tl.pad = PAD;
    const FftTask* t = &tl;
    const int local = bid - t->block_begin;
    Work wk;
    wk.w = local / t->nmc;
    const int mc = local - wk.w * t->nmc;
    wk.m0 = mc * t->cm;
    wk.mlen = min(t->cm, t->b - wk.m0);
    dispatch_n<InvX, C, CLS>(t->Nx, tl, wk, tile);
    __syncthreads();
    dispatch_n<InvY, C, CLS>(t->Ny, tl, wk, tile);
}

// ---------------------------------------------------------------- inverse, half-height tile

// The padded inverse in two halves: the even-ky rows are transformed along x
// into a tile of Ny rows and then along y into registers; the odd-ky rows
// follow through the same tile and are added.  The tile is half as tall as the
// one-pass kernel's, so two workgroups share a CU and one's loads overlap the
// other's arithmetic (or one workgroup takes twice the m-chunk).
template<typename C, int NX>
struct InvXHalf {
    static __device__ __forceinline__ void run(const FftTask& tt, Work wk, C* tile, int par) {
        const FftTask* t = &tt;
        const int cm = t->cm, b = t->b, W = t->W;
        const int Px = 2 * NX;
        const int tid = threadIdx.x;
        if (tid >= t->Ny * cm) return;
        const int a = tid / cm, mi = tid - a * cm;
        if (mi >= wk.mlen) return;
        const int ky = 2 * a + par;
        const C* __restrict__ src = static_cast<const C*>(t->in) + (size_t)wk.w * b + wk.m0 + mi;
        const size_t ks = (size_t)W * b;
        C* row = tile + a * t->rs + mi;
        if (sizeof(C) == 16) {
            // FP64: one half-length vector live at a time, the odd-kx half added in LDS
            C v[NX];
#pragma unroll
            for (int i = 0; i < NX; ++i) v[i] = src[(size_t)(ky * Px + 2 * i) * ks];
            Fft<C, NX, 1>::run(v);
#pragma unroll
            for (int ix = 0; ix < NX; ++ix) row[ix * cm] = v[ix];
#pragma unroll
            for (int i = 0; i < NX; ++i) v[i] = src[(size_t)(ky * Px + 2 * i + 1) * ks];
            Fft<C, NX, 1>::run(v);
            Fft<C, NX, 1>::tw2(v);
#pragma unroll
            for (int ix = 0; ix < NX; ++ix) row[ix * cm] = cadd(row[ix * cm], v[ix]);
            return;
        }
        C v[NX], o[NX];
#pragma unroll
        for (int i = 0; i < NX; ++i) {
            v[i] = src[(size_t)(ky * Px + 2 * i) * ks];
            o[i] = src[(size_t)(ky * Px + 2 * i + 1) * ks];
        }
        Fft<C, NX, 1>::run(v);
        Fft<C, NX, 1>::run(o);
        Fft<C, NX, 1>::tw2(o);
#pragma unroll
        for (int ix = 0; ix < NX; ++ix) row[ix * cm] = cadd(v[ix], o[ix]);
    }
};

template<typename C, int NY>
struct InvYHalf {
    // par 0: e = the y-transform of the even rows; par 1: out = e + the twiddled
    // y-transform of the odd rows, cropped, scaled and with the addend
    static __device__ __forceinline__ void run(const FftTask& tt, Work wk, const C* tile, C* e, int par) {
        const FftTask* t = &tt;
        typedef typename CTraits<C>::real R;
        const int Nx = t->Nx, cm = t->cm, b = t->b;
        const int tid = threadIdx.x;
        if (tid >= Nx * cm) return;
        const int ix = tid / cm, mi = tid - ix * cm;
        if (mi >= wk.mlen) return;
        const C* col = tile + ix * cm + mi;
        const int rs = t->rs;
        const size_t off = (size_t)wk.w * ((size_t)NY * Nx * b + t->colpad) + (size_t)ix * b + wk.m0 + mi;
        const size_t ys = (size_t)Nx * b;
        // the addend is requested before the odd half's transform, which hides its latency
        C av[NY];
        if (par == 1 && t->addend) {
            const C* __restrict__ add = static_cast<const C*>(t->addend) + off;
#pragma unroll
            for (int iy = 0; iy < NY; ++iy) av[iy] = add[iy * ys];
        }
        C v[NY];
#pragma unroll
        for (int j = 0; j < NY; ++j) v[j] = col[j * rs];
        Fft<C, NY, 1>::run(v);
        if (par == 0) {
#pragma unroll
            for (int j = 0; j < NY; ++j) e[j] = v[j];
            return;
        }
        Fft<C, NY, 1>::tw2(v);
#pragma unroll
        for (int iy = 0; iy < NY; ++iy) v[iy] = cadd(v[iy], e[iy]);
        C* __restrict__ dst = static_cast<C*>(t->out) + off;
        const R alpha = (R)t->alpha;
        if (t->addend) {
            const R beta = (R)t->beta;
#pragma unroll
            for (int iy = 0; iy < NY; ++iy)
                dst[iy * ys] = cmake<C>(v[iy].x * alpha + av[iy].x * beta, v[iy].y * alpha + av[iy].y * beta);
        } else {
#pragma unroll
            for (int iy = 0; iy < NY; ++iy) dst[iy * ys] = cscale(v[iy], alpha);
        }
    }
};

template<typename C, int CLS, int LB>
__global__ void __launch_bounds__(LB) fft_inv_half_kernel(FftTask t0, const FftTask* tasks, int ntasks) {
    extern __shared__ unsigned char smem_raw[];
    C* tile = reinterpret_cast<C*>(smem_raw);
    const int bid = work_index();
    FftTask tl = ntasks > 0 ? *find_task(tasks, ntasks, bid) : t0;
    tl.pad = 1;
    const FftTask* t = &tl;
    const int local = bid - t->block_begin;
    Work wk;
    wk.w = local / t->nmc;
    const int mc = local - wk.w * t->nmc;
    wk.m0 = mc * t->cm;
    wk.mlen = min(t->cm, t->b - wk.m0);
    C e[32];
    dispatch_n<InvXHalf, C, CLS>(t->Nx, tl, wk, tile, 0);
    __syncthreads();
    dispatch_n<InvYHalf, C, CLS>(t->Ny, tl, wk, (const C*)tile, e, 0);
    __syncthreads();
    dispatch_n<InvXHalf, C, CLS>(t->Nx, tl, wk, tile, 1);
    __syncthreads();
    dispatch_n<InvYHalf, C, CLS>(t->Ny, tl, wk, (const C*)tile, e, 1);
}

// ---------------------------------------------------------------- host side

static const size_t kLdsBudget = 160 * 1024;

// tuned m-chunk and tile choice per (prec, pad, dir, Nx, Ny, b); cm 0: the default
// rule, half -1: the default choice
struct FftChoice {
    int cm = 0;
    int half = -1;
};
static std::map<std::tuple<int, int, int, int, int, int>, FftChoice> g_fft_override;

void fft_set_choice(int prec, int pad, int dir, int Nx, int Ny, int b, int cm, int half) {
    const auto key = std::make_tuple(prec, pad, dir, Nx, Ny, b);
    if (cm <= 0 && half < 0) { g_fft_override.erase(key); return; }
    g_fft_override[key] = FftChoice{cm > 0 ? cm : 0, half};
}

static FftChoice choice_of(int prec, int pad, int dir, int Nx, int Ny, int b) {
    auto it = g_fft_override.find(std::make_tuple(prec, pad, dir, Nx, Ny, b));
    return it == g_fft_override.end() ? FftChoice{} : it->second;
}

// Half-height tile: by default every padded transform whose lengths are not the
// primes 17..31; those take it when tuned to (their direct DFTs and the parked
// half-length vector need the 256-thread bound below).
bool fft_use_half(int prec, int pad, int dir, int Nx, int Ny, int b) {
    if (!pad) return false;
    const FftChoice c = choice_of(prec, pad, dir, Nx, Ny, b);
    if (c.half >= 0) return c.half != 0;
    return std::max(len_class(Nx), len_class(Ny)) <= 1;
}

// threads a workgroup may have: the FP64 half-height kernels, and the FP32 ones of
// the prime lengths, are bounded at 256 so that a wave may hold the parked
// half-length vector (and a direct DFT) in up to 512 registers without spilling
static int thread_limit(int prec, bool half, int cls) { return half && (prec == P64 || cls == 2) ? 256 : 512; }

// LDS rows of a tile
static int tile_rows(int pad, bool half, int Ny) { return pad && !half ? 2 * Ny : Ny; }

// Row stride of a tile in elements.  A wave reads 64 / cm rows of cm consecutive
// elements each (the x-transforms); with the stride a multiple of the segment
// width plus one segment modulo the 256-byte LDS bank period, the rows fall on
// successive banks instead of all on the same ones.
static int tile_stride(int eb, int Nx, int cm) {
    int rs = Nx * cm;
    if (cm * eb >= 256) return rs;
    while (((rs - cm) * eb) % 256 != 0) ++rs;
    return rs;
}

static int elem_bytes(int prec) { return prec == P64 ? 16 : 8; }

static bool cm_fits(int prec, int pad, bool half, int Nx, int Ny, int cm) {
    const int eb = elem_bytes(prec);
    const int Py = tile_rows(pad, half, Ny);
    const int cls = std::max(len_class(Nx), len_class(Ny));
    return (size_t)Py * tile_stride(eb, Nx, cm) * eb <= kLdsBudget &&
           (Py > Nx ? Py : Nx) * cm <= thread_limit(prec, half, cls);
}

// largest power-of-two m-chunk (up to 64 and b) the launch limits allow for a tile choice
int fft_max_cm(int prec, int pad, int half, int Nx, int Ny, int b) {
    int cm = 64;
    if (cm > b) cm = b;
    while (cm > 1 && !cm_fits(prec, pad, half != 0, Nx, Ny, cm)) cm >>= 1;
    return cm;
}

void fft_get_choice(int prec, int pad, int dir, int Nx, int Ny, int b, int* cm, int* half) {
    *cm = choice_of(prec, pad, dir, Nx, Ny, b).cm;
    *half = fft_use_half(prec, pad, dir, Nx, Ny, b) ? 1 : 0;
}

void plan_fft_tasks(int prec, FftTask* tasks, int ntasks, int dir, int* grid, int* block, size_t* lds) {
    const int eb = elem_bytes(prec);
    int g = 0, blk = 64;
    size_t l = 0;
    for (int i = 0; i < ntasks; ++i) {
        FftTask& t = tasks[i];
        const bool half = fft_use_half(prec, t.pad, dir, t.Nx, t.Ny, t.b);
        const int Py = tile_rows(t.pad, half, t.Ny);
        // default: 128-byte contiguous runs per series group (whole 128-byte lines of
        // the spectrum), 64-byte runs when that would leave fewer than 2048
        // workgroups; shrink when LDS or the thread limit would overflow
        int cm = choice_of(prec, t.pad, dir, t.Nx, t.Ny, t.b).cm;
        if (cm <= 0) cm = (size_t)t.W * ((t.b + 128 / eb - 1) / (128 / eb)) >= 2048 ? 128 / eb : 64 / eb;
        if (cm > t.b) cm = t.b;
        while (cm > 1 && !cm_fits(prec, t.pad, half, t.Nx, t.Ny, cm)) cm >>= 1;
        t.cm = cm;
        t.nmc = (t.b + cm - 1) / cm;
        t.block_begin = g;
        g += t.nmc * t.W;
        int thr = (Py > t.Nx ? Py : t.Nx) * cm;
        thr = (thr + 63) / 64 * 64;
        if (thr > blk) blk = thr;
        t.rs = tile_stride(eb, t.Nx, cm);
        const size_t ll = (size_t)Py * t.rs * eb;
        if (ll > l) l = ll;
    }
    *grid = g;
    *block = blk;
    *lds = l;
}

int fft_group_key(int prec, const FftTask& t, int dir) {
    FftTask one = t;
    int grid, block;
    size_t lds;
    plan_fft_tasks(prec, &one, 1, dir, &grid, &block, &lds);
    int bucket = 0;
    while (((size_t)1 << bucket) < lds) ++bucket;
    const int half = fft_use_half(prec, t.pad, dir, t.Nx, t.Ny, t.b) ? 1 : 0;
    return (half * 4 + std::max(len_class(t.Nx), len_class(t.Ny))) * 64 + bucket;
}

typedef void (*FftKernel)(FftTask, const FftTask*, int);

static FftKernel with_lds(FftKernel k) {
    (void)hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsBudget);
    return k;
}

template<typename C, int INV>
static FftKernel pick_kernel(int cls, int pad) {
#define PICK(CL, PD) if (cls == CL && pad == PD) \
        return with_lds(INV ? (FftKernel)fft_inv_kernel<C, CL, PD> : (FftKernel)fft_fwd_kernel<C, CL, PD>);
    PICK(0, 0) PICK(0, 1) PICK(1, 0) PICK(1, 1) PICK(2, 0) PICK(2, 1)
#undef PICK
    return nullptr;
}

template<typename C, int INV>
static FftKernel pick_half(int cls) {
    constexpr int LB = sizeof(C) == 16 ? 256 : 512;
    if (INV) {
        if (cls == 2) return with_lds((FftKernel)fft_inv_half_kernel<C, 2, 256>);
        return with_lds(cls == 0 ? (FftKernel)fft_inv_half_kernel<C, 0, LB> : (FftKernel)fft_inv_half_kernel<C, 1, LB>);
    }
    if (cls == 2) return with_lds((FftKernel)fft_fwd_half_kernel<C, 2, 256>);
    return with_lds(cls == 0 ? (FftKernel)fft_fwd_half_kernel<C, 0, LB> : (FftKernel)fft_fwd_half_kernel<C, 1, LB>);
}

template<typename C, int INV>
static hipError_t launch_t(const FftTask* th, const FftTask* td, int ntasks, hipStream_t s) {
    // the host copy is already planned (cm, nmc, block_begin filled)
    int grid = 0, block = 64, cls = 0;
    size_t lds = 0;
    const int eb = sizeof(C);
    const int prec = sizeof(C) == 16 ? P64 : P32;
    if (ntasks <= 0) return hipSuccess;
    const bool half = fft_use_half(prec, th[0].pad, INV, th[0].Nx, th[0].Ny, th[0].b);
    for (int i = 0; i < ntasks; ++i) {
        const FftTask& t = th[i];
        if (t.pad != th[0].pad || fft_use_half(prec, t.pad, INV, t.Nx, t.Ny, t.b) != half) return hipErrorInvalidValue;
        const int Py = tile_rows(t.pad, half, t.Ny);
        grid = t.block_begin + t.nmc * t.W > grid ? t.block_begin + t.nmc * t.W : grid;
        int thr = ((Py > t.Nx ? Py : t.Nx) * t.cm + 63) / 64 * 64;
        if (thr > block) block = thr;
        size_t ll = (size_t)Py * t.rs * eb;
        if (ll > lds) lds = ll;
        cls = std::max(cls, std::max(len_class(t.Nx), len_class(t.Ny)));
    }
    if (grid == 0) return hipSuccess;
    if (block > thread_limit(prec, half, cls) || lds > kLdsBudget) return hipErrorInvalidValue;
    FftKernel k = half ? pick_half<C, INV>(cls) : pick_kernel<C, INV>(cls, th[0].pad);
    if (!k) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k, dim3(grid), dim3(block), lds, s, th[0], ntasks > 1 ? td : nullptr, ntasks > 1 ? ntasks : 0);
    return hipGetLastError();
}

hipError_t launch_fft_fwd(int prec, const FftTask* th, const FftTask* td, int ntasks, hipStream_t s) {
    if (prec == P64) return launch_t<double2, 0>(th, td, ntasks, s);
    return launch_t<float2, 0>(th, td, ntasks, s);
}

hipError_t launch_fft_inv(int prec, const FftTask* th, const FftTask* td, int ntasks, hipStream_t s) {
    if (prec == P64) return launch_t<double2, 1>(th, td, ntasks, s);
    return launch_t<float2, 1>(th, td, ntasks, s);
}

}  // namespace mlfft
