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

namespace mlfft {

#define MLFFT_CASES(X) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) \
    X(14) X(15) X(16) X(17) X(18) X(19) X(20) X(21) X(22) X(23) X(24) X(25) X(26) X(27) X(28) \
    X(29) X(30) X(31) X(32)

template<template<typename, int> class F, typename C, typename... A>
__device__ __forceinline__ void dispatch_n(int n, A... a) {
    switch (n) {
#define MLFFT_CASE(N) case N: F<C, N>::run(a...); break;
        MLFFT_CASES(MLFFT_CASE)
#undef MLFFT_CASE
        default: break;
    }
}

struct Work {
    int w, m0, mlen;
};

__device__ __forceinline__ const FftTask* find_task(const FftTask* tasks, int ntasks) {
    int lo = 0, hi = ntasks - 1;
    const int bid = blockIdx.x;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (tasks[mid].block_begin <= bid) lo = mid; else hi = mid - 1;
    }
    return tasks + lo;
}

// ---------------------------------------------------------------- forward

template<typename C, int NY>
struct FwdY {
    static __device__ __forceinline__ void run(const FftTask& tt, Work wk, C* tile) {
        const FftTask* t = &tt;
        const int Nx = t->Nx, cm = t->cm, b = t->b;
        const int tid = threadIdx.x;
        if (tid >= Nx * cm) return;
        const int ix = tid / cm, mi = tid - ix * cm;
        if (mi >= wk.mlen) return;
        const C* __restrict__ src = static_cast<const C*>(t->in)
            + ((size_t)wk.w * NY * Nx + ix) * b + wk.m0 + mi;
        const size_t ys = (size_t)Nx * b;
        const int H = t->pad ? 2 : 1;
        for (int h = 0; h < H; ++h) {
            C v[NY];
#pragma unroll
            for (int iy = 0; iy < NY; ++iy) v[iy] = src[iy * ys];
            if (h) Fft<C, NY, -1>::tw2(v);
            Fft<C, NY, -1>::run(v);
#pragma unroll
            for (int j = 0; j < NY; ++j) {
                const int ky = t->pad ? 2 * j + h : j;
                tile[(ky * Nx + ix) * cm + mi] = v[j];
            }
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
        C* __restrict__ dst = static_cast<C*>(t->out) + (size_t)wk.w * b + wk.m0 + mi;
        const size_t ks = (size_t)W * b;
        for (int g = 0; g < H; ++g) {
            C v[NX];
#pragma unroll
            for (int ix = 0; ix < NX; ++ix) v[ix] = tile[(ky * NX + ix) * cm + mi];
            if (g) Fft<C, NX, -1>::tw2(v);
            Fft<C, NX, -1>::run(v);
#pragma unroll
            for (int i = 0; i < NX; ++i) {
                const int kx = t->pad ? 2 * i + g : i;
                dst[(size_t)(ky * Px + kx) * ks] = v[i];
            }
        }
    }
};

template<typename C>
__global__ void __launch_bounds__(512) fft_fwd_kernel(FftTask t0, const FftTask* tasks, int ntasks) {
    extern __shared__ unsigned char smem_raw[];
    C* tile = reinterpret_cast<C*>(smem_raw);
    const FftTask tl = ntasks > 0 ? *find_task(tasks, ntasks) : t0;
    const FftTask* t = &tl;
    const int local = blockIdx.x - t->block_begin;
    Work wk;
    wk.w = local / t->nmc;
    const int mc = local - wk.w * t->nmc;
    wk.m0 = mc * t->cm;
    wk.mlen = min(t->cm, t->b - wk.m0);
    dispatch_n<FwdY, C>(t->Ny, tl, wk, tile);
    __syncthreads();
    dispatch_n<FwdX, C>(t->Nx, tl, wk, (const C*)tile);
}

// ---------------------------------------------------------------- inverse

template<typename C, int NX>
struct InvX {
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
        C acc[NX];
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
                for (int ix = 0; ix < NX; ++ix) acc[ix] = cadd(acc[ix], v[ix]);
            } else {
#pragma unroll
                for (int ix = 0; ix < NX; ++ix) acc[ix] = v[ix];
            }
        }
#pragma unroll
        for (int ix = 0; ix < NX; ++ix) tile[(ky * NX + ix) * cm + mi] = acc[ix];
    }
};

template<typename C, int NY>
struct InvY {
    static __device__ __forceinline__ void run(const FftTask& tt, Work wk, const C* tile) {
        const FftTask* t = &tt;
        typedef typename CTraits<C>::real R;
        const int Nx = t->Nx, cm = t->cm, b = t->b;
        const int H = t->pad ? 2 : 1;
        const int tid = threadIdx.x;
        if (tid >= Nx * cm) return;
        const int ix = tid / cm, mi = tid - ix * cm;
        if (mi >= wk.mlen) return;
        C acc[NY];
        for (int h = 0; h < H; ++h) {
            C v[NY];
#pragma unroll
            for (int j = 0; j < NY; ++j) {
                const int ky = t->pad ? 2 * j + h : j;
                v[j] = tile[(ky * Nx + ix) * cm + mi];
            }
            Fft<C, NY, 1>::run(v);
            if (h) {
                Fft<C, NY, 1>::tw2(v);
#pragma unroll
                for (int iy = 0; iy < NY; ++iy) acc[iy] = cadd(acc[iy], v[iy]);
            } else {
#pragma unroll
                for (int iy = 0; iy < NY; ++iy) acc[iy] = v[iy];
            }
        }
        const size_t off = ((size_t)wk.w * NY * Nx + ix) * b + wk.m0 + mi;
        const size_t ys = (size_t)Nx * b;
        C* __restrict__ dst = static_cast<C*>(t->out) + off;
        const R alpha = (R)t->alpha;
        if (t->addend) {
            const C* __restrict__ add = static_cast<const C*>(t->addend) + off;
            const R beta = (R)t->beta;
#pragma unroll
            for (int iy = 0; iy < NY; ++iy) {
                const C a = add[iy * ys];
                dst[iy * ys] = cmake<C>(acc[iy].x * alpha + a.x * beta, acc[iy].y * alpha + a.y * beta);
            }
        } else {
#pragma unroll
            for (int iy = 0; iy < NY; ++iy) dst[iy * ys] = cscale(acc[iy], alpha);
        }
    }
};

template<typename C>
__global__ void __launch_bounds__(512) fft_inv_kernel(FftTask t0, const FftTask* tasks, int ntasks) {
    extern __shared__ unsigned char smem_raw[];
    C* tile = reinterpret_cast<C*>(smem_raw);
    const FftTask tl = ntasks > 0 ? *find_task(tasks, ntasks) : t0;
    const FftTask* t = &tl;
    const int local = blockIdx.x - t->block_begin;
    Work wk;
    wk.w = local / t->nmc;
    const int mc = local - wk.w * t->nmc;
    wk.m0 = mc * t->cm;
    wk.mlen = min(t->cm, t->b - wk.m0);
    dispatch_n<InvX, C>(t->Nx, tl, wk, tile);
    __syncthreads();
    dispatch_n<InvY, C>(t->Ny, tl, wk, (const C*)tile);
}

// ---------------------------------------------------------------- host side

static const size_t kLdsBudget = 160 * 1024;

static int elem_bytes(int prec) { return prec == P64 ? 16 : 8; }

void plan_fft_tasks(int prec, FftTask* tasks, int ntasks, int* grid, int* block, size_t* lds) {
    const int eb = elem_bytes(prec);
    int g = 0, blk = 64;
    size_t l = 0;
    for (int i = 0; i < ntasks; ++i) {
        FftTask& t = tasks[i];
        const int H = t.pad ? 2 : 1;
        const int Py = H * t.Ny;
        // 64-byte contiguous runs per series group; shrink when LDS would overflow
        int cm = 64 / eb;
        if (cm > t.b) cm = t.b;
        while (cm > 1 && (size_t)Py * t.Nx * cm * eb > kLdsBudget) cm >>= 1;
        while (cm > 1 && (Py > t.Nx ? Py : t.Nx) * cm > 512) cm >>= 1;
        t.cm = cm;
        t.nmc = (t.b + cm - 1) / cm;
        t.block_begin = g;
        g += t.nmc * t.W;
        int thr = (Py > t.Nx ? Py : t.Nx) * cm;
        thr = (thr + 63) / 64 * 64;
        if (thr > blk) blk = thr;
        const size_t ll = (size_t)Py * t.Nx * cm * eb;
        if (ll > l) l = ll;
    }
    *grid = g;
    *block = blk;
    *lds = l;
}

template<typename C>
static hipError_t launch_fwd_t(const FftTask* th, const FftTask* td, int ntasks, hipStream_t s) {
    // the host copy is already planned (cm, nmc, block_begin filled)
    int grid = 0, block = 64;
    size_t lds = 0;
    const int eb = sizeof(C);
    for (int i = 0; i < ntasks; ++i) {
        const FftTask& t = th[i];
        const int H = t.pad ? 2 : 1, Py = H * t.Ny;
        grid = t.block_begin + t.nmc * t.W > grid ? t.block_begin + t.nmc * t.W : grid;
        int thr = ((Py > t.Nx ? Py : t.Nx) * t.cm + 63) / 64 * 64;
        if (thr > block) block = thr;
        size_t ll = (size_t)Py * t.Nx * t.cm * eb;
        if (ll > lds) lds = ll;
    }
    if (grid == 0) return hipSuccess;
    hipLaunchKernelGGL(fft_fwd_kernel<C>, dim3(grid), dim3(block), lds, s, th[0],
                       ntasks > 1 ? td : nullptr, ntasks > 1 ? ntasks : 0);
    return hipGetLastError();
}

template<typename C>
static hipError_t launch_inv_t(const FftTask* th, const FftTask* td, int ntasks, hipStream_t s) {
    int grid = 0, block = 64;
    size_t lds = 0;
    const int eb = sizeof(C);
    for (int i = 0; i < ntasks; ++i) {
        const FftTask& t = th[i];
        const int H = t.pad ? 2 : 1, Py = H * t.Ny;
        grid = t.block_begin + t.nmc * t.W > grid ? t.block_begin + t.nmc * t.W : grid;
        int thr = ((Py > t.Nx ? Py : t.Nx) * t.cm + 63) / 64 * 64;
        if (thr > block) block = thr;
        size_t ll = (size_t)Py * t.Nx * t.cm * eb;
        if (ll > lds) lds = ll;
    }
    if (grid == 0) return hipSuccess;
    hipLaunchKernelGGL(fft_inv_kernel<C>, dim3(grid), dim3(block), lds, s, th[0],
                       ntasks > 1 ? td : nullptr, ntasks > 1 ? ntasks : 0);
    return hipGetLastError();
}

static bool lds_attr_done[2] = {false, false};

static void set_lds_attr() {
    if (lds_attr_done[0]) return;
    (void)hipFuncSetAttribute((const void*)fft_fwd_kernel<float2>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsBudget);
    (void)hipFuncSetAttribute((const void*)fft_fwd_kernel<double2>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsBudget);
    (void)hipFuncSetAttribute((const void*)fft_inv_kernel<float2>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsBudget);
    (void)hipFuncSetAttribute((const void*)fft_inv_kernel<double2>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsBudget);
    lds_attr_done[0] = true;
}

hipError_t launch_fft_fwd(int prec, const FftTask* th, const FftTask* td, int ntasks, hipStream_t s) {
    set_lds_attr();
    if (prec == P64) return launch_fwd_t<double2>(th, td, ntasks, s);
    return launch_fwd_t<float2>(th, td, ntasks, s);
}

hipError_t launch_fft_inv(int prec, const FftTask* th, const FftTask* td, int ntasks, hipStream_t s) {
    set_lds_attr();
    if (prec == P64) return launch_inv_t<double2>(th, td, ntasks, s);
    return launch_inv_t<float2>(th, td, ntasks, s);
}

}  // namespace mlfft
