// Setup kernels (FP64): block spectra of the circulant embedding, the Strang
// block-circulant preconditioner's spectrum and its per-frequency inverses.
//
// Spectra (eq. multL: F^[2] C_1^[2]; eqs. circL1/circL2 for the embedding): the
// block at lag (p, q) sits at grid position (p mod Py, q mod Px), so the 2-D DFT
// of the embedded grid is, per block entry (m, n),
//     G_hat(ky, kx) = sum_{p,q} w_y(p) w_x(q) R_{p,q} exp(-2 pi i (p ky/Py + q kx/Px)).
// It is evaluated separably, one lag axis at a time, directly over the lags
// (no zero samples are visited).  The weights are 1 for the MLFFT embedding and
// the Strang fold weights (1 inside, 1/2 at the Nyquist lag, 0 outside) for the
// block-circulant preconditioner on the Ny x Nx torus.
#include "internal.h"

namespace mlfft {

// out[o][k][i] = sum_{l < L} w[l] * in[o][l][i] * exp(-2 pi i ((l + lag0) k mod P) / P)
// One workgroup: one outer index o and 64 consecutive inner indices.
__global__ void __launch_bounds__(256) lag_dft_kernel(const double2* __restrict__ in, double2* __restrict__ out,
                                                      int L, int lag0, int P, long inner,
                                                      const double* __restrict__ w) {
    __shared__ double2 tile[64 * 64];
    __shared__ double2 tw[64];
    __shared__ double wl[64];
    const int nchunks = (int)((inner + 63) / 64);
    const int o = blockIdx.x / nchunks;
    const long i0 = (long)(blockIdx.x % nchunks) * 64;
    const int li = threadIdx.x & 63, kg = threadIdx.x >> 6;
    if (threadIdx.x < P) {
        double s, c;
        sincospi(-2.0 * threadIdx.x / P, &s, &c);
        tw[threadIdx.x] = make_double2(c, s);
    }
    if (threadIdx.x < L) wl[threadIdx.x] = w ? w[threadIdx.x] : 1.0;
    const double2* src = in + (size_t)o * L * inner;
    for (int e = threadIdx.x; e < L * 64; e += blockDim.x) {
        const int l = e >> 6, ii = e & 63;
        tile[e] = (i0 + ii < inner) ? src[(size_t)l * inner + i0 + ii] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    if (i0 + li >= inner) return;
    double2* dst = out + (size_t)o * P * inner + i0 + li;
    for (int k = kg; k < P; k += 4) {
        double re = 0.0, im = 0.0;
        int e = ((lag0 % P) * k) % P;
        if (e < 0) e += P;
        for (int l = 0; l < L; ++l) {
            const double2 v = tile[l * 64 + li];
            const double2 t = tw[e];
            const double wv = wl[l];
            re = fma(wv * v.x, t.x, fma(-wv * v.y, t.y, re));
            im = fma(wv * v.x, t.y, fma(wv * v.y, t.x, im));
            e += k;
            if (e >= P) e -= P;
        }
        dst[(size_t)k * inner] = make_double2(re, im);
    }
}

hipError_t launch_lag_dft_x(const double2* R, double2* T, int nlagy, int nlagx, int lagx0, int Px,
                            const double* wx, int bb, hipStream_t s) {
    const int nchunks = (bb + 63) / 64;
    hipLaunchKernelGGL(lag_dft_kernel, dim3(nlagy * nchunks), dim3(256), 0, s, R, T, nlagx, lagx0, Px,
                       (long)bb, wx);
    return hipGetLastError();
}

hipError_t launch_lag_dft_y(const double2* T, double2* G, int nlagy, int lagy0, int Py, int Px,
                            const double* wy, int bb, hipStream_t s) {
    const long inner = (long)Px * bb;
    const int nchunks = (int)((inner + 63) / 64);
    hipLaunchKernelGGL(lag_dft_kernel, dim3(nchunks), dim3(256), 0, s, T, G, nlagy, lagy0, Py, inner, wy);
    return hipGetLastError();
}

__global__ void cast_c64_c32_kernel(const double2* __restrict__ a, float2* __restrict__ b, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        b[i] = make_float2((float)a[i].x, (float)a[i].y);
}

__global__ void cast_c64_bf16_kernel(const double2* __restrict__ a, uint32_t* __restrict__ b, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const uint32_t re = f32_to_bf16_bits((float)a[i].x), im = f32_to_bf16_bits((float)a[i].y);
        b[i] = re | (im << 16);
    }
}

static dim3 grid_for(size_t n) {
    size_t g = (n + 255) / 256;
    if (g > 65536) g = 65536;
    if (g == 0) g = 1;
    return dim3((unsigned)g);
}

hipError_t launch_cast_c64_to_c32(const double2* a, float2* b, size_t n, hipStream_t s) {
    hipLaunchKernelGGL(cast_c64_c32_kernel, grid_for(n), dim3(256), 0, s, a, b, n);
    return hipGetLastError();
}

hipError_t launch_cast_c64_to_bf16(const double2* a, uint32_t* b, size_t n, hipStream_t s) {
    hipLaunchKernelGGL(cast_c64_bf16_kernel, grid_for(n), dim3(256), 0, s, a, b, n);
    return hipGetLastError();
}

// out = alpha * x + beta * y elementwise over n complex values (y may be NULL),
// reading TI and writing TO (complex128 or complex64; the sum is formed in FP64)
template<typename TI, typename TO>
__global__ void axpby_kernel(const TI* x, const TI* y, double alpha, double beta,
                             TO* out, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        double re = alpha * (double)x[i].x, im = alpha * (double)x[i].y;
        if (y) {
            re += beta * (double)y[i].x;
            im += beta * (double)y[i].y;
        }
        TO o;
        o.x = re;
        o.y = im;
        out[i] = o;
    }
}

hipError_t launch_axpby(int in_prec, const void* x, const void* y, double alpha, double beta, int out_prec, void* out,
                        size_t n, hipStream_t s) {
    if (in_prec == P64 && out_prec == P64)
        hipLaunchKernelGGL((axpby_kernel<double2, double2>), grid_for(n), dim3(256), 0, s, (const double2*)x,
                           (const double2*)y, alpha, beta, (double2*)out, n);
    else if (in_prec == P64)
        hipLaunchKernelGGL((axpby_kernel<double2, float2>), grid_for(n), dim3(256), 0, s, (const double2*)x,
                           (const double2*)y, alpha, beta, (float2*)out, n);
    else if (out_prec == P64)
        hipLaunchKernelGGL((axpby_kernel<float2, double2>), grid_for(n), dim3(256), 0, s, (const float2*)x,
                           (const float2*)y, alpha, beta, (double2*)out, n);
    else
        hipLaunchKernelGGL((axpby_kernel<float2, float2>), grid_for(n), dim3(256), 0, s, (const float2*)x,
                           (const float2*)y, alpha, beta, (float2*)out, n);
    return hipGetLastError();
}

// Gauss-Jordan inversion with partial pivoting of nb independent b x b complex
// matrices, one workgroup per matrix.  A is destroyed (used as the left half of
// the augmented matrix in place: the inverse is built in Ainv).  rcond[i] is the
// reciprocal 1-norm condition number 1 / (||A||_1 ||A^{-1}||_1); info[i] is 0,
// or j + 1 if the j-th pivot was exactly zero.
__global__ void __launch_bounds__(256) gj_inverse_kernel(double2* __restrict__ Aall, double2* __restrict__ Xall,
                                                         double* __restrict__ rcond, int* __restrict__ info, int b) {
    extern __shared__ double smem[];
    double2* fac = reinterpret_cast<double2*>(smem);          // b factors
    double* red = smem + 2 * b;                               // 256 reduction slots
    int* redi = reinterpret_cast<int*>(red + 256);            // 256 index slots
    __shared__ double2 pivinv;
    __shared__ int piv;
    __shared__ int bad;
    double2* A = Aall + (size_t)blockIdx.x * b * b;
    double2* X = Xall + (size_t)blockIdx.x * b * b;
    const int tid = threadIdx.x, nt = blockDim.x;
    // ||A||_1 = max column sum
    double cmax = 0.0;
    for (int c = tid; c < b; c += nt) {
        double sacc = 0.0;
        for (int r = 0; r < b; ++r) { const double2 v = A[(size_t)r * b + c]; sacc += hypot(v.x, v.y); }
        cmax = fmax(cmax, sacc);
    }
    red[tid] = cmax;
    __syncthreads();
    for (int st = nt / 2; st > 0; st >>= 1) { if (tid < st) red[tid] = fmax(red[tid], red[tid + st]); __syncthreads(); }
    const double anorm = red[0];
    __syncthreads();
    for (size_t e = tid; e < (size_t)b * b; e += nt) {
        const int r = (int)(e / b), c = (int)(e % b);
        X[e] = make_double2(r == c ? 1.0 : 0.0, 0.0);
    }
    if (tid == 0) bad = 0;
    __syncthreads();
    for (int c = 0; c < b; ++c) {
        // pivot search in column c, rows c..b-1
        double best = -1.0;
        int bi = c;
        for (int r = c + tid; r < b; r += nt) {
            const double2 v = A[(size_t)r * b + c];
            const double m = hypot(v.x, v.y);
            if (m > best) { best = m; bi = r; }
        }
        red[tid] = best;
        redi[tid] = bi;
        __syncthreads();
        for (int st = nt / 2; st > 0; st >>= 1) {
            if (tid < st) {
                if (red[tid + st] > red[tid] || (red[tid + st] == red[tid] && redi[tid + st] < redi[tid])) {
                    red[tid] = red[tid + st];
                    redi[tid] = redi[tid + st];
                }
            }
            __syncthreads();
        }
        if (tid == 0) {
            piv = redi[0];
            if (!(red[0] > 0.0) && bad == 0) bad = c + 1;
        }
        __syncthreads();
        const int p = piv;
        if (p != c) {
            for (int j = tid; j < b; j += nt) {
                double2 t1 = A[(size_t)c * b + j]; A[(size_t)c * b + j] = A[(size_t)p * b + j]; A[(size_t)p * b + j] = t1;
                double2 t2 = X[(size_t)c * b + j]; X[(size_t)c * b + j] = X[(size_t)p * b + j]; X[(size_t)p * b + j] = t2;
            }
        }
        __syncthreads();
        if (tid == 0) {
            const double2 d = A[(size_t)c * b + c];
            const double den = d.x * d.x + d.y * d.y;
            pivinv = den > 0.0 ? make_double2(d.x / den, -d.y / den) : make_double2(0.0, 0.0);
        }
        __syncthreads();
        const double2 pi = pivinv;
        for (int j = tid; j < b; j += nt) {
            A[(size_t)c * b + j] = cmul(A[(size_t)c * b + j], pi);
            X[(size_t)c * b + j] = cmul(X[(size_t)c * b + j], pi);
        }
        for (int r = tid; r < b; r += nt) fac[r] = A[(size_t)r * b + c];
        __syncthreads();
        for (size_t e = tid; e < (size_t)b * b; e += nt) {
            const int r = (int)(e / b), j = (int)(e % b);
            if (r == c) continue;
            const double2 f = fac[r];
            if (f.x == 0.0 && f.y == 0.0) continue;
            A[e] = csub(A[e], cmul(f, A[(size_t)c * b + j]));
            X[e] = csub(X[e], cmul(f, X[(size_t)c * b + j]));
        }
        __syncthreads();
    }
    // ||A^{-1}||_1
    cmax = 0.0;
    for (int c = tid; c < b; c += nt) {
        double sacc = 0.0;
        for (int r = 0; r < b; ++r) { const double2 v = X[(size_t)r * b + c]; sacc += hypot(v.x, v.y); }
        cmax = fmax(cmax, sacc);
    }
    red[tid] = cmax;
    __syncthreads();
    for (int st = nt / 2; st > 0; st >>= 1) { if (tid < st) red[tid] = fmax(red[tid], red[tid + st]); __syncthreads(); }
    if (tid == 0) {
        const double xn = red[0];
        const bool ok = bad == 0 && anorm > 0.0 && isfinite(xn) && xn > 0.0;
        rcond[blockIdx.x] = ok ? 1.0 / (anorm * xn) : 0.0;
        info[blockIdx.x] = bad;
    }
}

hipError_t launch_batched_inverse(double2* A, double2* Ainv, double* rcond, int* info, int nb, int b,
                                  hipStream_t s) {
    if (nb <= 0) return hipSuccess;
    const size_t lds = (size_t)2 * b * sizeof(double) + 256 * sizeof(double) + 256 * sizeof(int);
    hipLaunchKernelGGL(gj_inverse_kernel, dim3(nb), dim3(256), lds, s, A, Ainv, rcond, info, b);
    return hipGetLastError();
}

// Replace the inverse blocks of frequencies flagged in bad[] by R00inv (the
// Kindt self-block preconditioner, Sec. III-B).
__global__ void fallback_kernel(double2* __restrict__ Sinv, const double2* __restrict__ R00inv,
                                const int* __restrict__ bad, int b) {
    if (!bad[blockIdx.x]) return;
    double2* dst = Sinv + (size_t)blockIdx.x * b * b;
    for (int e = threadIdx.x; e < b * b; e += blockDim.x) dst[e] = R00inv[e];
}

hipError_t launch_fill_identity_fallback(double2* Sinv, const double2* R00inv, const int* bad, int nb, int b,
                                         hipStream_t s) {
    if (nb <= 0) return hipSuccess;
    hipLaunchKernelGGL(fallback_kernel, dim3(nb), dim3(256), 0, s, Sinv, R00inv, bad, b);
    return hipGetLastError();
}

}  // namespace mlfft

namespace mlfft {

// flag[0] |= 1 if any of the n doubles is NaN or infinite
__global__ void nonfinite_kernel(const double* __restrict__ a, size_t n, int* __restrict__ flag) {
    int bad = 0;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        if (!isfinite(a[i])) bad = 1;
    if (bad) atomicOr(flag, 1);
}

hipError_t launch_nonfinite(const double* a, size_t n, int* flag, hipStream_t s) {
    hipLaunchKernelGGL(nonfinite_kernel, grid_for(n), dim3(256), 0, s, a, n, flag);
    return hipGetLastError();
}

// Kindt preconditioner as a per-frequency block set: every one of the nb blocks is R00inv.
__global__ void replicate_kernel(double2* __restrict__ dst, const double2* __restrict__ src, int bb) {
    double2* d = dst + (size_t)blockIdx.x * bb;
    for (int e = threadIdx.x; e < bb; e += blockDim.x) d[e] = src[e];
}

hipError_t launch_replicate(double2* dst, const double2* src, int nb, int bb, hipStream_t s) {
    if (nb <= 0) return hipSuccess;
    hipLaunchKernelGGL(replicate_kernel, dim3(nb), dim3(256), 0, s, dst, src, bb);
    return hipGetLastError();
}

}  // namespace mlfft
