// Batched per-RHS restarted GMRES building blocks (Sec. III-C: GMRES driven by
// a matvec and a preconditioner; one independent Krylov space per right-hand
// side, all W of them advanced together).
//
// Storage: the Krylov basis is Vb[i][w][n] (i-th basis vector of column w,
// n < N = Nx*Ny*b) in the inner precision (complex64 or complex128); the
// Hessenberg matrices, Givens rotations and least-squares right-hand sides are
// complex128 per column: H[w][i][j] ((m+1) x m, row-major), cs[w][j],
// sn[w][j], g[w][i].  All inner products and norms accumulate in FP64.
// state[w]: 0 = iterating in this cycle, 1 = done for this cycle, 2 = inactive.
// Columns of several arrays share one launch: column w of a vector starts at
// element coff[w] and has cN[w] entries; basis vector i lives at i * S.
#include "internal.h"
#include "krylov.h"

namespace mlfft {

template<typename C> struct Acc;   // widen a stored complex to complex128
template<> struct Acc<float2> { static __device__ __forceinline__ double2 w(float2 a) { return make_double2(a.x, a.y); } };
template<> struct Acc<double2> { static __device__ __forceinline__ double2 w(double2 a) { return a; } };

template<typename C> __device__ __forceinline__ C narrow(double2 a);
template<> __device__ __forceinline__ float2 narrow<float2>(double2 a) { return make_float2((float)a.x, (float)a.y); }
template<> __device__ __forceinline__ double2 narrow<double2>(double2 a) { return a; }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Block-wide sums (256 threads = 4 waves) of the per-thread values vals[i] for
// the i < CNT with keep(i) (a condition uniform over the block); results land in
// out[] (LDS) for all threads.  red holds 4 * CNT doubles.  The loop bound is a
// compile-time constant so vals[] stays in registers.
template<int CNT, typename K>
__device__ __forceinline__ void block_sum_if(const double* vals, K keep, double* red, double* out) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
    for (int i = 0; i < CNT; ++i) {
        if (keep(i)) {
            const double s = wave_sum(vals[i]);
            if (lane == 0) red[wave * CNT + i] = s;
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < CNT; i += blockDim.x) {
        if (keep(i)) {
            double s = 0.0;
            for (int q = 0; q < nw; ++q) s += red[q * CNT + i];
            out[i] = s;
        }
    }
    __syncthreads();
}

// the same for vals[i], i < lim, and the last value vals[CNT-1]
template<int CNT>
__device__ __forceinline__ void block_sum(const double* vals, int lim, double* red, double* out) {
    block_sum_if<CNT>(vals, [=](int i) { return i < lim || i == CNT - 1; }, red, out);
}

// Per-column norms ||x_w||_2 in FP64.
template<typename C>
__global__ void __launch_bounds__(256) colnorm_kernel(const C* __restrict__ x, const size_t* __restrict__ coff,
                                                      const int* __restrict__ cN, double* __restrict__ out) {
    __shared__ double red[4 * 72];
    __shared__ double res[1];
    const C* xw = x + coff[blockIdx.x];
    const size_t N = cN[blockIdx.x];
    double s = 0.0;
    for (size_t n = threadIdx.x; n < N; n += blockDim.x) {
        const double2 v = Acc<C>::w(xw[n]);
        s = fma(v.x, v.x, fma(v.y, v.y, s));
    }
    block_sum<1>(&s, 0, red, res);
    if (threadIdx.x == 0) out[blockIdx.x] = sqrt(res[0]);
}

// One Arnoldi step for every iterating column: orthogonalise u = Vb[j+1] against
// the stored basis V = Vb[0..j] (classical Gram-Schmidt, applied twice when
// orth == 2), store the coefficients in H[:, j] and the normalised remainder in
// Vb[j+1].
//
// A column is cut into chunks of kArnChunk entries, one workgroup each, so that
// a launch has many more workgroups than the chip has CUs whatever W is.  Two
// passes over the j+2 vectors:
//   dots    per chunk: partial sums of h1 = Vᴴu and ||u||², and with orth == 2
//           also of g = Vᴴv_j, column j of the Gram matrix G = VᴴV of the
//           stored (rounded) basis
//   update  h1, ||u||² and g summed over the column's chunks; with orth == 2 the
//           second projection is formed from G rather than from a second pass:
//           Vᴴ(u - V h1) = h1 - G h1 holds exactly, so h2 = h1 - G h1, h = h1 + h2
//           and beta² = ||u - V h||² = ||u||² - 2 Re(hᴴh1) + hᴴGh; with orth == 1
//           h = h1 and beta² = ||u||² - ||h1||².  Then v_{j+1} = (u - V h) / beta.
// Columns 0..j-1 of G were formed by the earlier steps of the cycle and are kept
// per Krylov column in FP64.  Every workgroup of a column reduces that column's
// partials itself, in the same order, so the result does not depend on
// scheduling.
constexpr int kArnT = 256;
constexpr int kArnE = 32;
constexpr int kArnChunk = kArnT * kArnE;

__device__ __forceinline__ int chunk_column(const int* __restrict__ choff, int W, int c) {
    int lo = 0, hi = W - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (choff[mid] <= c) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// out[i] = sum over the column's chunks of part[i][chunk], i < cnt, in a fixed
// order, by the threads of one workgroup (used when columns have few chunks).
__device__ __forceinline__ void reduce_parts(const double* __restrict__ part, int nchT, int c0, int nch, int cnt,
                                             double* out) {
    for (int i = threadIdx.x; i < cnt; i += blockDim.x) {
        const double* __restrict__ row = part + (size_t)i * nchT + c0;
        double s = 0.0;
        for (int q = 0; q < nch; ++q) s += row[q];
        out[i] = s;
    }
}

// hsum[w][i] = sum over the column's chunks of part[i][chunk], i < cnt, in a
// fixed order (strided per-thread sums, then a fixed tree): one workgroup per
// iterating column.  Partial sums are stored coefficient-major, part[i][chunk],
// so this read is coalesced.
__global__ void __launch_bounds__(256) arnoldi_reduce_kernel(const double* __restrict__ part, int nchT,
                                                             const int* __restrict__ choff,
                                                             const int* __restrict__ state, int stride, int cnt,
                                                             double* __restrict__ hsum) {
    __shared__ double red[4];
    const int w = blockIdx.x;
    if (state[w] != 0) return;
    const int c0 = choff[w], nch = choff[w + 1] - c0;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int i = 0; i < cnt; ++i) {
        const double* __restrict__ row = part + (size_t)i * nchT + c0;
        double s = 0.0;
        for (int q = threadIdx.x; q < nch; q += blockDim.x) s += row[q];
        s = wave_sum(s);
        if (lane == 0) red[wave] = s;
        __syncthreads();
        if (threadIdx.x == 0) hsum[(size_t)w * stride + i] = (red[0] + red[1]) + (red[2] + red[3]);
        __syncthreads();
    }
}

template<typename C, int MAXJ, int GRAM>
__global__ void __launch_bounds__(256) arnoldi_dots_kernel(const C* __restrict__ Vb, int j, size_t vstride,
                                                           const size_t* __restrict__ coff, const int* __restrict__ cN,
                                                           const int* __restrict__ choff, int W,
                                                           const int* __restrict__ state, double* __restrict__ out,
                                                           int nchT) {
    // vals: [0, 2 MAXJ) Vᴴu, [2 MAXJ, 4 MAXJ) Vᴴv_j (GRAM), last ||u||²
    constexpr int NV = GRAM ? 4 * MAXJ + 1 : 2 * MAXJ + 1;
    __shared__ double red[4 * NV];
    __shared__ double sh[NV];
    const int c = blockIdx.x;
    const int w = chunk_column(choff, W, c);
    if (state[w] != 0) return;
    const int c0 = choff[w];
    const size_t N = cN[w];
    const size_t n0 = (size_t)(c - c0) * kArnChunk;
    const C* __restrict__ V = Vb + coff[w];
    const C* __restrict__ u = Vb + (size_t)(j + 1) * vstride + coff[w];
    double vals[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) vals[i] = 0.0;
    for (int k = 0; k < kArnE; ++k) {
        const size_t n = n0 + (size_t)k * kArnT + threadIdx.x;
        if (n >= N) break;
        // every load is issued unconditionally, its index clamped to j, so that
        // they are all in flight together; the sums of slots beyond j are unused
        C vv[MAXJ];
#pragma unroll
        for (int i = 0; i < MAXJ; ++i) vv[i] = V[(size_t)(i < j ? i : j) * vstride + n];
        const double2 x = Acc<C>::w(u[n]);
        vals[NV - 1] = fma(x.x, x.x, fma(x.y, x.y, vals[NV - 1]));
        const double2 y = Acc<C>::w(vv[MAXJ - 1]);       // v_j (j < MAXJ)
#pragma unroll
        for (int i = 0; i < MAXJ; ++i) {
            const double2 v = Acc<C>::w(vv[i]);
            vals[2 * i] = fma(v.x, x.x, fma(v.y, x.y, vals[2 * i]));
            vals[2 * i + 1] = fma(v.x, x.y, fma(-v.y, x.x, vals[2 * i + 1]));
            if (GRAM) {
                vals[2 * MAXJ + 2 * i] = fma(v.x, y.x, fma(v.y, y.y, vals[2 * MAXJ + 2 * i]));
                vals[2 * MAXJ + 2 * i + 1] = fma(v.x, y.y, fma(-v.y, y.x, vals[2 * MAXJ + 2 * i + 1]));
            }
        }
    }
    const int J2 = 2 * (j + 1);
    block_sum_if<NV>(vals, [=](int i) { return (i < NV - 1 && (i % (2 * MAXJ)) < J2) || i == NV - 1; }, red, sh);
    // partial-sum rows: [0, 2J) Vᴴu, 2J ||u||², [2J + 1, 4J + 1) Vᴴv_j (J = j + 1)
    for (int i = threadIdx.x; i < J2; i += blockDim.x) {
        out[(size_t)i * nchT + c] = sh[i];
        if (GRAM) out[(size_t)(J2 + 1 + i) * nchT + c] = sh[2 * MAXJ + i];
    }
    if (threadIdx.x == 0) out[(size_t)J2 * nchT + c] = sh[NV - 1];
}

__device__ __forceinline__ double2 cmul_d(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

template<typename C, int MAXJ>
__global__ void __launch_bounds__(256) arnoldi_update_kernel(C* __restrict__ Vb, int j, size_t vstride,
                                                             const size_t* __restrict__ coff,
                                                             const int* __restrict__ cN,
                                                             const int* __restrict__ choff, int W,
                                                             double2* __restrict__ H, int m,
                                                             const int* __restrict__ state, int orth,
                                                             const double* __restrict__ hsum,
                                                             const double* __restrict__ part, int nchT, int stride,
                                                             int inl, double2* __restrict__ gram) {
    __shared__ double sm[4 * MAXJ + 1];
    __shared__ double2 hh[MAXJ];
    __shared__ double2 tt[MAXJ];
    __shared__ double2 gs[MAXJ * MAXJ];
    const int c = blockIdx.x;
    const int w = chunk_column(choff, W, c);
    const int c0 = choff[w], nch = choff[w + 1] - c0;
    const size_t N = cN[w];
    const size_t n0 = (size_t)(c - c0) * kArnChunk;
    const C* __restrict__ V = Vb + coff[w];
    C* __restrict__ u = Vb + (size_t)(j + 1) * vstride + coff[w];
    if (state[w] != 0) {
        // retired column: keep its unused basis slot at zero so repeated products stay finite
        for (int k = 0; k < kArnE; ++k) {
            const size_t n = n0 + (size_t)k * kArnT + threadIdx.x;
            if (n >= N) break;
            u[n] = narrow<C>(make_double2(0.0, 0.0));
        }
        return;
    }
    const int J = j + 1, J2 = 2 * J;
    const int cnt = orth == 2 ? 2 * J2 + 1 : J2 + 1;
    if (inl) reduce_parts(part, nchT, c0, nch, cnt, sm);
    else
        for (int i = threadIdx.x; i < cnt; i += blockDim.x) sm[i] = hsum[(size_t)w * stride + i];
    __syncthreads();
    const int t = threadIdx.x;
    const double unorm2 = sm[J2];
    const double* h1 = sm;
    double beta2;
    if (orth == 2) {
        // Gram matrix of the stored basis: column k at Gw[k (m+1) + i] for i <= k;
        // column j (this step's) comes from the fresh sums, the others from the
        // earlier steps.  The (j+1)² entries are gathered into LDS in one round
        // of loads.
        double2* Gw = gram + (size_t)w * (m + 1) * (m + 1);
        const double* gj = sm + J2 + 1;
        if (c == c0 && t <= j) Gw[(size_t)j * (m + 1) + t] = make_double2(gj[2 * t], gj[2 * t + 1]);
        for (int e = t; e < J * J; e += blockDim.x) {
            const int i = e / J, k = e - i * J;
            double2 g;
            if (i <= k) g = k == j ? make_double2(gj[2 * i], gj[2 * i + 1]) : Gw[(size_t)k * (m + 1) + i];
            else {
                g = i == j ? make_double2(gj[2 * k], gj[2 * k + 1]) : Gw[(size_t)i * (m + 1) + k];
                g.y = -g.y;
            }
            gs[i * MAXJ + k] = g;
        }
        __syncthreads();
        auto G = [&](int i, int k) -> double2 { return gs[i * MAXJ + k]; };
        // h = h1 + (h1 - G h1)
        if (t <= j) {
            double2 a = make_double2(0.0, 0.0);
            for (int k = 0; k <= j; ++k) {
                const double2 p = cmul_d(G(t, k), make_double2(h1[2 * k], h1[2 * k + 1]));
                a.x += p.x;
                a.y += p.y;
            }
            hh[t] = make_double2(2.0 * h1[2 * t] - a.x, 2.0 * h1[2 * t + 1] - a.y);
        }
        if (t > j && t < MAXJ) hh[t] = make_double2(0.0, 0.0);
        __syncthreads();
        // G h
        if (t <= j) {
            double2 a = make_double2(0.0, 0.0);
            for (int k = 0; k <= j; ++k) {
                const double2 p = cmul_d(G(t, k), hh[k]);
                a.x += p.x;
                a.y += p.y;
            }
            tt[t] = a;
        }
        __syncthreads();
        // ||u - V h||² = ||u||² - 2 Re(hᴴh1) + Re(hᴴ G h)
        double s1 = 0.0, s2 = 0.0;
        for (int i = 0; i <= j; ++i) {
            s1 += hh[i].x * h1[2 * i] + hh[i].y * h1[2 * i + 1];
            s2 += hh[i].x * tt[i].x + hh[i].y * tt[i].y;
        }
        beta2 = unorm2 - 2.0 * s1 + s2;
    } else {
        if (t <= j) hh[t] = make_double2(h1[2 * t], h1[2 * t + 1]);
        if (t > j && t < MAXJ) hh[t] = make_double2(0.0, 0.0);
        __syncthreads();
        double hn = 0.0;
        for (int i = 0; i <= j; ++i) hn += hh[i].x * hh[i].x + hh[i].y * hh[i].y;
        beta2 = unorm2 - hn;
    }
    double beta = beta2 > 0.0 ? sqrt(beta2) : 0.0;
    // happy breakdown: the new direction vanishes relative to the product.  beta²
    // is a difference of terms of size up to a few ||u||², whose FP64 rounding is
    // about 1e-14 ||u||²; below 1e-13 ||u||² (beta below 3e-7 ||u||) it is not
    // resolved and the direction counts as vanished.  The FP64 true residual of
    // the refinement loop decides whether the column is really converged.
    const bool brk = !(beta2 > 1e-13 * unorm2) || !(beta > 1e-300);
    if (brk) beta = 0.0;
    const double inv = brk ? 0.0 : 1.0 / beta;
    for (int k = 0; k < kArnE; ++k) {
        const size_t n = n0 + (size_t)k * kArnT + threadIdx.x;
        if (n >= N) break;
        // unconditional loads (index clamped to j) with zero coefficients beyond j
        C vv[MAXJ];
#pragma unroll
        for (int i = 0; i < MAXJ; ++i) vv[i] = V[(size_t)(i < j ? i : j) * vstride + n];
        double2 up = Acc<C>::w(u[n]);
#pragma unroll
        for (int i = 0; i < MAXJ; ++i) {
            const double2 v = Acc<C>::w(vv[i]);
            const double2 h = hh[i];
            up.x -= h.x * v.x - h.y * v.y;
            up.y -= h.x * v.y + h.y * v.x;
        }
        u[n] = narrow<C>(make_double2(up.x * inv, up.y * inv));
    }
    if (c == c0) {
        if (t <= j) H[((size_t)w * (m + 1) + t) * m + j] = hh[t];
        if (t == 0) H[((size_t)w * (m + 1) + j + 1) * m + j] = make_double2(beta, 0.0);
    }
}

// Apply the earlier rotations to H[:, j], build rotation j, update g, record
// the residual estimate |g[j+1]| and retire columns that reached their target.
__global__ void givens_kernel(double2* __restrict__ H, double* __restrict__ cs, double2* __restrict__ sn,
                              double2* __restrict__ g, int j, int m, int W, int* __restrict__ state,
                              const double* __restrict__ target, int* __restrict__ kcyc, int* __restrict__ iters,
                              double* __restrict__ est, double* __restrict__ hist, int hist_len,
                              const double* __restrict__ scale) {
    const int w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= W || state[w] != 0) return;
    double2* Hw = H + (size_t)w * (m + 1) * m;
    double* csw = cs + (size_t)w * m;
    double2* snw = sn + (size_t)w * m;
    double2* gw = g + (size_t)w * (m + 1);
    for (int i = 0; i < j; ++i) {
        const double2 a = Hw[i * m + j], b = Hw[(i + 1) * m + j];
        const double c = csw[i];
        const double2 s = snw[i];
        // [c, s; -conj(s), c] [a; b]
        Hw[i * m + j] = make_double2(c * a.x + (s.x * b.x - s.y * b.y), c * a.y + (s.x * b.y + s.y * b.x));
        Hw[(i + 1) * m + j] = make_double2(-(s.x * a.x + s.y * a.y) + c * b.x, -(s.x * a.y - s.y * a.x) + c * b.y);
    }
    const double2 a = Hw[j * m + j], b = Hw[(j + 1) * m + j];
    const double na = hypot(a.x, a.y), nb = hypot(b.x, b.y);
    double c;
    double2 s;
    if (nb == 0.0) { c = 1.0; s = make_double2(0.0, 0.0); }
    else if (na == 0.0) { c = 0.0; s = make_double2(b.x / nb, -b.y / nb); }
    else {
        const double r = hypot(na, nb);
        c = na / r;
        // s = (a/|a|) conj(b) / r
        const double2 ph = make_double2(a.x / na, a.y / na);
        s = make_double2((ph.x * b.x + ph.y * b.y) / r, (ph.y * b.x - ph.x * b.y) / r);
    }
    csw[j] = c;
    snw[j] = s;
    Hw[j * m + j] = make_double2(c * a.x + (s.x * b.x - s.y * b.y), c * a.y + (s.x * b.y + s.y * b.x));
    Hw[(j + 1) * m + j] = make_double2(0.0, 0.0);
    const double2 gj = gw[j];
    gw[j + 1] = make_double2(-(s.x * gj.x + s.y * gj.y), -(s.x * gj.y - s.y * gj.x));
    gw[j] = make_double2(c * gj.x, c * gj.y);
    const double e = hypot(gw[j + 1].x, gw[j + 1].y);
    est[w] = e;
    kcyc[w] = j + 1;
    const int it = ++iters[w];
    if (hist && it <= hist_len) hist[(size_t)(it - 1) * W + w] = e * (scale ? scale[w] : 1.0);
    if (!(e > target[w]) || nb == 0.0) state[w] = 1;
}

// Start a cycle: beta = ||r_w||; columns at or below target become inactive;
// v_0 = r / beta, g = (beta, 0, ...).  Three launches over the Arnoldi chunks
// (so one long column, as in the global mode, is spread over the whole chip):
// partial sums of |r|^2 per chunk, one workgroup per column for beta and the
// column state, then the scaling.
template<typename C>
__global__ void __launch_bounds__(256) cycle_norm_kernel(const C* __restrict__ r, const size_t* __restrict__ coff,
                                                         const int* __restrict__ cN, const int* __restrict__ choff,
                                                         int W, const int* __restrict__ state,
                                                         double* __restrict__ part, int nchT) {
    __shared__ double red[4 * 72];
    __shared__ double res[1];
    const int c = blockIdx.x;
    const int w = chunk_column(choff, W, c);
    if (state[w] == 2) return;
    const size_t N = cN[w];
    const size_t n0 = (size_t)(c - choff[w]) * kArnChunk;
    const C* __restrict__ rw = r + coff[w];
    double s = 0.0;
    for (int k = 0; k < kArnE; ++k) {
        const size_t n = n0 + (size_t)k * kArnT + threadIdx.x;
        if (n >= N) break;
        const double2 v = Acc<C>::w(rw[n]);
        s = fma(v.x, v.x, fma(v.y, v.y, s));
    }
    block_sum<1>(&s, 0, red, res);
    if (threadIdx.x == 0) part[c] = res[0];
}

// The three steps in one launch when every column is a single chunk (one
// workgroup per column).
template<typename C>
__global__ void __launch_bounds__(256) cycle_start_small_kernel(const C* __restrict__ r, C* __restrict__ v0,
                                                                const size_t* __restrict__ coff,
                                                                const int* __restrict__ cN, double2* __restrict__ g,
                                                                int m, int* __restrict__ state,
                                                                const double* __restrict__ target,
                                                                int* __restrict__ kcyc, double* __restrict__ est) {
    __shared__ double red[4 * 72];
    __shared__ double res[1];
    const int w = blockIdx.x;
    const size_t N = cN[w];
    C* __restrict__ vw = v0 + coff[w];
    if (state[w] == 2) {
        if (threadIdx.x == 0) kcyc[w] = 0;
        for (size_t n = threadIdx.x; n < N; n += blockDim.x) vw[n] = narrow<C>(make_double2(0.0, 0.0));
        return;
    }
    const C* __restrict__ rw = r + coff[w];
    double s = 0.0;
    for (size_t n = threadIdx.x; n < N; n += blockDim.x) {
        const double2 v = Acc<C>::w(rw[n]);
        s = fma(v.x, v.x, fma(v.y, v.y, s));
    }
    block_sum<1>(&s, 0, red, res);
    const double beta = sqrt(res[0]);
    const bool done = !(beta > target[w]);
    if (threadIdx.x == 0) {
        est[w] = beta;
        kcyc[w] = 0;
        state[w] = done ? 2 : 0;
        for (int i = 0; i <= m; ++i) g[(size_t)w * (m + 1) + i] = make_double2(i == 0 ? beta : 0.0, 0.0);
    }
    const double inv = done ? 0.0 : 1.0 / beta;
    for (size_t n = threadIdx.x; n < N; n += blockDim.x) {
        const double2 v = Acc<C>::w(rw[n]);
        vw[n] = narrow<C>(make_double2(v.x * inv, v.y * inv));
    }
}

__global__ void __launch_bounds__(256) cycle_state_kernel(const double* __restrict__ part,
                                                          const int* __restrict__ choff, double2* __restrict__ g,
                                                          int m, int* __restrict__ state,
                                                          const double* __restrict__ target, int* __restrict__ kcyc,
                                                          double* __restrict__ est, double* __restrict__ beta_out) {
    __shared__ double red[4];
    const int w = blockIdx.x;
    if (state[w] == 2) {
        if (threadIdx.x == 0) kcyc[w] = 0;
        return;
    }
    const int c0 = choff[w], nch = choff[w + 1] - c0;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double s = 0.0;
    for (int q = threadIdx.x; q < nch; q += blockDim.x) s += part[c0 + q];
    s = wave_sum(s);
    if (lane == 0) red[wave] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double beta = sqrt((red[0] + red[1]) + (red[2] + red[3]));
        const bool done = !(beta > target[w]);
        est[w] = beta;
        kcyc[w] = 0;
        state[w] = done ? 2 : 0;
        beta_out[w] = beta;
        for (int i = 0; i <= m; ++i) g[(size_t)w * (m + 1) + i] = make_double2(i == 0 ? beta : 0.0, 0.0);
    }
}

template<typename C>
__global__ void __launch_bounds__(256) cycle_scale_kernel(const C* __restrict__ r, C* __restrict__ v0,
                                                          const size_t* __restrict__ coff, const int* __restrict__ cN,
                                                          const int* __restrict__ choff, int W,
                                                          const int* __restrict__ state,
                                                          const double* __restrict__ beta) {
    const int c = blockIdx.x;
    const int w = chunk_column(choff, W, c);
    const size_t N = cN[w];
    const size_t n0 = (size_t)(c - choff[w]) * kArnChunk;
    const C* __restrict__ rw = r + coff[w];
    C* __restrict__ vw = v0 + coff[w];
    const bool off = state[w] == 2;
    const double inv = off ? 0.0 : 1.0 / beta[w];
    for (int k = 0; k < kArnE; ++k) {
        const size_t n = n0 + (size_t)k * kArnT + threadIdx.x;
        if (n >= N) break;
        const double2 v = off ? make_double2(0.0, 0.0) : Acc<C>::w(rw[n]);
        vw[n] = narrow<C>(make_double2(v.x * inv, v.y * inv));
    }
}

// y = H(1:k, 1:k)^{-1} g(1:k) per column (upper triangular after the rotations).
__global__ void lsq_kernel(const double2* __restrict__ H, const double2* __restrict__ g, double2* __restrict__ y,
                           const int* __restrict__ kcyc, int m, int W) {
    const int w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= W) return;
    const int k = kcyc[w];
    const double2* Hw = H + (size_t)w * (m + 1) * m;
    const double2* gw = g + (size_t)w * (m + 1);
    double2* yw = y + (size_t)w * m;
    for (int i = k - 1; i >= 0; --i) {
        double2 s = gw[i];
        for (int l = i + 1; l < k; ++l) {
            const double2 h = Hw[i * m + l], yl = yw[l];
            s.x -= h.x * yl.x - h.y * yl.y;
            s.y -= h.x * yl.y + h.y * yl.x;
        }
        const double2 d = Hw[i * m + i];
        const double den = d.x * d.x + d.y * d.y;
        yw[i] = den > 0.0 ? make_double2((s.x * d.x + s.y * d.y) / den, (s.y * d.x - s.x * d.y) / den)
                          : make_double2(0.0, 0.0);
    }
    for (int i = k; i < m; ++i) yw[i] = make_double2(0.0, 0.0);
}

// out_w (+)= sum_{i < k_w} y[w][i] B_i[w]  (accumulate != 0 adds to out).  KB >= every
// k_w: the KB loads are issued unconditionally (index clamped to k_w - 1) so that
// they are in flight together, with zero weights beyond k_w.
template<typename C, int KB>
__global__ void __launch_bounds__(256) combine_kernel(const C* __restrict__ B, size_t bstride,
                                                      const size_t* __restrict__ coff, const int* __restrict__ cN,
                                                      const double2* __restrict__ y, const int* __restrict__ kcyc,
                                                      int m, C* __restrict__ out, int accumulate) {
    const int w = blockIdx.y;
    const int k = kcyc[w];
    const size_t n = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= (size_t)cN[w]) return;
    const size_t o = coff[w] + n;
    if (k <= 0) {
        if (!accumulate) out[o] = narrow<C>(make_double2(0.0, 0.0));
        return;
    }
    C bb[KB];
#pragma unroll
    for (int i = 0; i < KB; ++i) bb[i] = B[(size_t)(i < k ? i : k - 1) * bstride + o];
    double2 acc = accumulate ? Acc<C>::w(out[o]) : make_double2(0.0, 0.0);
#pragma unroll
    for (int i = 0; i < KB; ++i) {
        const double2 yc = y[(size_t)w * m + (i < k ? i : k - 1)];
        const double f = i < k ? 1.0 : 0.0;
        const double2 b = Acc<C>::w(bb[i]);
        acc.x += f * (yc.x * b.x - yc.y * b.y);
        acc.y += f * (yc.x * b.y + yc.y * b.x);
    }
    out[o] = narrow<C>(acc);
}

// dst += src (per column, same precision)
template<typename C>
__global__ void add_cols_kernel(C* __restrict__ dst, const C* __restrict__ src, const size_t* __restrict__ coff,
                                const int* __restrict__ cN) {
    const int w = blockIdx.y;
    const size_t n = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= (size_t)cN[w]) return;
    const size_t o = coff[w] + n;
    const double2 a = Acc<C>::w(dst[o]), b = Acc<C>::w(src[o]);
    dst[o] = narrow<C>(make_double2(a.x + b.x, a.y + b.y));
}

// dst = src * s[w] (per column real scale; converts precision)
template<typename A, typename B>
__global__ void scale_cols_kernel(const A* __restrict__ src, B* __restrict__ dst, const size_t* __restrict__ coff,
                                  const int* __restrict__ cN, const double* __restrict__ s, int invert) {
    const int w = blockIdx.y;
    const size_t n = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= (size_t)cN[w]) return;
    const size_t o = coff[w] + n;
    double f = s ? s[w] : 1.0;
    if (invert) f = f > 0.0 ? 1.0 / f : 0.0;
    const double2 v = Acc<A>::w(src[o]);
    dst[o] = narrow<B>(make_double2(v.x * f, v.y * f));
}

// x64 += s[w] * d (d in the inner precision), or x64 = s[w] * d and zero in the
// unmasked columns when assign is set
template<typename C>
__global__ void axpy_cols_kernel(double2* __restrict__ x, const C* __restrict__ d, const size_t* __restrict__ coff,
                                 const int* __restrict__ cN, const double* __restrict__ s, const int* __restrict__ mask,
                                 int assign) {
    const int w = blockIdx.y;
    const bool on = !mask || mask[w];
    if (!on && !assign) return;
    const size_t n = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= (size_t)cN[w]) return;
    const size_t o = coff[w] + n;
    if (!on) {
        x[o] = make_double2(0.0, 0.0);
        return;
    }
    const double f = s ? s[w] : 1.0;
    const double2 v = Acc<C>::w(d[o]);
    double2 xo = assign ? make_double2(0.0, 0.0) : x[o];
    xo.x = fma(f, v.x, xo.x);
    xo.y = fma(f, v.y, xo.y);
    x[o] = xo;
}

// ------------------------------------------------------------------ launchers

static dim3 cols_grid(size_t maxN, int W) { return dim3((unsigned)((maxN + 255) / 256), (unsigned)W); }

template<typename C>
hipError_t k_colnorm(const void* x, const Cols& c, double* out, hipStream_t s) {
    if (c.W <= 0) return hipSuccess;
    hipLaunchKernelGGL(colnorm_kernel<C>, dim3(c.W), dim3(256), 0, s, (const C*)x, c.off, c.N, out);
    return hipGetLastError();
}

int arnoldi_chunks(size_t N) { return (int)((N + kArnChunk - 1) / kArnChunk); }

template<typename C, int MAXJ>
static hipError_t arnoldi_t(C* Vb, int j, const Cols& c, double2* H, int m, const int* state, int orth,
                            hipStream_t s) {
    const int stride = 4 * m + 3;
    const int cnt = orth == 2 ? 4 * (j + 1) + 1 : 2 * (j + 1) + 1;
    const dim3 grid((unsigned)c.nch);
    // columns of a few chunks: every workgroup reduces its column's partials itself
    // (no reduction launch); long columns: one reduction workgroup per column
    const int inl = c.maxch <= 16 ? 1 : 0;
    if (orth == 2)
        hipLaunchKernelGGL((arnoldi_dots_kernel<C, MAXJ, 1>), grid, dim3(kArnT), 0, s, (const C*)Vb, j, c.S, c.off,
                           c.N, c.choff, c.W, state, c.part1, c.nch);
    else
        hipLaunchKernelGGL((arnoldi_dots_kernel<C, MAXJ, 0>), grid, dim3(kArnT), 0, s, (const C*)Vb, j, c.S, c.off,
                           c.N, c.choff, c.W, state, c.part1, c.nch);
    if (!inl)
        hipLaunchKernelGGL(arnoldi_reduce_kernel, dim3(c.W), dim3(256), 0, s, (const double*)c.part1, c.nch, c.choff,
                           state, stride, cnt, c.hsum1);
    hipLaunchKernelGGL((arnoldi_update_kernel<C, MAXJ>), grid, dim3(kArnT), 0, s, Vb, j, c.S, c.off, c.N, c.choff,
                       c.W, H, m, state, orth, (const double*)c.hsum1, (const double*)c.part1, c.nch, stride, inl,
                       c.gram);
    return hipGetLastError();
}

template<typename C>
hipError_t k_arnoldi(void* Vb, int j, const Cols& c, double2* H, int m, const int* state, int orth, hipStream_t s) {
    if (c.nch <= 0 || !c.choff || !c.part1 || !c.hsum1 || (orth == 2 && !c.gram)) return hipErrorInvalidValue;
    if (j + 1 > m || m > 31) return hipErrorInvalidValue;
    // the kernels load a fixed number of basis vectors: exactly j + 1 up to 8,
    // then the next of 12, 16, 24, 32
    C* V = (C*)Vb;
    switch (j + 1) {
        case 1: return arnoldi_t<C, 1>(V, j, c, H, m, state, orth, s);
        case 2: return arnoldi_t<C, 2>(V, j, c, H, m, state, orth, s);
        case 3: return arnoldi_t<C, 3>(V, j, c, H, m, state, orth, s);
        case 4: return arnoldi_t<C, 4>(V, j, c, H, m, state, orth, s);
        case 5: return arnoldi_t<C, 5>(V, j, c, H, m, state, orth, s);
        case 6: return arnoldi_t<C, 6>(V, j, c, H, m, state, orth, s);
        case 7: return arnoldi_t<C, 7>(V, j, c, H, m, state, orth, s);
        case 8: return arnoldi_t<C, 8>(V, j, c, H, m, state, orth, s);
        default: break;
    }
    if (j + 1 <= 12) return arnoldi_t<C, 12>(V, j, c, H, m, state, orth, s);
    if (j + 1 <= 16) return arnoldi_t<C, 16>(V, j, c, H, m, state, orth, s);
    if (j + 1 <= 24) return arnoldi_t<C, 24>(V, j, c, H, m, state, orth, s);
    if (j + 1 <= 32) return arnoldi_t<C, 32>(V, j, c, H, m, state, orth, s);
    return hipErrorInvalidValue;
}

hipError_t k_givens(double2* H, double* cs, double2* sn, double2* g, int j, int m, int W, int* state,
                    const double* target, int* kcyc, int* iters, double* est, double* hist, int hist_len,
                    const double* scale, hipStream_t s) {
    hipLaunchKernelGGL(givens_kernel, dim3((W + 63) / 64), dim3(64), 0, s, H, cs, sn, g, j, m, W, state, target, kcyc,
                       iters, est, hist, hist_len, scale);
    return hipGetLastError();
}

template<typename C>
hipError_t k_cycle_start(const void* r, void* v0, const Cols& c, double2* g, int m, int* state, const double* target,
                         int* kcyc, double* est, hipStream_t s) {
    if (c.nch <= 0 || !c.choff || !c.part1 || !c.hsum1) return hipErrorInvalidValue;
    if (c.maxch == 1) {
        hipLaunchKernelGGL(cycle_start_small_kernel<C>, dim3(c.W), dim3(256), 0, s, (const C*)r, (C*)v0, c.off, c.N,
                           g, m, state, target, kcyc, est);
        return hipGetLastError();
    }
    const dim3 grid((unsigned)c.nch);
    hipLaunchKernelGGL(cycle_norm_kernel<C>, grid, dim3(kArnT), 0, s, (const C*)r, c.off, c.N, c.choff, c.W, state,
                       c.part1, c.nch);
    hipLaunchKernelGGL(cycle_state_kernel, dim3(c.W), dim3(256), 0, s, (const double*)c.part1, c.choff, g, m, state,
                       target, kcyc, est, c.hsum1);
    hipLaunchKernelGGL(cycle_scale_kernel<C>, grid, dim3(kArnT), 0, s, (const C*)r, (C*)v0, c.off, c.N, c.choff, c.W,
                       (const int*)state, (const double*)c.hsum1);
    return hipGetLastError();
}

hipError_t k_lsq(const double2* H, const double2* g, double2* y, const int* kcyc, int m, int W, hipStream_t s) {
    hipLaunchKernelGGL(lsq_kernel, dim3((W + 63) / 64), dim3(64), 0, s, H, g, y, kcyc, m, W);
    return hipGetLastError();
}

template<typename C>
hipError_t k_combine(const void* B, const Cols& c, const double2* y, const int* kcyc, int m, int kmax, void* out,
                     int acc, hipStream_t s) {
    if (kmax < 1 || kmax > m || m > 31) return hipErrorInvalidValue;
#define COMBINE(KB) \
    hipLaunchKernelGGL((combine_kernel<C, KB>), cols_grid(c.maxN, c.W), dim3(256), 0, s, (const C*)B, c.S, c.off, \
                       c.N, y, kcyc, m, (C*)out, acc)
    switch (kmax) {
        case 1: COMBINE(1); break;
        case 2: COMBINE(2); break;
        case 3: COMBINE(3); break;
        case 4: COMBINE(4); break;
        case 5: COMBINE(5); break;
        case 6: COMBINE(6); break;
        case 7: COMBINE(7); break;
        case 8: COMBINE(8); break;
        default:
            if (kmax <= 12) COMBINE(12);
            else if (kmax <= 16) COMBINE(16);
            else if (kmax <= 24) COMBINE(24);
            else COMBINE(32);
    }
#undef COMBINE
    return hipGetLastError();
}

template<typename C>
hipError_t k_add_cols(void* dst, const void* src, const Cols& c, hipStream_t s) {
    hipLaunchKernelGGL(add_cols_kernel<C>, cols_grid(c.maxN, c.W), dim3(256), 0, s, (C*)dst, (const C*)src, c.off,
                       c.N);
    return hipGetLastError();
}

template<typename A, typename B>
hipError_t k_scale_cols(const void* src, void* dst, const Cols& c, const double* sc, int invert, hipStream_t s) {
    hipLaunchKernelGGL((scale_cols_kernel<A, B>), cols_grid(c.maxN, c.W), dim3(256), 0, s, (const A*)src, (B*)dst,
                       c.off, c.N, sc, invert);
    return hipGetLastError();
}

template<typename C>
hipError_t k_axpy_cols(double2* x, const void* d, const Cols& c, const double* sc, const int* mask, int assign,
                       hipStream_t s) {
    hipLaunchKernelGGL(axpy_cols_kernel<C>, cols_grid(c.maxN, c.W), dim3(256), 0, s, x, (const C*)d, c.off, c.N, sc,
                       mask, assign);
    return hipGetLastError();
}

#define INST(C)                                                                                                   \
    template hipError_t k_colnorm<C>(const void*, const Cols&, double*, hipStream_t);                             \
    template hipError_t k_arnoldi<C>(void*, int, const Cols&, double2*, int, const int*, int, hipStream_t);       \
    template hipError_t k_cycle_start<C>(const void*, void*, const Cols&, double2*, int, int*, const double*,     \
                                         int*, double*, hipStream_t);                                             \
    template hipError_t k_combine<C>(const void*, const Cols&, const double2*, const int*, int, int, void*, int,  \
                                     hipStream_t);                                                                \
    template hipError_t k_add_cols<C>(void*, const void*, const Cols&, hipStream_t);                              \
    template hipError_t k_axpy_cols<C>(double2*, const void*, const Cols&, const double*, const int*, int,       \
                                       hipStream_t);
INST(float2)
INST(double2)
template hipError_t k_scale_cols<double2, float2>(const void*, void*, const Cols&, const double*, int, hipStream_t);
template hipError_t k_scale_cols<double2, double2>(const void*, void*, const Cols&, const double*, int, hipStream_t);
template hipError_t k_scale_cols<float2, float2>(const void*, void*, const Cols&, const double*, int, hipStream_t);
template hipError_t k_scale_cols<float2, double2>(const void*, void*, const Cols&, const double*, int, hipStream_t);

}  // namespace mlfft
