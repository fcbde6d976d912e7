// Kernels of the learned correction to the block-circulant preconditioner.
//
// The complex field of one column, y[w][iy][ix][m], is a real NHWC image with
// 2b channels (channel 2m + part).  The network is four 3x3 convolutions with
// zero "same" padding and no bias, 2b -> H -> H -> H -> 2b, ReLU after the first
// three.  Each convolution sees bf16 inputs and bf16 weights and accumulates in
// FP32 on the MFMA units (v_mfma_f32_16x16x32_bf16) as an implicit GEMM:
// rows = pixels, reduction = (tap, input channel), columns = output channels.
// Activations are stored as bf16 NHWC with the channel count padded to a
// multiple of 32 (zeros in the padding), so one reduction step of 32 never
// straddles two taps.  Training runs the same forward, then FP32 backward
// kernels (input and weight gradients) that use the bf16-rounded operands of
// the forward, then Adam on FP32 master weights.
#include "internal.h"
#include "net.h"

namespace mlfft {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short ushortx8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// ---------------------------------------------------------------- normalisation

// Per column w (one workgroup): s = ||y_w||, phi = arg y_w[n*] with n* the first
// index of the largest |y|; yhat = y exp(-i phi) / s (FP32, vector layout) and
// a0 = bf16(yhat) as NHWC with cpad channels.  s = 0 gives yhat = 0.
__global__ void __launch_bounds__(256) normalise_kernel(const float2* __restrict__ y, size_t N, int npix, int b,
                                                        int cpad, float2* __restrict__ yhat,
                                                        unsigned short* __restrict__ a0, double* __restrict__ scale,
                                                        double2* __restrict__ phase) {
    __shared__ double rs[4];
    __shared__ double rm[4];
    __shared__ long ri[4];
    __shared__ double s_norm;
    __shared__ double2 s_ph;
    const int w = blockIdx.x;
    const float2* yw = y + (size_t)w * N;
    double acc = 0.0;
    double best = -1.0;
    long bi = 0;
    for (size_t n = threadIdx.x; n < N; n += blockDim.x) {
        const float2 v = yw[n];
        const double m2 = (double)v.x * v.x + (double)v.y * v.y;
        acc += m2;
        if (m2 > best) { best = m2; bi = (long)n; }
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    acc = wsum(acc);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double ob = __shfl_xor(best, o, 64);
        const long oi = __shfl_xor(bi, o, 64);
        if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
    }
    if (lane == 0) { rs[wave] = acc; rm[wave] = best; ri[wave] = bi; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        double bb = -1.0;
        long ii = 0;
        for (int q = 0; q < (int)(blockDim.x >> 6); ++q) {
            t += rs[q];
            if (rm[q] > bb || (rm[q] == bb && ri[q] < ii)) { bb = rm[q]; ii = ri[q]; }
        }
        const double s = sqrt(t);
        const float2 v = yw[ii];
        const double mag = sqrt((double)v.x * v.x + (double)v.y * v.y);
        s_norm = s;
        s_ph = mag > 0.0 ? make_double2(v.x / mag, v.y / mag) : make_double2(1.0, 0.0);
        scale[w] = s;
        phase[w] = s_ph;
    }
    __syncthreads();
    const double s = s_norm;
    const double inv = s > 0.0 ? 1.0 / s : 0.0;
    const double2 ph = s_ph;
    float2* yh = yhat + (size_t)w * N;
    for (size_t n = threadIdx.x; n < N; n += blockDim.x) {
        const float2 v = yw[n];
        // y * conj(ph) / s
        const double re = ((double)v.x * ph.x + (double)v.y * ph.y) * inv;
        const double im = ((double)v.y * ph.x - (double)v.x * ph.y) * inv;
        const float2 o = make_float2((float)re, (float)im);
        yh[n] = o;
        const size_t pix = n / b;
        const int m = (int)(n - pix * b);
        uint32_t* dst = reinterpret_cast<uint32_t*>(a0 + ((size_t)w * npix + pix) * cpad + 2 * m);
        *dst = (uint32_t)f32_to_bf16_bits(o.x) | ((uint32_t)f32_to_bf16_bits(o.y) << 16);
    }
    // zero the padding channels
    const int padc = cpad - 2 * b;
    if (padc > 0) {
        for (size_t e = threadIdx.x; e < (size_t)npix * padc; e += blockDim.x) {
            const size_t pix = e / padc;
            a0[((size_t)w * npix + pix) * cpad + 2 * b + (e - pix * padc)] = 0;
        }
    }
}

// Targets of training: ehat = e exp(-i phi) / s as FP32 NHWC (cpad channels, zero padding).
__global__ void target_kernel(const float2* __restrict__ e, size_t N, int npix, int b, int cpad,
                              const double* __restrict__ scale, const double2* __restrict__ phase,
                              float* __restrict__ tgt) {
    const int w = blockIdx.y;
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (size_t)npix * cpad) return;
    const size_t pix = t / cpad;
    const int c = (int)(t - pix * cpad);
    float val = 0.f;
    if (c < 2 * b) {
        const double s = scale[w];
        const double inv = s > 0.0 ? 1.0 / s : 0.0;
        const double2 ph = phase[w];
        const float2 v = e[(size_t)w * N + pix * b + (c >> 1)];
        val = (c & 1) ? (float)(((double)v.y * ph.x - (double)v.x * ph.y) * inv)
                      : (float)(((double)v.x * ph.x + (double)v.y * ph.y) * inv);
    }
    tgt[(size_t)w * npix * cpad + t] = val;
}

// ---------------------------------------------------------------- convolution (forward)

// out[n][p][co] = sum_{tap, ci} wt[co][tap][ci] * act[n][p + off(tap)][ci]
// act: bf16 [nimg][H*Wd][cin]; wt: bf16 [cout][9][cin] (cin, cout multiples of 32);
// OUT_BF16_RELU: out = bf16(relu(.)) with cout channels, else FP32.
// Workgroup: 4 waves x 64 pixels (4 groups of 16 per wave), 64 output channels (4 groups of 16).
template<int OUT_BF16_RELU>
__global__ void __launch_bounds__(256) conv3x3_fwd_kernel(const unsigned short* __restrict__ act,
                                                          const unsigned short* __restrict__ wt, void* __restrict__ out,
                                                          int nimg, int H, int Wd, int cin, int cout) {
    // Each wave computes 4 x 16 pixels x 64 channels: per reduction step of 32
    // it loads 4 activation and 4 weight fragments for 16 MFMAs.
    constexpr int PG = 4;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int npix = H * Wd;
    const long M = (long)nimg * npix;
    const int kg = lane >> 4;                 // which 8 of the 32 reduction entries
    const int c0 = blockIdx.y * 64;
    const int ngroups = min(4, (cout - c0) >> 4);
    const long pbase = ((long)blockIdx.x * 4 + wave) * (16 * PG);
    int n[PG], i[PG], j[PG];
    bool prow[PG];
#pragma unroll
    for (int pg = 0; pg < PG; ++pg) {
        const long p = pbase + pg * 16 + (lane & 15);
        prow[pg] = p < M;
        n[pg] = 0; i[pg] = 0; j[pg] = 0;
        if (prow[pg]) {
            n[pg] = (int)(p / npix);
            const int q = (int)(p - (long)n[pg] * npix);
            i[pg] = q / Wd;
            j[pg] = q - i[pg] * Wd;
        }
    }
    floatx4 acc[PG][4];
#pragma unroll
    for (int pg = 0; pg < PG; ++pg)
#pragma unroll
        for (int g = 0; g < 4; ++g) acc[pg][g] = floatx4{0.f, 0.f, 0.f, 0.f};
    const ushortx8 zero8 = ushortx8{0, 0, 0, 0, 0, 0, 0, 0};
    for (int tap = 0; tap < 9; ++tap) {
        const unsigned short* arow[PG];
        bool ok[PG];
#pragma unroll
        for (int pg = 0; pg < PG; ++pg) {
            const int ii = i[pg] + tap / 3 - 1, jj = j[pg] + tap % 3 - 1;
            ok[pg] = prow[pg] && ii >= 0 && ii < H && jj >= 0 && jj < Wd;
            arow[pg] = act + ((size_t)n[pg] * npix + (size_t)(ok[pg] ? ii * Wd + jj : 0)) * cin + 8 * kg;
        }
        for (int ci = 0; ci < cin; ci += 32) {
            ushortx8 av[PG], bv[4];
#pragma unroll
            for (int pg = 0; pg < PG; ++pg) av[pg] = ok[pg] ? *reinterpret_cast<const ushortx8*>(arow[pg] + ci) : zero8;
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                const int co = c0 + g * 16 + (lane & 15);
                bv[g] = g < ngroups ? *reinterpret_cast<const ushortx8*>(wt + ((size_t)co * 9 + tap) * cin + ci + 8 * kg)
                                    : zero8;
            }
#pragma unroll
            for (int pg = 0; pg < PG; ++pg)
#pragma unroll
                for (int g = 0; g < 4; ++g)
                    if (g < ngroups)
                        acc[pg][g] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, av[pg]),
                                                                             __builtin_bit_cast(bf16x8, bv[g]), acc[pg][g],
                                                                             0, 0, 0);
        }
    }
    // lane holds rows 4*(lane/16)+r (pixels) of column lane%16 (channel) in each group
#pragma unroll
    for (int pg = 0; pg < PG; ++pg) {
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            if (g >= ngroups) continue;
            const int co = c0 + g * 16 + (lane & 15);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const long pr = pbase + pg * 16 + 4 * kg + r;
                if (pr >= M) continue;
                const float v = acc[pg][g][r];
                if (OUT_BF16_RELU) {
                    static_cast<unsigned short*>(out)[(size_t)pr * cout + co] = f32_to_bf16_bits(v > 0.f ? v : 0.f);
                } else {
                    static_cast<float*>(out)[(size_t)pr * cout + co] = v;
                }
            }
        }
    }
}

// z = s e^{i phi} (yhat + netout) in the vector layout; a column whose result is
// not finite falls back to the plain input y and is flagged.
__global__ void __launch_bounds__(256) finish_kernel(const float2* __restrict__ y, const float2* __restrict__ yhat,
                                                     const float* __restrict__ netout, size_t N, int b, int cpad,
                                                     const double* __restrict__ scale,
                                                     const double2* __restrict__ phase, float2* __restrict__ z,
                                                     int* __restrict__ fallback) {
    __shared__ int bad;
    const int w = blockIdx.x;
    if (threadIdx.x == 0) bad = 0;
    __syncthreads();
    const double s = scale[w];
    const double2 ph = phase[w];
    const float2* yh = yhat + (size_t)w * N;
    float2* zw = z + (size_t)w * N;
    int mybad = 0;
    for (size_t n = threadIdx.x; n < N; n += blockDim.x) {
        const size_t pix = n / b;
        const int m = (int)(n - pix * b);
        const float* o = netout + ((size_t)w * (N / b) + pix) * cpad + 2 * m;
        const double re = (double)yh[n].x + o[0], im = (double)yh[n].y + o[1];
        const float2 v = make_float2((float)(s * (re * ph.x - im * ph.y)), (float)(s * (re * ph.y + im * ph.x)));
        if (!isfinite(v.x) || !isfinite(v.y)) mybad = 1;
        zw[n] = v;
    }
    if (mybad) atomicOr(&bad, 1);
    __syncthreads();
    if (bad) {
        for (size_t n = threadIdx.x; n < N; n += blockDim.x) zw[n] = y[(size_t)w * N + n];
        if (threadIdx.x == 0 && fallback) fallback[w] += 1;
    }
}

// ---------------------------------------------------------------- training

// Loss of every sample and dL/d(netout) = 2 (yhat + out - tgt) / (||tgt||^2 B) (FP32 NHWC).
__global__ void __launch_bounds__(256) loss_grad_kernel(const float2* __restrict__ yhat, const float* __restrict__ out,
                                                        const float* __restrict__ tgt, size_t N, int b, int cpad,
                                                        int B, float* __restrict__ gout, double* __restrict__ loss) {
    __shared__ double r1[4], r2[4];
    __shared__ double den_s;
    const int w = blockIdx.x;
    const int npix = (int)(N / b);
    const size_t base = (size_t)w * npix * cpad;
    double dd = 0.0, tt = 0.0;
    for (size_t e = threadIdx.x; e < (size_t)npix * cpad; e += blockDim.x) {
        const size_t pix = e / cpad;
        const int c = (int)(e - pix * cpad);
        if (c >= 2 * b) continue;
        const float2 yv = yhat[(size_t)w * N + pix * b + (c >> 1)];
        const double t = (c & 1) ? yv.y : yv.x;
        const double d = t + out[base + e] - tgt[base + e];
        dd += d * d;
        tt += (double)tgt[base + e] * tgt[base + e];
    }
    dd = wsum(dd);
    tt = wsum(tt);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) { r1[wave] = dd; r2[wave] = tt; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0, c = 0.0;
        for (int q = 0; q < (int)(blockDim.x >> 6); ++q) { a += r1[q]; c += r2[q]; }
        den_s = c;
        loss[w] = c > 0.0 ? a / c : 0.0;
    }
    __syncthreads();
    const double den = den_s;
    const double f = den > 0.0 ? 2.0 / (den * B) : 0.0;
    for (size_t e = threadIdx.x; e < (size_t)npix * cpad; e += blockDim.x) {
        const size_t pix = e / cpad;
        const int c = (int)(e - pix * cpad);
        float gv = 0.f;
        if (c < 2 * b) {
            const float2 yv = yhat[(size_t)w * N + pix * b + (c >> 1)];
            const double t = (c & 1) ? yv.y : yv.x;
            gv = (float)(f * (t + out[base + e] - tgt[base + e]));
        }
        gout[base + e] = gv;
    }
}

// ---------------------------------------------------------------- gradients on MFMA (FP32)

// Pixel p of the batch, decoded as image n and position (i, j), stepped by 4.
struct PixPos {
    int n, i, j;
    __device__ __forceinline__ void set(long p, int H, int Wd) {
        const int npix = H * Wd;
        n = (int)(p / npix);
        const int q = (int)(p - (long)n * npix);
        i = q / Wd;
        j = q - i * Wd;
    }
    __device__ __forceinline__ void advance4(int H, int Wd) {
        j += 4;
        while (j >= Wd) { j -= Wd; if (++i == H) { i = 0; ++n; } }
    }
};

// Weight gradient as a GEMM over the batch's pixels, split into chunks:
// part[c][co][tap][ci] = sum over the pixels p of chunk c of g[p][co] a[p + off(tap)][ci]
// (v_mfma_f32_16x16x4f32: rows co, columns ci, reduction over 4 pixels per step).
// A wave owns a 16 x 16 (co, ci) tile for all nine taps; the four waves of a
// workgroup take consecutive ci tiles of one co tile and one pixel chunk.
// g: FP32 [P][cout]; act: bf16 [P][cin]; cin, cout multiples of 16 (of 32 here).
__global__ void __launch_bounds__(256) conv3x3_wgrad_mfma_kernel(const float* __restrict__ g,
                                                                 const unsigned short* __restrict__ act,
                                                                 float* __restrict__ part, int nimg, int H, int Wd,
                                                                 int cin, int cout, int pch) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int col = lane & 15, k = lane >> 4;
    const int nct = cin >> 4;
    const int ct = blockIdx.x * 4 + wave;                  // ci tile
    const int co0 = blockIdx.y * 16, ci0 = ct * 16;
    const int chunk = blockIdx.z;
    const long P = (long)nimg * H * Wd;
    const long p0 = (long)chunk * pch;
    const long p1 = min(P, p0 + pch);
    if (ct >= nct) return;
    floatx4 acc[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) acc[t] = floatx4{0.f, 0.f, 0.f, 0.f};
    const int npix = H * Wd;
    PixPos pp;
    pp.set(p0 + k, H, Wd);
    for (long p = p0 + k; p - k < p1; p += 4) {
        const bool in = p < p1;
        const float av = in ? g[p * cout + co0 + col] : 0.f;
        float bv[9];
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            const int ii = pp.i + t / 3 - 1, jj = pp.j + t % 3 - 1;
            const bool ok = in && ii >= 0 && ii < H && jj >= 0 && jj < Wd;
            bv[t] = ok ? bf16_bits_to_f32(act[((size_t)pp.n * npix + ii * Wd + jj) * cin + ci0 + col]) : 0.f;
        }
#pragma unroll
        for (int t = 0; t < 9; ++t) acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv[t], acc[t], 0, 0, 0);
        pp.advance4(H, Wd);
    }
    // lane holds rows co0 + 4k + r of column ci0 + col
    float* dst = part + (size_t)chunk * cout * 9 * cin;
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r)
            dst[((size_t)(co0 + 4 * k + r) * 9 + t) * cin + ci0 + col] = acc[t][r];
}

// dw[e] = sum over the chunks of part[c][e], in chunk order
__global__ void __launch_bounds__(256) chunk_sum_kernel(const float* __restrict__ part, float* __restrict__ dw, long n,
                                                        int nchunk) {
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    float s = 0.f;
    for (int c = 0; c < nchunk; ++c) s += part[(size_t)c * n + e];
    dw[e] = s;
}

// Input gradient as a GEMM: gin[p][ci] = relu'(a[p][ci]) sum_{tap, co} g[p - off(tap)][co] w[co][tap][ci]
// (v_mfma_f32_16x16x4f32: rows = 16 pixels, columns = 16 ci, reduction over 4 co per step and
// the nine taps).  A wave owns 16 pixels x 64 ci (four column tiles).
__global__ void __launch_bounds__(256) conv3x3_dgrad_mfma_kernel(const float* __restrict__ g,
                                                                 const unsigned short* __restrict__ wt,
                                                                 const unsigned short* __restrict__ amask,
                                                                 float* __restrict__ gin, int nimg, int H, int Wd,
                                                                 int cin, int cout) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int row = lane & 15, k = lane >> 4;
    const long P = (long)nimg * H * Wd;
    const int npix = H * Wd;
    const long pt = ((long)blockIdx.x * 4 + wave) * 16;    // first pixel of the wave's tile
    const int c0 = blockIdx.y * 64;
    const int ngroups = min(4, (cin - c0) >> 4);
    if (pt >= P) return;
    // this lane's pixel of the A operand (row) and its position
    const long pa = pt + row;
    PixPos pp;
    pp.set(pa < P ? pa : P - 1, H, Wd);
    floatx4 acc[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[q] = floatx4{0.f, 0.f, 0.f, 0.f};
    for (int tap = 0; tap < 9; ++tap) {
        // output pixel (i - di + 1, j - dj + 1) read this pixel through tap (di, dj)
        const int oi = pp.i - tap / 3 + 1, oj = pp.j - tap % 3 + 1;
        const bool ok = pa < P && oi >= 0 && oi < H && oj >= 0 && oj < Wd;
        const float* __restrict__ gp = g + ((size_t)pp.n * npix + (ok ? oi * Wd + oj : 0)) * cout;
        const unsigned short* __restrict__ wp = wt + (size_t)tap * cin;
        for (int co = 0; co < cout; co += 4) {
            const float av = ok ? gp[co + k] : 0.f;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (q < ngroups) {
                    const float bv = bf16_bits_to_f32(wp[(size_t)(co + k) * 9 * cin + c0 + q * 16 + row]);
                    acc[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc[q], 0, 0, 0);
                }
            }
        }
    }
    // lane holds rows (pixels) pt + 4k + r of column (ci) c0 + q * 16 + row
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if (q >= ngroups) continue;
        const int ci = c0 + q * 16 + row;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const long p = pt + 4 * k + r;
            if (p >= P) continue;
            const size_t e = (size_t)p * cin + ci;
            gin[e] = bf16_bits_to_f32(amask[e]) > 0.f ? acc[q][r] : 0.f;
        }
    }
}

// Adam on the FP32 master weights (layout [co][ci][3][3] of one layer, unpadded),
// gradient taken from the padded [co][tap][ci] layout; then the bf16 copy.
__global__ void adam_kernel(float* __restrict__ wmaster, float* __restrict__ m, float* __restrict__ v,
                            const float* __restrict__ dw, unsigned short* __restrict__ wbf, int cin, int cout,
                            int cinp, float lr, float b1, float b2, float eps, float c1, float c2) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long)cout * cin * 9) return;
    const int tap = (int)(t % 9);
    const int ci = (int)((t / 9) % cin);
    const int co = (int)(t / (9L * cin));
    const size_t pidx = ((size_t)co * 9 + tap) * cinp + ci;
    const float gr = dw[pidx];
    const float mm = b1 * m[t] + (1.f - b1) * gr;
    const float vv = b2 * v[t] + (1.f - b2) * gr * gr;
    m[t] = mm;
    v[t] = vv;
    const float mh = mm / c1, vh = vv / c2;
    const float nw = wmaster[t] - lr * mh / (sqrtf(vh) + eps);
    wmaster[t] = nw;
    wbf[pidx] = f32_to_bf16_bits(nw);
}

// bf16 padded copy of FP32 master weights ([co][ci][3][3] -> [co][tap][cinp], zeros elsewhere)
__global__ void pack_weights_kernel(const float* __restrict__ wmaster, unsigned short* __restrict__ wbf, int cin, int cout,
                                    int cinp, int coutp) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long)coutp * 9 * cinp) return;
    const int ci = (int)(t % cinp);
    const int tap = (int)((t / cinp) % 9);
    const int co = (int)(t / (9L * cinp));
    float v = 0.f;
    if (co < cout && ci < cin) v = wmaster[((size_t)co * cin + ci) * 9 + tap];
    wbf[t] = f32_to_bf16_bits(v);
}

// gradient in the padded layout -> master layout [co][ci][3][3]
__global__ void unpack_grad_kernel(const float* __restrict__ dwp, float* __restrict__ dw, int cin, int cout, int cinp) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long)cout * cin * 9) return;
    const int tap = (int)(t % 9);
    const int ci = (int)((t / 9) % cin);
    const int co = (int)(t / (9L * cin));
    dw[t] = dwp[((size_t)co * 9 + tap) * cinp + ci];
}

// ---------------------------------------------------------------- launchers

static dim3 g1(long n) { return dim3((unsigned)((n + 255) / 256)); }

hipError_t n_normalise(const float2* y, size_t N, int W, int npix, int b, int cpad, float2* yhat, unsigned short* a0,
                       double* scale, double2* phase, hipStream_t s) {
    hipLaunchKernelGGL(normalise_kernel, dim3(W), dim3(256), 0, s, y, N, npix, b, cpad, yhat, a0, scale, phase);
    return hipGetLastError();
}

hipError_t n_target(const float2* e, size_t N, int W, int npix, int b, int cpad, const double* scale,
                    const double2* phase, float* tgt, hipStream_t s) {
    hipLaunchKernelGGL(target_kernel, dim3((unsigned)(((size_t)npix * cpad + 255) / 256), W), dim3(256), 0, s, e, N,
                       npix, b, cpad, scale, phase, tgt);
    return hipGetLastError();
}

hipError_t n_conv_fwd(const unsigned short* act, const unsigned short* wt, void* out, int nimg, int H, int Wd,
                      int cin, int cout, int bf16_relu, hipStream_t s) {
    const long M = (long)nimg * H * Wd;
    dim3 grid((unsigned)((M + 255) / 256), (unsigned)((cout + 63) / 64));
    if (bf16_relu)
        hipLaunchKernelGGL(conv3x3_fwd_kernel<1>, grid, dim3(256), 0, s, act, wt, out, nimg, H, Wd, cin, cout);
    else
        hipLaunchKernelGGL(conv3x3_fwd_kernel<0>, grid, dim3(256), 0, s, act, wt, out, nimg, H, Wd, cin, cout);
    return hipGetLastError();
}

hipError_t n_finish(const float2* y, const float2* yhat, const float* netout, size_t N, int W, int b, int cpad,
                    const double* scale, const double2* phase, float2* z, int* fallback, hipStream_t s) {
    hipLaunchKernelGGL(finish_kernel, dim3(W), dim3(256), 0, s, y, yhat, netout, N, b, cpad, scale, phase, z, fallback);
    return hipGetLastError();
}

hipError_t n_loss_grad(const float2* yhat, const float* out, const float* tgt, size_t N, int W, int b, int cpad,
                       float* gout, double* loss, hipStream_t s) {
    hipLaunchKernelGGL(loss_grad_kernel, dim3(W), dim3(256), 0, s, yhat, out, tgt, N, b, cpad, W, gout, loss);
    return hipGetLastError();
}

hipError_t n_dgrad(const float* g, const unsigned short* wt, const unsigned short* amask, float* gin, int nimg, int H,
                   int Wd, int cin, int cout, hipStream_t s) {
    if (cin % 16 || cout % 4) return hipErrorInvalidValue;
    const long P = (long)nimg * H * Wd;
    dim3 grid((unsigned)((P + 63) / 64), (unsigned)((cin + 63) / 64));
    hipLaunchKernelGGL(conv3x3_dgrad_mfma_kernel, grid, dim3(256), 0, s, g, wt, amask, gin, nimg, H, Wd, cin, cout);
    return hipGetLastError();
}

int n_wgrad_chunks(long P, int cin, int cout) {
    // enough (ci tile group, co tile, chunk) workgroups to fill the chip, chunks of at least 64 pixels
    const long tiles = (long)((cin / 16 + 3) / 4) * (cout / 16);
    long nc = (2048 + tiles - 1) / tiles;
    nc = std::min(nc, std::max(1L, P / 64));
    return (int)std::max(1L, nc);
}

hipError_t n_wgrad(const float* g, const unsigned short* act, float* dw, float* part, int nimg, int H, int Wd, int cin,
                   int cout, hipStream_t s) {
    if (cin % 16 || cout % 16) return hipErrorInvalidValue;
    const long P = (long)nimg * H * Wd;
    const int nc = n_wgrad_chunks(P, cin, cout);
    int pch = (int)((P + nc - 1) / nc);
    pch = (pch + 3) / 4 * 4;
    const int nchunk = (int)((P + pch - 1) / pch);
    dim3 grid((unsigned)((cin / 16 + 3) / 4), (unsigned)(cout / 16), (unsigned)nchunk);
    hipLaunchKernelGGL(conv3x3_wgrad_mfma_kernel, grid, dim3(256), 0, s, g, act, part, nimg, H, Wd, cin, cout, pch);
    const long n = (long)cout * 9 * cin;
    hipLaunchKernelGGL(chunk_sum_kernel, g1(n), dim3(256), 0, s, part, dw, n, nchunk);
    return hipGetLastError();
}

hipError_t n_adam(float* wmaster, float* m, float* v, const float* dw, unsigned short* wbf, int cin, int cout, int cinp,
                  float lr, float b1, float b2, float eps, float c1, float c2, hipStream_t s) {
    hipLaunchKernelGGL(adam_kernel, g1((long)cout * cin * 9), dim3(256), 0, s, wmaster, m, v, dw, wbf, cin, cout, cinp,
                       lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t n_pack_weights(const float* wmaster, unsigned short* wbf, int cin, int cout, int cinp, int coutp,
                          hipStream_t s) {
    hipLaunchKernelGGL(pack_weights_kernel, g1((long)coutp * 9 * cinp), dim3(256), 0, s, wmaster, wbf, cin, cout, cinp,
                       coutp);
    return hipGetLastError();
}

hipError_t n_unpack_grad(const float* dwp, float* dw, int cin, int cout, int cinp, hipStream_t s) {
    hipLaunchKernelGGL(unpack_grad_kernel, g1((long)cout * cin * 9), dim3(256), 0, s, dwp, dw, cin, cout, cinp);
    return hipGetLastError();
}

}  // namespace mlfft

namespace mlfft {

// FP32 NHWC with c channels -> bf16 NHWC with cpad channels (zero padding)
__global__ void pack_nhwc_kernel(const float* __restrict__ x, unsigned short* __restrict__ a, long total, int c, int cpad) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= total * cpad) return;
    const long p = t / cpad;
    const int ch = (int)(t - p * cpad);
    a[t] = ch < c ? f32_to_bf16_bits(x[p * c + ch]) : (unsigned short)0;
}

// FP32 NHWC with cpad channels -> FP32 NHWC with c channels
__global__ void unpack_nhwc_kernel(const float* __restrict__ o, float* __restrict__ x, long total, int c, int cpad) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= total * c) return;
    const long p = t / c;
    x[t] = o[p * cpad + (t - p * c)];
}

hipError_t n_pack_nhwc(const float* x, unsigned short* a, long npix_total, int c, int cpad, hipStream_t s) {
    hipLaunchKernelGGL(pack_nhwc_kernel, g1(npix_total * cpad), dim3(256), 0, s, x, a, npix_total, c, cpad);
    return hipGetLastError();
}

hipError_t n_unpack_nhwc(const float* o, float* x, long npix_total, int c, int cpad, hipStream_t s) {
    hipLaunchKernelGGL(unpack_nhwc_kernel, g1(npix_total * c), dim3(256), 0, s, o, x, npix_total, c, cpad);
    return hipGetLastError();
}

}  // namespace mlfft
