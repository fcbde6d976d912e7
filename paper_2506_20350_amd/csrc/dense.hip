// Dense complex linear algebra on the device, for the direct block-Toeplitz
// solver (Sec. III-D), the row preconditioner P'_Z (Sec. III-B), the border
// blocks (Sec. III-E) and the spectrum diagnostics (Sec. V):
//  - a complex GEMM on MFMA (FP64: v_mfma_f64_16x16x4f64, FP32:
//    v_mfma_f32_16x16x4f32), column-major operands with leading dimensions and
//    batch strides, C = alpha A B + beta C;
//  - a blocked right-looking LU with partial pivoting in FP64 (panels of 32
//    columns factored by one workgroup, row interchanges, a triangular solve of
//    the block row and the trailing update on the GEMM), and the forward and
//    backward triangular solves that use it;
//  - small helpers (1-norms, identity, level-1 block assembly).
#include "dense.h"

namespace mlfft {

namespace {

constexpr int kTile = 64;      // C tile of a GEMM workgroup (64 x 64 complex values)
constexpr int kKt = 16;        // reduction step staged through LDS
constexpr int kLdsPad = 4;

template<typename T> struct DMfma;
typedef double dx4 __attribute__((ext_vector_type(4)));
typedef float fx4 __attribute__((ext_vector_type(4)));
// A operand of lane l: row l%16, column l/16; B operand: row l/16, column l%16.
// Accumulator register r of lane l: column l%16 and row 4r + l/16 (FP64),
// row 4(l/16) + r (FP32).
template<> struct DMfma<double> {
    typedef dx4 acc_t;
    typedef double2 c_t;
    static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int r) { return 4 * r + (lane >> 4); }
};
template<> struct DMfma<float> {
    typedef fx4 acc_t;
    typedef float2 c_t;
    static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

// C[M x N] = alpha A[M x K] B[K x N] + beta C, column-major, one 64 x 64 tile of C
// per workgroup of four waves (each wave a 32 x 32 quarter: 2 x 2 MFMA tiles, real
// and imaginary accumulators), the reduction staged through LDS 16 at a time with
// the next step's operands prefetched into registers.  Complex products take four
// real MFMAs (the real part subtracts Im A Im B through a negated operand).
// blockIdx.z selects the batch entry (strides sA, sB, sC in elements).
template<typename T, bool CONJA>
__global__ void __launch_bounds__(256) zgemm_kernel(int M, int N, int K, double2 alpha, const typename DMfma<T>::c_t* A,
                                                   long lda, long sA, const typename DMfma<T>::c_t* B, long ldb, long sB,
                                                   double2 beta, typename DMfma<T>::c_t* Cm, long ldc, long sC) {
    typedef DMfma<T> MM;
    typedef typename MM::c_t C;
    typedef typename MM::acc_t acc_t;
    __shared__ T sAr[kKt][kTile + kLdsPad], sAi[kKt][kTile + kLdsPad];
    __shared__ T sBr[kKt][kTile + kLdsPad], sBi[kKt][kTile + kLdsPad];
    const int tilesM = (M + kTile - 1) / kTile;
    const int tm = blockIdx.x % tilesM, tn = blockIdx.x / tilesM;
    const int row0 = tm * kTile, col0 = tn * kTile;
    A += (size_t)blockIdx.z * sA;
    B += (size_t)blockIdx.z * sB;
    Cm += (size_t)blockIdx.z * sC;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int wr = wave & 1, wc = wave >> 1;
    acc_t cr[2][2], ci[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) { cr[a][b][r] = 0; ci[a][b][r] = 0; }
    C pa[4], pb[4];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int e = tid + 256 * i;
            if (!CONJA) {
                const int ar = e & 63, ak = e >> 6;       // A: 64 consecutive rows of one column
                const int gr = row0 + ar, gk = k0 + ak;
                pa[i] = (gr < M && gk < K) ? A[(size_t)gk * lda + gr] : czero<C>();
            } else {
                // op(A) = A^H with A stored K x M: 16 consecutive rows of one stored column
                const int ak = e & 15, ar = e >> 4;
                const int gr = row0 + ar, gk = k0 + ak;
                C v = (gr < M && gk < K) ? A[(size_t)gr * lda + gk] : czero<C>();
                v.y = -v.y;
                pa[i] = v;
            }
            const int bk = e & 15, bc = e >> 4;           // B: 16 consecutive rows of one column
            const int hk = k0 + bk, hc = col0 + bc;
            pb[i] = (hk < K && hc < N) ? B[(size_t)hc * ldb + hk] : czero<C>();
        }
    };
    fetch(0);
    for (int k0 = 0; k0 < K; k0 += kKt) {
        __syncthreads();
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int e = tid + 256 * i;
            const int ak = CONJA ? (e & 15) : (e >> 6), ar = CONJA ? (e >> 4) : (e & 63);
            sAr[ak][ar] = pa[i].x;
            sAi[ak][ar] = pa[i].y;
            sBr[e & 15][e >> 4] = pb[i].x;
            sBi[e & 15][e >> 4] = pb[i].y;
        }
        __syncthreads();
        if (k0 + kKt < K) fetch(k0 + kKt);
#pragma unroll
        for (int kk = 0; kk < kKt; kk += 4) {
            const int k = kk + (lane >> 4);
            T ar[2], ai[2], br[2], bi[2];
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                ar[t] = sAr[k][wr * 32 + t * 16 + (lane & 15)];
                ai[t] = sAi[k][wr * 32 + t * 16 + (lane & 15)];
                br[t] = sBr[k][wc * 32 + t * 16 + (lane & 15)];
                bi[t] = sBi[k][wc * 32 + t * 16 + (lane & 15)];
            }
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    cr[a][b] = MM::mma(ar[a], br[b], cr[a][b]);
                    cr[a][b] = MM::mma(-ai[a], bi[b], cr[a][b]);
                    ci[a][b] = MM::mma(ar[a], bi[b], ci[a][b]);
                    ci[a][b] = MM::mma(ai[a], br[b], ci[a][b]);
                }
        }
    }
    const bool use_beta = beta.x != 0.0 || beta.y != 0.0;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const int gc = col0 + wc * 32 + b * 16 + (lane & 15);
            if (gc >= N) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int gr = row0 + wr * 32 + a * 16 + MM::row(lane, r);
                if (gr >= M) continue;
                const double xr = cr[a][b][r], xi = ci[a][b][r];
                double yr = alpha.x * xr - alpha.y * xi, yi = alpha.x * xi + alpha.y * xr;
                C* dst = Cm + (size_t)gc * ldc + gr;
                if (use_beta) {
                    const C o = *dst;
                    yr += beta.x * (double)o.x - beta.y * (double)o.y;
                    yi += beta.x * (double)o.y + beta.y * (double)o.x;
                }
                *dst = cmake<C>((T)yr, (T)yi);
            }
        }
}

__device__ __forceinline__ double cabs1(double2 a) { return fabs(a.x) + fabs(a.y); }

__device__ __forceinline__ double2 crecip(double2 a) {
    // 1 / a with scaling against overflow (Smith's method)
    if (fabs(a.x) >= fabs(a.y)) {
        const double r = a.y / a.x, d = a.x + a.y * r;
        return make_double2(1.0 / d, -r / d);
    }
    const double r = a.x / a.y, d = a.y + a.x * r;
    return make_double2(r / d, -1.0 / d);
}

// Unblocked LU with partial pivoting of the panel A[k0:n, k0:k0+nb) (nb <= 32),
// one workgroup: for each column, the row of largest |Re| + |Im| at or below the
// diagonal (the first one on ties) becomes the pivot row, the two rows are
// interchanged across the panel, the column below the diagonal is divided by the
// pivot and the rest of the panel gets the rank-1 update.  ipiv[c] = pivot row
// (absolute index); a zero pivot sets *info = c + 1 (first one) and skips the
// division, as LAPACK's zgetf2 does.
__global__ void __launch_bounds__(1024) getf2_panel_kernel(double2* A, long lda, int n, int k0, int nb, int* ipiv,
                                                           int* info) {
    __shared__ double rv[16];
    __shared__ int ri[16];
    __shared__ int s_p;
    __shared__ double2 s_u[32];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int j = 0; j < nb; ++j) {
        const int c = k0 + j;
        double2* colc = A + (size_t)c * lda;
        double best = -1.0;
        int bi = n;
        for (int r = c + tid; r < n; r += 1024) {
            const double v = cabs1(colc[r]);
            if (v > best) { best = v; bi = r; }
        }
        for (int o = 32; o > 0; o >>= 1) {
            const double ob = __shfl_xor(best, o, 64);
            const int oi = __shfl_xor(bi, o, 64);
            if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
        }
        if (lane == 0) { rv[wave] = best; ri[wave] = bi; }
        __syncthreads();
        if (tid == 0) {
            double b = rv[0];
            int p = ri[0];
            for (int w = 1; w < 16; ++w)
                if (rv[w] > b || (rv[w] == b && ri[w] < p)) { b = rv[w]; p = ri[w]; }
            if (p >= n) p = c;
            ipiv[c] = p;
            if (!(b > 0.0) && *info == 0) *info = c + 1;
            s_p = p;
        }
        __syncthreads();
        const int p = s_p;
        if (p != c && tid < nb) {
            double2* col = A + (size_t)(k0 + tid) * lda;
            const double2 t = col[c];
            col[c] = col[p];
            col[p] = t;
        }
        __syncthreads();
        const double2 piv = colc[c];
        const bool nz = piv.x != 0.0 || piv.y != 0.0;
        if (nz) {
            const double2 inv = crecip(piv);
            for (int r = c + 1 + tid; r < n; r += 1024) colc[r] = cmul(colc[r], inv);
        }
        if (tid < nb) s_u[tid] = A[(size_t)(k0 + tid) * lda + c];
        __syncthreads();
        for (int r = c + 1 + tid; r < n; r += 1024) {
            const double2 l = colc[r];
            for (int cc = j + 1; cc < nb; ++cc) {
                double2* dst = A + (size_t)(k0 + cc) * lda + r;
                *dst = csub(*dst, cmul(l, s_u[cc]));
            }
        }
        __syncthreads();
    }
}

// Row interchanges ipiv[k0 .. k1) (in that order) applied to the columns [c0, c1) of A
// (one thread per column); ipiv holds absolute row indices.
template<typename C>
__global__ void laswp_kernel(C* A, long lda, int c0, int c1, int k0, int k1, const int* ipiv) {
    const int c = c0 + blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= c1) return;
    C* col = A + (size_t)c * lda;
    for (int k = k0; k < k1; ++k) {
        const int p = ipiv[k];
        if (p != k) {
            const C t = col[k];
            col[k] = col[p];
            col[p] = t;
        }
    }
}

// B[k0:k0+nb, c] <- L^{-1} B[k0:k0+nb, c] (unit lower triangular L = the diagonal block
// of the LU at k0) for the columns c of B; UPPER: B <- U^{-1} B with the non-unit upper
// triangular diagonal block.  One thread per column of B, the block staged in LDS.
template<int NB, bool UPPER>
__global__ void __launch_bounds__(256) trsm_block_kernel(const double2* A, long lda, int k0, int nb, double2* B,
                                                         long ldb, int ncols) {
    __shared__ double2 L[NB][NB + 1];
    for (int e = threadIdx.x; e < nb * nb; e += blockDim.x) {
        const int i = e % nb, j = e / nb;
        L[i][j] = A[(size_t)(k0 + j) * lda + k0 + i];
    }
    __syncthreads();
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncols) return;
    double2* col = B + (size_t)c * ldb + k0;
    double2 x[NB];
#pragma unroll
    for (int i = 0; i < NB; ++i) x[i] = i < nb ? col[i] : make_double2(0.0, 0.0);
    if (!UPPER) {
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            if (i >= nb) break;
            double2 s = x[i];
#pragma unroll
            for (int l = 0; l < i; ++l) s = csub(s, cmul(L[i][l], x[l]));
            x[i] = s;
        }
    } else {
#pragma unroll
        for (int i = NB - 1; i >= 0; --i) {
            if (i >= nb) continue;
            double2 s = x[i];
#pragma unroll
            for (int l = i + 1; l < NB; ++l)
                if (l < nb) s = csub(s, cmul(L[i][l], x[l]));
            const double2 d = L[i][i];
            x[i] = (d.x != 0.0 || d.y != 0.0) ? cmul(s, crecip(d)) : s;
        }
    }
#pragma unroll
    for (int i = 0; i < NB; ++i)
        if (i < nb) col[i] = x[i];
}

// out[c] = sum_r |A[r, c]| (complex modulus) for the n columns of an m x n matrix
__global__ void colabs_kernel(const double2* A, long lda, int m, int n, double* out) {
    const int c = blockIdx.x;
    if (c >= n) return;
    const double2* col = A + (size_t)c * lda;
    double s = 0.0;
    for (int r = threadIdx.x; r < m; r += blockDim.x) s += hypot(col[r].x, col[r].y);
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    __shared__ double ws[4];
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) out[c] = ws[0] + ws[1] + ws[2] + ws[3];
}

// *out = max_i v[i] (one workgroup)
__global__ void max_kernel(const double* v, int n, double* out) {
    double m = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) m = fmax(m, v[i]);
    for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
    __shared__ double ws[4];
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) *out = fmax(fmax(ws[0], ws[1]), fmax(ws[2], ws[3]));
}

// A (m x n, column-major) = identity
template<typename C>
__global__ void identity_kernel(C* A, long lda, int m, int n) {
    const size_t tot = (size_t)m * n;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < tot; e += (size_t)gridDim.x * blockDim.x) {
        const int r = (int)(e % m), c = (int)(e / m);
        A[(size_t)c * lda + r] = cmake<C>(r == c ? 1.0 : 0.0, 0.0);
    }
}

// The level-1 blocks T^[1]_p (p = p0 .. p0 + np - 1) as dense column-major matrices of
// order n = Nx b: T_p[(ix b + m), (jx b + n')] = R_{p, ix - jx}[m][n'] with the unique
// blocks R in the library layout [p + Ny - 1][q + Nx - 1][m][n'] (eq. Tblock).
__global__ void level1_kernel(const double2* R, int Nx, int Ny, int b, int p0, int np, double2* T) {
    const int n = Nx * b;
    const size_t per = (size_t)n * n, tot = per * np;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < tot; e += (size_t)gridDim.x * blockDim.x) {
        const int pi = (int)(e / per);
        const size_t rem = e - (size_t)pi * per;
        const int col = (int)(rem / n), row = (int)(rem - (size_t)col * n);
        const int ix = row / b, m = row - ix * b, jx = col / b, nn = col - jx * b;
        const int p = p0 + pi, q = ix - jx;
        T[e] = R[(((size_t)(p + Ny - 1) * (2 * Nx - 1) + (q + Nx - 1)) * b + m) * b + nn];
    }
}

// out = alpha X + beta Y over an m x n block (column-major, leading dimensions; Y may
// be NULL; out may be X or Y itself)
template<typename C>
__global__ void axpby2d_kernel(int m, int n, double2 alpha, const C* X, long ldx, double2 beta, const C* Y, long ldy,
                               C* out, long ldo) {
    const size_t tot = (size_t)m * n;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < tot; e += (size_t)gridDim.x * blockDim.x) {
        const int r = (int)(e % m), c = (int)(e / m);
        const C x = X[(size_t)c * ldx + r];
        double yr = alpha.x * (double)x.x - alpha.y * (double)x.y, yi = alpha.x * (double)x.y + alpha.y * (double)x.x;
        if (Y) {
            const C y = Y[(size_t)c * ldy + r];
            yr += beta.x * (double)y.x - beta.y * (double)y.y;
            yi += beta.x * (double)y.y + beta.y * (double)y.x;
        }
        out[(size_t)c * ldo + r] = cmake<C>(yr, yi);
    }
}

// out (n x m, column-major, ld ldo) = A^T for the m x n column-major A (ld lda)
template<typename C>
__global__ void transpose_kernel(const C* A, long lda, int m, int n, C* out, long ldo) {
    const size_t tot = (size_t)m * n;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < tot; e += (size_t)gridDim.x * blockDim.x) {
        const int r = (int)(e % m), c = (int)(e / m);
        out[(size_t)r * ldo + c] = A[(size_t)c * lda + r];
    }
}

// out = conj(x) over n complex128 values (out may be x)
__global__ void conj_kernel(const double2* x, double2* out, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const double2 v = x[i];
        out[i] = make_double2(v.x, -v.y);
    }
}

// Eigenvalues of T = L^{-1} M L^{-H} for l x l Hermitian G = L L^H (positive definite)
// and M (column-major, overwritten), one workgroup: Cholesky of G in place, two
// forward substitutions (X = L^{-1} M, T = L^{-1} X^H, since M = M^H), then cyclic
// two-sided Jacobi on T with the round-robin pairing (l/2 disjoint rotations at a
// time; each rotation's angle, the inner one, from its 2 x 2 block before the round,
// columns then rows updated).  out[i] = sqrt(max(lambda_i, 0)) in descending order.
// X: l x l scratch; info: 1 if G is not positive definite.
__global__ void __launch_bounds__(1024) herm_sqrt_eig_kernel(double2* G, double2* M, double2* X, int l, int sweeps,
                                                             double* out, int* info) {
    const int tid = threadIdx.x, nt = blockDim.x;
    __shared__ double s_d;
    __shared__ int s_bad;
    if (tid == 0) s_bad = 0;
    __syncthreads();
    auto at = [l](double2* A, int r, int c) -> double2& { return A[(size_t)c * l + r]; };
    // Cholesky, lower triangle of G
    for (int j = 0; j < l; ++j) {
        if (tid == 0) {
            const double d = at(G, j, j).x;
            if (!(d > 0.0)) s_bad = 1;
            s_d = d > 0.0 ? sqrt(d) : 1.0;
        }
        __syncthreads();
        const double dj = s_d;
        for (int i = j + tid; i < l; i += nt) {
            double2& g = at(G, i, j);
            g = i == j ? make_double2(dj, 0.0) : make_double2(g.x / dj, g.y / dj);
        }
        __syncthreads();
        // trailing update G[i][k] -= L[i][j] conj(L[k][j]) for j < k <= i
        const int rem = l - j - 1;
        for (int e = tid; e < rem * rem; e += nt) {
            const int i = j + 1 + e % rem, k = j + 1 + e / rem;
            if (k > i) continue;
            const double2 li = at(G, i, j), lk = at(G, k, j);
            double2& g = at(G, i, k);
            g = csub(g, cconjmul(lk, li));        // li * conj(lk)
        }
        __syncthreads();
    }
    // X = L^{-1} M, one column per thread
    for (int c = tid; c < l; c += nt)
        for (int i = 0; i < l; ++i) {
            double2 v = at(M, i, c);
            for (int k = 0; k < i; ++k) v = csub(v, cmul(at(G, i, k), at(X, k, c)));
            const double d = at(G, i, i).x;
            at(X, i, c) = make_double2(v.x / d, v.y / d);
        }
    __syncthreads();
    // T = L^{-1} X^H into M
    for (int c = tid; c < l; c += nt)
        for (int i = 0; i < l; ++i) {
            const double2 xh = at(X, c, i);
            double2 v = make_double2(xh.x, -xh.y);
            for (int k = 0; k < i; ++k) v = csub(v, cmul(at(G, i, k), at(M, k, c)));
            const double d = at(G, i, i).x;
            at(M, i, c) = make_double2(v.x / d, v.y / d);
        }
    __syncthreads();
    // symmetrise (T is Hermitian up to rounding): keep the average of T and T^H
    for (int e = tid; e < l * l; e += nt) {
        const int i = e % l, k = e / l;
        if (k < i) {
            const double2 a = at(M, i, k), b = at(M, k, i);
            const double2 m = make_double2(0.5 * (a.x + b.x), 0.5 * (a.y - b.y));
            at(M, i, k) = m;
            at(M, k, i) = make_double2(m.x, -m.y);
        } else if (k == i) {
            at(M, i, i).y = 0.0;
        }
    }
    __syncthreads();
    // round-robin Jacobi; n even (a dummy index n - 1 = l when l is odd is skipped)
    const int n = (l + 1) & ~1;
    __shared__ int pp[512], qq[512];
    __shared__ double cs[512], sn[512];
    __shared__ double2 ph[512];
    for (int sw = 0; sw < sweeps; ++sw) {
        for (int r = 0; r < n - 1; ++r) {
            // pairs of round r: position 0 fixed, the others rotated by r
            for (int k = tid; k < n / 2; k += nt) {
                auto player = [n, r](int pos) { return pos == 0 ? 0 : 1 + (pos - 1 + r) % (n - 1); };
                int p = player(k), q = player(n - 1 - k);
                if (p > q) { const int t = p; p = q; q = t; }
                pp[k] = p;
                qq[k] = q;
                double c = 1.0, sv = 0.0;
                double2 u = make_double2(1.0, 0.0);
                if (q < l) {
                    const double2 t = at(M, p, q);
                    const double rr = hypot(t.x, t.y);
                    if (rr > 0.0) {
                        u = make_double2(t.x / rr, t.y / rr);
                        // the inner rotation, |theta| <= pi/4 (the outer one swaps p and q and slows
                        // the convergence of the sweeps)
                        double th = 0.5 * atan2(2.0 * rr, at(M, p, p).x - at(M, q, q).x);
                        if (th > 0.7853981633974483) th -= 1.5707963267948966;
                        c = cos(th);
                        sv = sin(th);
                    }
                }
                cs[k] = c;
                sn[k] = sv;
                ph[k] = u;
            }
            __syncthreads();
            // columns: T <- T U
            for (int e = tid; e < (n / 2) * l; e += nt) {
                const int k = e / l, row = e - k * l;
                const int p = pp[k], q = qq[k];
                if (q >= l || sn[k] == 0.0) continue;
                const double c = cs[k], sv = sn[k];
                const double2 u = ph[k];
                const double2 a = at(M, row, p), b = at(M, row, q);
                // col p: a c + b s conj(u);  col q: -a s u + b c
                at(M, row, p) = cadd(cscale(a, c), cscale(cconjmul(u, b), sv));
                at(M, row, q) = csub(cscale(b, c), cscale(cmul(a, u), sv));
            }
            __syncthreads();
            // rows: T <- U^H T
            for (int e = tid; e < (n / 2) * l; e += nt) {
                const int k = e / l, col = e - k * l;
                const int p = pp[k], q = qq[k];
                if (q >= l || sn[k] == 0.0) continue;
                const double c = cs[k], sv = sn[k];
                const double2 u = ph[k];
                const double2 a = at(M, p, col), b = at(M, q, col);
                // row p: c a + s u b;  row q: -s conj(u) a + c b
                at(M, p, col) = cadd(cscale(a, c), cscale(cmul(u, b), sv));
                at(M, q, col) = csub(cscale(b, c), cscale(cconjmul(u, a), sv));
            }
            __syncthreads();
        }
    }
    // sqrt of the diagonal, ranked in descending order (ties by index)
    for (int i = tid; i < l; i += nt) {
        const double v = at(M, i, i).x;
        int rank = 0;
        for (int j = 0; j < l; ++j) {
            const double w = at(M, j, j).x;
            rank += (w > v) || (w == v && j < i);
        }
        out[rank] = sqrt(fmax(v, 0.0));
    }
    if (tid == 0) *info = s_bad;
}

dim3 grid1(size_t n) {
    size_t g = (n + 255) / 256;
    if (g > 65536) g = 65536;
    if (g == 0) g = 1;
    return dim3((unsigned)g);
}

}  // namespace

hipError_t dense_gemm(int prec, int M, int N, int K, double2 alpha, const void* A, long lda, long sA, const void* B,
                      long ldb, long sB, double2 beta, void* C, long ldc, long sC, int batch, hipStream_t s) {
    if (M <= 0 || N <= 0 || batch <= 0) return hipSuccess;
    const int tiles = ((M + kTile - 1) / kTile) * ((N + kTile - 1) / kTile);
    const dim3 grid(tiles, 1, batch);
    if (K <= 0) {
        // C = beta C: run the kernel with a zero-length reduction
        K = 0;
    }
    if (prec == 0)
        hipLaunchKernelGGL((zgemm_kernel<double, false>), grid, dim3(256), 0, s, M, N, K, alpha, (const double2*)A, lda,
                           sA, (const double2*)B, ldb, sB, beta, (double2*)C, ldc, sC);
    else
        hipLaunchKernelGGL((zgemm_kernel<float, false>), grid, dim3(256), 0, s, M, N, K, alpha, (const float2*)A, lda,
                           sA, (const float2*)B, ldb, sB, beta, (float2*)C, ldc, sC);
    return hipGetLastError();
}

hipError_t dense_gemm_ah(int M, int N, int K, double2 alpha, const double2* A, long lda, const double2* B, long ldb,
                         double2 beta, double2* C, long ldc, hipStream_t s) {
    if (M <= 0 || N <= 0) return hipSuccess;
    const int tiles = ((M + kTile - 1) / kTile) * ((N + kTile - 1) / kTile);
    hipLaunchKernelGGL((zgemm_kernel<double, true>), dim3(tiles, 1, 1), dim3(256), 0, s, M, N, K, alpha, A, lda, 0L,
                       B, ldb, 0L, beta, C, ldc, 0L);
    return hipGetLastError();
}

hipError_t dense_getrf(double2* A, long lda, int n, int* ipiv, int* info, hipStream_t s) {
    constexpr int NB = 32;
    for (int k = 0; k < n; k += NB) {
        const int nb = n - k < NB ? n - k : NB;
        hipLaunchKernelGGL(getf2_panel_kernel, dim3(1), dim3(1024), 0, s, A, lda, n, k, nb, ipiv, info);
        if (k > 0)
            hipLaunchKernelGGL(laswp_kernel<double2>, grid1(k), dim3(256), 0, s, A, lda, 0, k, k, k + nb, ipiv);
        const int rest = n - k - nb;
        if (rest > 0) {
            hipLaunchKernelGGL(laswp_kernel<double2>, grid1(rest), dim3(256), 0, s, A, lda, k + nb, n, k, k + nb, ipiv);
            hipLaunchKernelGGL((trsm_block_kernel<NB, false>), grid1(rest), dim3(256), 0, s, A, lda, k, nb,
                               A + (size_t)(k + nb) * lda, lda, rest);
            const hipError_t e = dense_gemm(0, rest, rest, nb, make_double2(-1.0, 0.0),
                                            A + (size_t)k * lda + k + nb, lda, 0, A + (size_t)(k + nb) * lda + k, lda,
                                            0, make_double2(1.0, 0.0), A + (size_t)(k + nb) * lda + k + nb, lda, 0, 1,
                                            s);
            if (e != hipSuccess) return e;
        }
    }
    return hipGetLastError();
}

hipError_t dense_getrs(const double2* A, long lda, int n, const int* ipiv, double2* B, long ldb, int ncols,
                       hipStream_t s) {
    constexpr int NB = 32;
    if (ncols <= 0) return hipSuccess;
    hipLaunchKernelGGL(laswp_kernel<double2>, grid1(ncols), dim3(256), 0, s, B, ldb, 0, ncols, 0, n, ipiv);
    for (int k = 0; k < n; k += NB) {
        const int nb = n - k < NB ? n - k : NB;
        hipLaunchKernelGGL((trsm_block_kernel<NB, false>), grid1(ncols), dim3(256), 0, s, A, lda, k, nb, B, ldb, ncols);
        const int rest = n - k - nb;
        if (rest > 0) {
            const hipError_t e = dense_gemm(0, rest, ncols, nb, make_double2(-1.0, 0.0), A + (size_t)k * lda + k + nb,
                                            lda, 0, B + k, ldb, 0, make_double2(1.0, 0.0), B + k + nb, ldb, 0, 1, s);
            if (e != hipSuccess) return e;
        }
    }
    const int last = ((n - 1) / NB) * NB;
    for (int k = last; k >= 0; k -= NB) {
        const int nb = n - k < NB ? n - k : NB;
        hipLaunchKernelGGL((trsm_block_kernel<NB, true>), grid1(ncols), dim3(256), 0, s, A, lda, k, nb, B, ldb, ncols);
        if (k > 0) {
            const hipError_t e = dense_gemm(0, k, ncols, nb, make_double2(-1.0, 0.0), A + (size_t)k * lda, lda, 0,
                                            B + k, ldb, 0, make_double2(1.0, 0.0), B, ldb, 0, 1, s);
            if (e != hipSuccess) return e;
        }
    }
    return hipGetLastError();
}

hipError_t dense_norm1(const double2* A, long lda, int m, int n, double* work, double* out, hipStream_t s) {
    hipLaunchKernelGGL(colabs_kernel, dim3(n), dim3(256), 0, s, A, lda, m, n, work);
    hipLaunchKernelGGL(max_kernel, dim3(1), dim3(256), 0, s, work, n, out);
    return hipGetLastError();
}

hipError_t dense_identity(int prec, void* A, long lda, int m, int n, hipStream_t s) {
    if (prec == 0)
        hipLaunchKernelGGL(identity_kernel<double2>, grid1((size_t)m * n), dim3(256), 0, s, (double2*)A, lda, m, n);
    else
        hipLaunchKernelGGL(identity_kernel<float2>, grid1((size_t)m * n), dim3(256), 0, s, (float2*)A, lda, m, n);
    return hipGetLastError();
}

hipError_t dense_axpby2d(int prec, int m, int n, double2 alpha, const void* X, long ldx, double2 beta, const void* Y,
                         long ldy, void* out, long ldo, hipStream_t s) {
    if (m <= 0 || n <= 0) return hipSuccess;
    if (prec == 0)
        hipLaunchKernelGGL(axpby2d_kernel<double2>, grid1((size_t)m * n), dim3(256), 0, s, m, n, alpha,
                           (const double2*)X, ldx, beta, (const double2*)Y, ldy, (double2*)out, ldo);
    else
        hipLaunchKernelGGL(axpby2d_kernel<float2>, grid1((size_t)m * n), dim3(256), 0, s, m, n, alpha,
                           (const float2*)X, ldx, beta, (const float2*)Y, ldy, (float2*)out, ldo);
    return hipGetLastError();
}

hipError_t dense_transpose(const double2* A, long lda, int m, int n, double2* out, long ldo, hipStream_t s) {
    if (m <= 0 || n <= 0) return hipSuccess;
    hipLaunchKernelGGL(transpose_kernel<double2>, grid1((size_t)m * n), dim3(256), 0, s, A, lda, m, n, out, ldo);
    return hipGetLastError();
}

hipError_t dense_conj(const double2* x, double2* out, size_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(conj_kernel, grid1(n), dim3(256), 0, s, x, out, n);
    return hipGetLastError();
}

hipError_t dense_herm_sqrt_eig(double2* G, double2* M, double2* X, int l, int sweeps, double* out, int* info,
                               hipStream_t s) {
    hipLaunchKernelGGL(herm_sqrt_eig_kernel, dim3(1), dim3(1024), 0, s, G, M, X, l, sweeps, out, info);
    return hipGetLastError();
}

hipError_t dense_level1(const double2* R, int Nx, int Ny, int b, int p0, int np, double2* T, hipStream_t s) {
    const size_t n = (size_t)Nx * b;
    hipLaunchKernelGGL(level1_kernel, grid1(n * n * np), dim3(256), 0, s, R, Nx, Ny, b, p0, np, T);
    return hipGetLastError();
}

}  // namespace mlfft
