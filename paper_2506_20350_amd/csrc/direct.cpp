// Host side of the dense paths: the row preconditioner P'_Z (Sec. III-B), the
// direct block Rybicki solver on level 2 (Sec. III-D) and the dense GEMM / LU
// entry points.  Kernels are in dense.hip.
#include <algorithm>
#include <cmath>
#include <vector>

#include "dense.h"
#include "lib.h"

using namespace mlfft;

#define HIPCHK(call, what)                                   \
    do {                                                     \
        hipError_t e_ = (call);                              \
        if (e_ != hipSuccess) return c->hip_fail(e_, what);  \
    } while (0)
#define STCHK(call)                                          \
    do {                                                     \
        mlfft_status s_ = (call);                            \
        if (s_ < 0) return s_;                               \
    } while (0)

namespace {

const double2 kOne = {1.0, 0.0}, kZero = {0.0, 0.0}, kMinus = {-1.0, 0.0};

// Explicit inverse of the n x n matrix A (destroyed: it holds the LU afterwards) into
// Ainv, with its 1-norm reciprocal condition number 1 / (||A||_1 ||A^{-1}||_1).
// ws: n + 2 doubles and n + 1 ints of device scratch.
mlfft_status invert(Ctx* c, double2* A, double2* Ainv, int n, double* dws, int* iws, double* rcond, int* info) {
    hipStream_t s = c->stream;
    HIPCHK(dense_norm1(A, n, n, n, dws, dws + n, s), "norm");
    HIPCHK(hipMemsetAsync(iws + n, 0, sizeof(int), s), "lu info");
    HIPCHK(dense_getrf(A, n, n, iws, iws + n, s), "lu");
    HIPCHK(dense_identity(0, Ainv, n, n, n, s), "identity");
    HIPCHK(dense_getrs(A, n, n, iws, Ainv, n, n, s), "inverse");
    HIPCHK(dense_norm1(Ainv, n, n, n, dws, dws + n + 1, s), "norm");
    double h[2];
    int hi = 0;
    HIPCHK(hipMemcpyAsync(h, dws + n, 2 * sizeof(double), hipMemcpyDeviceToHost, s), "norm");
    HIPCHK(hipMemcpyAsync(&hi, iws + n, sizeof(int), hipMemcpyDeviceToHost, s), "lu info");
    HIPCHK(hipStreamSynchronize(s), "inverse");
    *info = hi;
    *rcond = (hi == 0 && h[0] > 0.0 && std::isfinite(h[1]) && h[1] > 0.0) ? 1.0 / (h[0] * h[1]) : 0.0;
    return MLFFT_OK;
}

}  // namespace

mlfft_status Ctx::row_precond_setup(Array& a) {
    Ctx* c = this;
    if (a.Z64.p && a.Z32.p) return MLFFT_OK;
    if (capturing) return fail(MLFFT_E_STATE, "row preconditioner not built before graph capture");
    const int n = a.Nx * a.b;
    const size_t nn = (size_t)n * n;
    Buf T(&alloc), dws(&alloc), iws(&alloc);
    HIPCHK(T.ensure(nn * sizeof(double2)), "row preconditioner");
    HIPCHK(dws.ensure((n + 2) * sizeof(double)), "row preconditioner");
    HIPCHK(iws.ensure((n + 1) * sizeof(int)), "row preconditioner");
    HIPCHK(a.Z64.ensure(nn * sizeof(double2)), "row preconditioner");
    HIPCHK(a.Z32.ensure(nn * sizeof(float2)), "row preconditioner");
    HIPCHK(dense_level1((const double2*)a.R64.p, a.Nx, a.Ny, a.b, 0, 1, (double2*)T.p, stream), "row block");
    double rc = 0.0;
    int info = 0;
    STCHK(invert(c, (double2*)T.p, (double2*)a.Z64.p, n, (double*)dws.p, (int*)iws.p, &rc, &info));
    if (info != 0 || !(rc >= 1e-14)) {
        a.Z64.release();
        a.Z32.release();
        return fail(MLFFT_E_SINGULAR, "row self block T^[1]_0 is singular (rcond %.3e)", rc);
    }
    HIPCHK(launch_cast_c64_to_c32((const double2*)a.Z64.p, (float2*)a.Z32.p, nn, stream), "cast");
    HIPCHK(hipStreamSynchronize(stream), "row preconditioner");
    a.row_rcond = rc;
    return MLFFT_OK;
}

// Block Rybicki on level 2 (Sec. III-D): the recursion runs over the Ny rows of the
// array, its blocks are the dense level-1 matrices R_p = T^[1]_p of order n = Nx b,
// and every right-hand side of the batch is carried along (x_j is row block j of
// all W columns, an n x W matrix with leading dimension N = Ny n).  Order M -> M+1:
//   D = sum_{j=1..M} R_{M+1-j} G_{M+1-j} - R_0,  x_{M+1} = D^{-1}(sum_j R_{M+1-j} x_j - y_{M+1})   (xmpo)
//   x_j <- x_j - G_{M+1-j} x_{M+1}                                                             (xi)
//   E = sum_j R_{j-(M+1)} H_{M+1-j} - R_0,  G_{M+1} = E^{-1}(sum_j R_{j-(M+1)} G_j - R_{-(M+1)}) (GM1)
//   H_{M+1} = D^{-1}(sum_j R_{M+1-j} H_j - R_{M+1})                                           (HM1)
//   G_j <- G_j - H_{M+1-j} G_{M+1},  H_j <- H_j - G_{M+1-j} H_{M+1}, both from the order-M values (GH, HM)
// The updates of G_j and H_{M+1-j} read only each other's order-M values, so they are
// done pairwise in place with one copy.  Every inverse is formed explicitly (LU with
// partial pivoting) and its 1-norm condition checked: a leading block section with
// rcond < 1e-14 stops the recursion (MLFFT_E_SINGULAR).
static mlfft_status rybicki(Ctx* c, Array& a, int W, const double2* V, long ldv, double2* I, long ldi,
                            double* min_rcond, double* flops) {
    hipStream_t s = c->stream;
    const int Ny = a.Ny, n = a.Nx * a.b;
    const size_t nn = (size_t)n * n;
    double fl = 0.0, rmin = 1.0;
    auto gemm = [&](int M, int Nc, int K, double2 al, const double2* A, long lda, const double2* B, long ldb, double2 be,
                    double2* Cm, long ldc) -> mlfft_status {
        HIPCHK(dense_gemm(0, M, Nc, K, al, A, lda, 0, B, ldb, 0, be, Cm, ldc, 0, 1, s), "block product");
        fl += 8.0 * M * (double)Nc * K;
        return MLFFT_OK;
    };
    const int nlag = 2 * Ny - 1;
    Buf Tb(&c->alloc), Gb(&c->alloc), Hb(&c->alloc), Wk(&c->alloc), Rt(&c->alloc), dws(&c->alloc), iws(&c->alloc);
    HIPCHK(Tb.ensure((size_t)nlag * nn * sizeof(double2)), "level-1 blocks");
    const int ng = std::max(Ny - 1, 1);
    HIPCHK(Gb.ensure((size_t)ng * nn * sizeof(double2)), "recursion blocks");
    HIPCHK(Hb.ensure((size_t)ng * nn * sizeof(double2)), "recursion blocks");
    HIPCHK(Wk.ensure(5 * nn * sizeof(double2)), "recursion workspace");
    HIPCHK(Rt.ensure((size_t)n * W * sizeof(double2)), "recursion workspace");
    HIPCHK(dws.ensure((n + 2) * sizeof(double)), "recursion workspace");
    HIPCHK(iws.ensure((n + 1) * sizeof(int)), "recursion workspace");
    double2* T = (double2*)Tb.p;
    auto R = [&](int p) { return T + (size_t)(p + Ny - 1) * nn; };          // R_p, |p| < Ny
    auto G = [&](int j) { return (double2*)Gb.p + (size_t)(j - 1) * nn; };  // G_j, j = 1 .. Ny-1
    auto H = [&](int j) { return (double2*)Hb.p + (size_t)(j - 1) * nn; };
    double2* LU = (double2*)Wk.p;
    double2* Dinv = LU + nn;
    double2* Einv = Dinv + nn;
    double2* S = Einv + nn;
    double2* Tmp = S + nn;
    auto xb = [&](int j) { return I + (size_t)j * n; };                      // x_{j+1}: row block j, ld N
    auto yb = [&](int j) { return V + (size_t)j * n; };
    HIPCHK(dense_level1((const double2*)a.R64.p, a.Nx, Ny, a.b, -(Ny - 1), nlag, T, s), "level-1 blocks");
    auto inv = [&](const double2* A, double2* Ainv, const char* what, int order) -> mlfft_status {
        HIPCHK(hipMemcpyAsync(LU, A, nn * sizeof(double2), hipMemcpyDeviceToDevice, s), "copy");
        double rc = 0.0;
        int info = 0;
        STCHK(invert(c, LU, Ainv, n, (double*)dws.p, (int*)iws.p, &rc, &info));
        fl += 8.0 * n * (double)n * n * (1.0 / 3.0 + 1.0);      // LU, then the solve against the identity
        rmin = std::min(rmin, rc);
        if (info != 0 || !(rc >= 1e-14))
            return c->fail(MLFFT_E_SINGULAR, "%s at order %d is singular (rcond %.3e)", what, order, rc);
        return MLFFT_OK;
    };
    // order 1: x_1 = R_0^{-1} y_1, G_1 = R_0^{-1} R_{-1}, H_1 = R_0^{-1} R_1
    STCHK(inv(R(0), Dinv, "R_0", 0));
    STCHK(gemm(n, W, n, kOne, Dinv, n, yb(0), ldv, kZero, xb(0), ldi));
    if (Ny > 1) {
        STCHK(gemm(n, n, n, kOne, Dinv, n, R(-1), n, kZero, G(1), n));
        STCHK(gemm(n, n, n, kOne, Dinv, n, R(1), n, kZero, H(1), n));
    }
    for (int M = 1; M < Ny; ++M) {
        // eq. xmpo
        HIPCHK(dense_axpby2d(0, n, n, kMinus, R(0), n, kZero, nullptr, 0, S, n, s), "copy");
        for (int j = 1; j <= M; ++j) STCHK(gemm(n, n, n, kOne, R(M + 1 - j), n, G(M + 1 - j), n, kOne, S, n));
        STCHK(inv(S, Dinv, "D", M));
        HIPCHK(dense_axpby2d(0, n, W, kMinus, yb(M), ldv, kZero, nullptr, 0, Rt.p, n, s), "copy");
        for (int j = 1; j <= M; ++j)
            STCHK(gemm(n, W, n, kOne, R(M + 1 - j), n, xb(j - 1), ldi, kOne, (double2*)Rt.p, n));
        STCHK(gemm(n, W, n, kOne, Dinv, n, (double2*)Rt.p, n, kZero, xb(M), ldi));
        // eq. xi
        for (int j = 1; j <= M; ++j) STCHK(gemm(n, W, n, kMinus, G(M + 1 - j), n, xb(M), ldi, kOne, xb(j - 1), ldi));
        if (M + 1 == Ny) break;
        // eq. GM1
        HIPCHK(dense_axpby2d(0, n, n, kMinus, R(0), n, kZero, nullptr, 0, S, n, s), "copy");
        for (int j = 1; j <= M; ++j) STCHK(gemm(n, n, n, kOne, R(j - (M + 1)), n, H(M + 1 - j), n, kOne, S, n));
        STCHK(inv(S, Einv, "E", M));
        HIPCHK(dense_axpby2d(0, n, n, kMinus, R(-(M + 1)), n, kZero, nullptr, 0, S, n, s), "copy");
        for (int j = 1; j <= M; ++j) STCHK(gemm(n, n, n, kOne, R(j - (M + 1)), n, G(j), n, kOne, S, n));
        STCHK(gemm(n, n, n, kOne, Einv, n, S, n, kZero, G(M + 1), n));
        // eq. HM1
        HIPCHK(dense_axpby2d(0, n, n, kMinus, R(M + 1), n, kZero, nullptr, 0, S, n, s), "copy");
        for (int j = 1; j <= M; ++j) STCHK(gemm(n, n, n, kOne, R(M + 1 - j), n, H(j), n, kOne, S, n));
        STCHK(gemm(n, n, n, kOne, Dinv, n, S, n, kZero, H(M + 1), n));
        // eqs. GH and HM: G_j and H_{M+1-j} from each other's order-M values
        for (int j = 1; j <= M; ++j) {
            HIPCHK(hipMemcpyAsync(Tmp, G(j), nn * sizeof(double2), hipMemcpyDeviceToDevice, s), "copy");
            STCHK(gemm(n, n, n, kMinus, H(M + 1 - j), n, G(M + 1), n, kOne, G(j), n));
            STCHK(gemm(n, n, n, kMinus, Tmp, n, H(M + 1), n, kOne, H(M + 1 - j), n));
        }
    }
    HIPCHK(hipStreamSynchronize(s), "direct solve");
    if (min_rcond) *min_rcond = rmin;
    if (flops) *flops = fl;
    return MLFFT_OK;
}

// Z I = V with the border moved to the right-hand side (Sec. III-E): Z_A [U F] = [V_A Z_B^T]
// by the block Rybicki recursion (W + Nc right-hand sides), then the Schur complement
// S = Z_C - Z_B F, I_C = S^{-1}(V_C - Z_B U) and I_A = U - F I_C.
static mlfft_status schur_direct(Ctx* c, Array& a, int W, const double2* V, double2* I, double* min_rcond,
                                 double* flops) {
    hipStream_t s = c->stream;
    const long N = (long)a.NA(), Nt = (long)a.Nt();
    const int Nc = a.Nc;
    const int Wr = W + Nc;
    Buf Rb(&c->alloc), Xb(&c->alloc), Sb(&c->alloc), Si(&c->alloc), Rc(&c->alloc), dws(&c->alloc), iws(&c->alloc);
    HIPCHK(Rb.ensure((size_t)N * Wr * sizeof(double2)), "border right-hand sides");
    HIPCHK(Xb.ensure((size_t)N * Wr * sizeof(double2)), "border right-hand sides");
    HIPCHK(Sb.ensure((size_t)Nc * Nc * sizeof(double2)), "Schur complement");
    HIPCHK(Si.ensure((size_t)Nc * Nc * sizeof(double2)), "Schur complement");
    HIPCHK(Rc.ensure((size_t)Nc * W * sizeof(double2)), "Schur complement");
    HIPCHK(dws.ensure((Nc + 2) * sizeof(double)), "Schur complement");
    HIPCHK(iws.ensure((Nc + 1) * sizeof(int)), "Schur complement");
    double2* R = (double2*)Rb.p;
    double2* X = (double2*)Xb.p;
    HIPCHK(dense_axpby2d(0, (int)N, W, kOne, V, Nt, kZero, nullptr, 0, R, N, s), "gather V_A");
    HIPCHK(hipMemcpyAsync(R + (size_t)N * W, a.Bt64.p, (size_t)N * Nc * sizeof(double2), hipMemcpyDeviceToDevice, s),
           "gather Z_B^T");
    double rc = 1.0, fl = 0.0;
    STCHK(rybicki(c, a, Wr, R, N, X, N, &rc, &fl));
    const double2* U = X;
    const double2* F = X + (size_t)N * W;
    double2* S = (double2*)Sb.p;
    HIPCHK(hipMemcpyAsync(S, a.C64.p, (size_t)Nc * Nc * sizeof(double2), hipMemcpyDeviceToDevice, s), "Schur");
    HIPCHK(dense_gemm(0, Nc, Nc, (int)N, kMinus, a.B64.p, Nc, 0, F, N, 0, kOne, S, Nc, 0, 1, s), "Schur");
    HIPCHK(dense_axpby2d(0, Nc, W, kOne, V + N, Nt, kZero, nullptr, 0, Rc.p, Nc, s), "gather V_C");
    HIPCHK(dense_gemm(0, Nc, W, (int)N, kMinus, a.B64.p, Nc, 0, U, N, 0, kOne, Rc.p, Nc, 0, 1, s), "Schur");
    double src = 0.0;
    int info = 0;
    STCHK(invert(c, S, (double2*)Si.p, Nc, (double*)dws.p, (int*)iws.p, &src, &info));
    if (info != 0 || !(src >= 1e-14))
        return c->fail(MLFFT_E_SINGULAR, "Schur complement Z_C - Z_B Z_A^{-1} Z_B^T is singular (rcond %.3e)", src);
    HIPCHK(dense_gemm(0, Nc, W, Nc, kOne, Si.p, Nc, 0, Rc.p, Nc, 0, kZero, I + N, Nt, 0, 1, s), "I_C");
    HIPCHK(dense_axpby2d(0, (int)N, W, kOne, U, N, kZero, nullptr, 0, I, Nt, s), "I_A");
    HIPCHK(dense_gemm(0, (int)N, W, Nc, kMinus, F, N, 0, I + N, Nt, 0, kOne, I, Nt, 0, 1, s), "I_A");
    HIPCHK(hipStreamSynchronize(s), "direct solve");
    fl += 8.0 * ((double)Nc * Nc * N + (double)Nc * W * N + (double)Nc * W * Nc + (double)N * W * Nc) +
          8.0 * (double)Nc * Nc * Nc * (1.0 / 3.0 + 1.0);
    if (min_rcond) *min_rcond = std::min(rc, src);
    if (flops) *flops = fl;
    return MLFFT_OK;
}

mlfft_status Ctx::border_matvec(const std::vector<MatvecItem>& items, int prec) {
    Ctx* c = this;
    const int p = prec == P64 ? 0 : 1;
    const int eb = prec_elem_bytes(prec);
    for (const MatvecItem& it : items) {
        const Array* a = it.arr;
        if (a->Nc == 0) continue;
        const long N = (long)a->NA(), ld = (long)a->Nt();
        const int Nc = a->Nc, W = it.W;
        const char* xa = (const char*)it.x;
        const char* xc = xa + N * eb;
        char* ya = (char*)it.y;
        char* yc = ya + N * eb;
        const double2 al = make_double2(it.alpha, 0.0);
        const int pr = prof_begin(PK_BORDER, prec, (double)eb * W * (2.0 * Nc + 3.0 * N) +
                                  (p ? 8.0 : 16.0) * ((double)2 * N * Nc + (double)Nc * Nc),
                                  8.0 * W * ((double)2 * N * Nc + (double)Nc * Nc));
        // y_A += alpha Z_B^T x_C
        HIPCHK(dense_gemm(p, (int)N, W, Nc, al, p ? a->Bt32.p : a->Bt64.p, N, 0, xc, ld, 0, kOne, ya, ld, 0, 1, stream),
               "border product");
        // y_C = alpha (Z_B x_A + Z_C x_C) + beta v_C
        double2 be = kZero;
        if (it.addend) {
            HIPCHK(dense_axpby2d(p, Nc, W, make_double2(it.beta, 0.0), (const char*)it.addend + N * eb, ld, kZero,
                                 nullptr, 0, yc, ld, stream), "border addend");
            be = kOne;
        }
        HIPCHK(dense_gemm(p, Nc, W, (int)N, al, p ? a->B32.p : a->B64.p, Nc, 0, xa, ld, 0, be, yc, ld, 0, 1, stream),
               "border product");
        HIPCHK(dense_gemm(p, Nc, W, Nc, al, p ? a->C32.p : a->C64.p, Nc, 0, xc, ld, 0, kOne, yc, ld, 0, 1, stream),
               "border product");
        prof_end(pr);
    }
    return MLFFT_OK;
}

mlfft_status Ctx::border_precond(const std::vector<MatvecItem>& items, int prec) {
    Ctx* c = this;
    const int p = prec == P64 ? 0 : 1;
    const int eb = prec_elem_bytes(prec);
    for (const MatvecItem& it : items) {
        const Array* a = it.arr;
        if (a->Nc == 0) continue;
        const long N = (long)a->NA(), ld = (long)a->Nt();
        const int Nc = a->Nc, W = it.W;
        char* zc = (char*)it.y + N * eb;
        double2 be = kZero;
        if (it.addend) {
            HIPCHK(dense_axpby2d(p, Nc, W, make_double2(it.beta, 0.0), (const char*)it.addend + N * eb, ld, kZero,
                                 nullptr, 0, zc, ld, stream), "border addend");
            be = kOne;
        }
        HIPCHK(dense_gemm(p, Nc, W, Nc, make_double2(it.alpha, 0.0), p ? a->Ci32.p : a->Ci64.p, Nc, 0,
                          (const char*)it.x + N * eb, ld, 0, be, zc, ld, 0, 1, stream), "border preconditioner");
    }
    return MLFFT_OK;
}

extern "C" {

mlfft_status mlfft_direct_solve(mlfft_ctx ctx, int array_id, int W, const void* V, void* I, double* min_rcond,
                                double* flops) {
    if (!ctx) return MLFFT_E_ARG;
    Ctx* c = ctx;
    Array* a = c->find(array_id);
    if (!a) return c->fail(MLFFT_E_STATE, "unknown array id %d", array_id);
    if (W < 0) return c->fail(MLFFT_E_ARG, "W must be >= 0");
    if (W == 0) return MLFFT_OK;
    if (!V || !I) return c->fail(MLFFT_E_ARG, "V or I is NULL");
    const size_t vb = (size_t)a->Nx * a->Ny * a->b * W * 16;
    if ((const char*)V < (const char*)I + vb && (const char*)I < (const char*)V + vb)
        return c->fail(MLFFT_E_ARG, "V and I overlap");
    HIPCHK(hipSetDevice(c->device), "set device");
    if (a->Nc > 0) return schur_direct(c, *a, W, (const double2*)V, (double2*)I, min_rcond, flops);
    const long N = (long)a->NA();
    return rybicki(c, *a, W, (const double2*)V, N, (double2*)I, N, min_rcond, flops);
}

mlfft_status mlfft_set_border(mlfft_ctx ctx, int array_id, int Nc, const void* ZB, const void* ZC, int on_device) {
    if (!ctx) return MLFFT_E_ARG;
    Ctx* c = ctx;
    Array* a = c->find(array_id);
    if (!a) return c->fail(MLFFT_E_STATE, "unknown array id %d", array_id);
    if (Nc < 0 || Nc > 65536) return c->fail(MLFFT_E_ARG, "Nc must be in [0, 65536]");
    HIPCHK(hipSetDevice(c->device), "set device");
    HIPCHK(hipStreamSynchronize(c->stream), "set border");
    for (Buf* x : {&a->B64, &a->B32, &a->Bt64, &a->Bt32, &a->C64, &a->C32, &a->Ci64, &a->Ci32, &a->Kc64, &a->Kc32})
        x->release();
    a->Nc = 0;
    if (Nc == 0) return MLFFT_OK;
    if (!ZB || !ZC) return c->fail(MLFFT_E_ARG, "ZB or ZC is NULL");
    const long N = (long)a->NA();
    const size_t nb = (size_t)N * Nc, nc = (size_t)Nc * Nc, bb = (size_t)a->b * a->b;
    if (!on_device) {
        const double* h = (const double*)ZB;
        for (size_t i = 0; i < 2 * nb; ++i)
            if (!std::isfinite(h[i])) return c->fail(MLFFT_E_ARG, "ZB contains a non-finite value");
        h = (const double*)ZC;
        for (size_t i = 0; i < 2 * nc; ++i)
            if (!std::isfinite(h[i])) return c->fail(MLFFT_E_ARG, "ZC contains a non-finite value");
    }
    hipStream_t s = c->stream;
    const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    Buf Ct(&c->alloc), dws(&c->alloc), iws(&c->alloc);
    HIPCHK(a->Bt64.ensure(nb * sizeof(double2)), "border");
    HIPCHK(a->B64.ensure(nb * sizeof(double2)), "border");
    HIPCHK(a->C64.ensure(nc * sizeof(double2)), "border");
    HIPCHK(a->Ci64.ensure(nc * sizeof(double2)), "border");
    HIPCHK(a->Kc64.ensure(bb * sizeof(double2)), "border");
    for (Buf* x : {&a->Bt32, &a->B32}) HIPCHK(x->ensure(nb * sizeof(float2)), "border");
    for (Buf* x : {&a->C32, &a->Ci32}) HIPCHK(x->ensure(nc * sizeof(float2)), "border");
    HIPCHK(a->Kc32.ensure(bb * sizeof(float2)), "border");
    HIPCHK(Ct.ensure(nc * sizeof(double2)), "border");
    HIPCHK(dws.ensure((Nc + 2) * sizeof(double)), "border");
    HIPCHK(iws.ensure((Nc + 1) * sizeof(int)), "border");
    // row-major Z_B (Nc x N) is the column-major N x Nc matrix Z_B^T; row-major Z_C is Z_C^T column-major
    HIPCHK(hipMemcpyAsync(a->Bt64.p, ZB, nb * sizeof(double2), kind, s), "border upload");
    HIPCHK(hipMemcpyAsync(Ct.p, ZC, nc * sizeof(double2), kind, s), "border upload");
    HIPCHK(dense_transpose((const double2*)a->Bt64.p, N, (int)N, Nc, (double2*)a->B64.p, Nc, s), "border");
    HIPCHK(dense_transpose((const double2*)Ct.p, Nc, Nc, Nc, (double2*)a->C64.p, Nc, s), "border");
    HIPCHK(dense_transpose((const double2*)a->K64.p, a->b, a->b, a->b, (double2*)a->Kc64.p, a->b, s), "border");
    if (on_device) {
        Buf flag(&c->alloc);
        HIPCHK(flag.ensure(sizeof(int)), "flag");
        HIPCHK(hipMemsetAsync(flag.p, 0, sizeof(int), s), "flag");
        HIPCHK(launch_nonfinite((const double*)a->Bt64.p, 2 * nb, (int*)flag.p, s), "finite check");
        HIPCHK(launch_nonfinite((const double*)a->C64.p, 2 * nc, (int*)flag.p, s), "finite check");
        int hflag = 0;
        HIPCHK(hipMemcpyAsync(&hflag, flag.p, sizeof(int), hipMemcpyDeviceToHost, s), "flag");
        HIPCHK(hipStreamSynchronize(s), "finite check");
        if (hflag) {
            for (Buf* x : {&a->B64, &a->B32, &a->Bt64, &a->Bt32, &a->C64, &a->C32, &a->Ci64, &a->Ci32, &a->Kc64, &a->Kc32})
                x->release();
            return c->fail(MLFFT_E_ARG, "ZB or ZC contains a non-finite value");
        }
    }
    // Z_C^{-1} for the border part of P_X (Sec. III-B: the LU of Z_C)
    HIPCHK(hipMemcpyAsync(Ct.p, a->C64.p, nc * sizeof(double2), hipMemcpyDeviceToDevice, s), "border");
    double rc = 0.0;
    int info = 0;
    STCHK(invert(c, (double2*)Ct.p, (double2*)a->Ci64.p, Nc, (double*)dws.p, (int*)iws.p, &rc, &info));
    if (info != 0 || !(rc >= 1e-14)) {
        for (Buf* x : {&a->B64, &a->B32, &a->Bt64, &a->Bt32, &a->C64, &a->C32, &a->Ci64, &a->Ci32, &a->Kc64, &a->Kc32})
            x->release();
        return c->fail(MLFFT_E_SINGULAR, "border self block Z_C is singular (rcond %.3e)", rc);
    }
    HIPCHK(launch_cast_c64_to_c32((const double2*)a->Bt64.p, (float2*)a->Bt32.p, nb, s), "cast");
    HIPCHK(launch_cast_c64_to_c32((const double2*)a->B64.p, (float2*)a->B32.p, nb, s), "cast");
    HIPCHK(launch_cast_c64_to_c32((const double2*)a->C64.p, (float2*)a->C32.p, nc, s), "cast");
    HIPCHK(launch_cast_c64_to_c32((const double2*)a->Ci64.p, (float2*)a->Ci32.p, nc, s), "cast");
    HIPCHK(launch_cast_c64_to_c32((const double2*)a->Kc64.p, (float2*)a->Kc32.p, bb, s), "cast");
    HIPCHK(hipStreamSynchronize(s), "set border");
    a->Nc = Nc;
    return MLFFT_OK;
}

mlfft_status mlfft_dense_gemm(mlfft_ctx ctx, int prec, int M, int N, int K, double alpha_re, double alpha_im,
                              const void* A, long lda, const void* B, long ldb, double beta_re, double beta_im, void* C,
                              long ldc) {
    if (!ctx) return MLFFT_E_ARG;
    Ctx* c = ctx;
    if (prec != MLFFT_FP64 && prec != MLFFT_FP32) return c->fail(MLFFT_E_ARG, "prec must be MLFFT_FP64 or MLFFT_FP32");
    if (M < 0 || N < 0 || K < 0) return c->fail(MLFFT_E_ARG, "negative dimension");
    if (M == 0 || N == 0) return MLFFT_OK;
    if (!C || (K > 0 && (!A || !B))) return c->fail(MLFFT_E_ARG, "NULL matrix");
    if (lda < std::max(M, 1) || ldb < std::max(K, 1) || ldc < M) return c->fail(MLFFT_E_ARG, "leading dimension too small");
    HIPCHK(hipSetDevice(c->device), "set device");
    HIPCHK(dense_gemm(prec, M, N, K, make_double2(alpha_re, alpha_im), A, lda, 0, B, ldb, 0,
                      make_double2(beta_re, beta_im), C, ldc, 0, 1, c->stream), "dense product");
    return MLFFT_OK;
}

mlfft_status mlfft_dense_gemm_ah(mlfft_ctx ctx, int M, int N, int K, double alpha_re, double alpha_im, const void* A,
                                 long lda, const void* B, long ldb, double beta_re, double beta_im, void* C, long ldc) {
    if (!ctx) return MLFFT_E_ARG;
    Ctx* c = ctx;
    if (M < 0 || N < 0 || K < 0) return c->fail(MLFFT_E_ARG, "negative dimension");
    if (M == 0 || N == 0) return MLFFT_OK;
    if (!C || (K > 0 && (!A || !B))) return c->fail(MLFFT_E_ARG, "NULL matrix");
    if (lda < std::max(K, 1) || ldb < std::max(K, 1) || ldc < M) return c->fail(MLFFT_E_ARG, "leading dimension too small");
    HIPCHK(hipSetDevice(c->device), "set device");
    HIPCHK(dense_gemm_ah(M, N, K, make_double2(alpha_re, alpha_im), (const double2*)A, lda, (const double2*)B, ldb,
                         make_double2(beta_re, beta_im), (double2*)C, ldc, c->stream), "dense product");
    return MLFFT_OK;
}

mlfft_status mlfft_dense_gen_eig(mlfft_ctx ctx, int l, void* G, void* M, double* sigma) {
    if (!ctx) return MLFFT_E_ARG;
    Ctx* c = ctx;
    if (l < 1 || l > 1024) return c->fail(MLFFT_E_ARG, "l must be in [1, 1024]");
    if (!G || !M || !sigma) return c->fail(MLFFT_E_ARG, "NULL argument");
    HIPCHK(hipSetDevice(c->device), "set device");
    Buf Xb(&c->alloc);
    HIPCHK(Xb.ensure((size_t)l * l * sizeof(double2) + l * sizeof(double) + 256), "eigenvalue workspace");
    double* sv = (double*)((double2*)Xb.p + (size_t)l * l);
    int* info = (int*)(sv + l);
    HIPCHK(dense_herm_sqrt_eig((double2*)G, (double2*)M, (double2*)Xb.p, l, 16, sv, info, c->stream), "eigenvalues");
    int hinfo = 0;
    HIPCHK(hipMemcpyAsync(sigma, sv, l * sizeof(double), hipMemcpyDeviceToHost, c->stream), "eigenvalues");
    HIPCHK(hipMemcpyAsync(&hinfo, info, sizeof(int), hipMemcpyDeviceToHost, c->stream), "eigenvalues");
    HIPCHK(hipStreamSynchronize(c->stream), "eigenvalues");
    if (hinfo) return c->fail(MLFFT_E_SINGULAR, "G is not positive definite");
    return MLFFT_OK;
}

mlfft_status mlfft_dense_solve(mlfft_ctx ctx, int n, void* A, long lda, void* B, long ldb, int ncols) {
    if (!ctx) return MLFFT_E_ARG;
    Ctx* c = ctx;
    if (n < 0 || ncols < 0) return c->fail(MLFFT_E_ARG, "negative dimension");
    if (n == 0) return MLFFT_OK;
    if (!A || (ncols > 0 && !B)) return c->fail(MLFFT_E_ARG, "NULL matrix");
    if (lda < n || (ncols > 0 && ldb < n)) return c->fail(MLFFT_E_ARG, "leading dimension too small");
    HIPCHK(hipSetDevice(c->device), "set device");
    Buf iws(&c->alloc);
    HIPCHK(iws.ensure((n + 1) * sizeof(int)), "pivots");
    hipStream_t s = c->stream;
    HIPCHK(hipMemsetAsync((int*)iws.p + n, 0, sizeof(int), s), "lu info");
    HIPCHK(dense_getrf((double2*)A, lda, n, (int*)iws.p, (int*)iws.p + n, s), "lu");
    if (ncols > 0) HIPCHK(dense_getrs((const double2*)A, lda, n, (int*)iws.p, (double2*)B, ldb, ncols, s), "solve");
    int info = 0;
    HIPCHK(hipMemcpyAsync(&info, (int*)iws.p + n, sizeof(int), hipMemcpyDeviceToHost, s), "lu info");
    HIPCHK(hipStreamSynchronize(s), "solve");
    if (info != 0) return c->fail(MLFFT_E_SINGULAR, "exactly zero pivot in column %d", info - 1);
    return MLFFT_OK;
}

}  // extern "C"
