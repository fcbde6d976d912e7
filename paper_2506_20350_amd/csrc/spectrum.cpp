// Singular values of the preconditioned operator A = P^{-1} Z (Sec. V, the spectra of
// P^{-1} Z for P = I, P_K, P_Z) by the randomized range finder of Halko, Martinsson and
// Tropp, with every product through the MLFFT matvec and the preconditioners in FP64.
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

struct Op {
    Ctx* c;
    Array* a;
    int kind;          // preconditioner: 0 none, 1 block circulant, 2 P'_K, 4 P'_Z
    int l;
    size_t n;          // entries of the l columns
    double2* t1;
    double2* t2;

    // y = P^{-1} Z x
    mlfft_status apply(const double2* x, double2* y) {
        std::vector<MatvecItem> it(1);
        if (kind == 0) {
            it[0] = MatvecItem{a, l, x, y, nullptr, 1.0, 0.0};
            return c->matvec_group(it, P64);
        }
        it[0] = MatvecItem{a, l, x, t1, nullptr, 1.0, 0.0};
        STCHK(c->matvec_group(it, P64));
        it[0] = MatvecItem{a, l, t1, y, nullptr, 1.0, 0.0};
        return c->precond_group(it, kind, P64);
    }

    // y = A^H x = Z^H P^{-H} x = conj(Z P^{-1} conj(x)): Z and P are complex symmetric
    // (reciprocal blocks), so their adjoints are their conjugates
    mlfft_status apply_adjoint(const double2* x, double2* y) {
        hipStream_t s = c->stream;
        if (hipError_t e = dense_conj(x, t2, n, s); e != hipSuccess) return c->hip_fail(e, "conjugate");
        std::vector<MatvecItem> it(1);
        const double2* src = t2;
        if (kind != 0) {
            it[0] = MatvecItem{a, l, t2, t1, nullptr, 1.0, 0.0};
            STCHK(c->precond_group(it, kind, P64));
            src = t1;
        }
        it[0] = MatvecItem{a, l, src, y, nullptr, 1.0, 0.0};
        STCHK(c->matvec_group(it, P64));
        if (hipError_t e = dense_conj(y, y, n, s); e != hipSuccess) return c->hip_fail(e, "conjugate");
        return MLFFT_OK;
    }
};

}  // namespace

extern "C" mlfft_status mlfft_spectrum(mlfft_ctx ctx, int array_id, int kind, int l, const void* Omega,
                                       int power_iters, double* sigma) {
    if (!ctx) return MLFFT_E_ARG;
    Ctx* c = ctx;
    Array* a = c->find(array_id);
    if (!a) return c->fail(MLFFT_E_STATE, "unknown array id %d", array_id);
    if (kind != 0 && kind != 1 && kind != 2 && kind != 4)
        return c->fail(MLFFT_E_ARG, "preconditioner kind must be 0, 1, 2 or 4");
    if (l < 1 || l > 1024) return c->fail(MLFFT_E_ARG, "l must be in [1, 1024]");
    if ((size_t)l > a->Nt()) return c->fail(MLFFT_E_ARG, "l must not exceed the number of unknowns");
    if (power_iters < 0 || power_iters > 8) return c->fail(MLFFT_E_ARG, "power_iters must be in [0, 8]");
    if (!Omega || !sigma) return c->fail(MLFFT_E_ARG, "Omega or sigma is NULL");
    HIPCHK(hipSetDevice(c->device), "set device");
    hipStream_t s = c->stream;
    const size_t n = a->Nt() * (size_t)l;
    Buf Yb(&c->alloc), Cb(&c->alloc), T1(&c->alloc), T2(&c->alloc), Sm(&c->alloc);
    for (Buf* x : {&Yb, &Cb, &T1, &T2}) HIPCHK(x->ensure(n * sizeof(double2)), "spectrum workspace");
    const size_t ll = (size_t)l * l;
    HIPCHK(Sm.ensure(3 * ll * sizeof(double2) + l * sizeof(double) + 256), "spectrum workspace");
    Op op{c, a, kind, l, n, (double2*)T1.p, (double2*)T2.p};
    double2* Y = (double2*)Yb.p;
    double2* C = (double2*)Cb.p;
    // 1. Y = A Omega;  2. power steps Y = A (A^H Y)
    STCHK(op.apply((const double2*)Omega, Y));
    for (int q = 0; q < power_iters; ++q) {
        STCHK(op.apply_adjoint(Y, C));
        STCHK(op.apply(C, Y));
    }
    // 3.-5. with Y = Q R (R^H R = G = Y^H Y) and C = A^H Y, B = Q^H A has
    // B B^H = R^{-H} C^H C R^{-1}: its eigenvalues are the squared singular values
    STCHK(op.apply_adjoint(Y, C));
    double2* G = (double2*)Sm.p;
    double2* M = G + ll;
    double2* X = M + ll;
    double* sv = (double*)(X + ll);
    int* info = (int*)(sv + l);
    const long ld = (long)a->Nt();
    const double2 one = make_double2(1.0, 0.0), zero = make_double2(0.0, 0.0);
    HIPCHK(dense_gemm_ah(l, l, (int)a->Nt(), one, Y, ld, Y, ld, zero, G, l, s), "Gram matrix");
    HIPCHK(dense_gemm_ah(l, l, (int)a->Nt(), one, C, ld, C, ld, zero, M, l, s), "Gram matrix");
    HIPCHK(dense_herm_sqrt_eig(G, M, X, l, 16, sv, info, s), "eigenvalues");
    int hinfo = 0;
    HIPCHK(hipMemcpyAsync(sigma, sv, l * sizeof(double), hipMemcpyDeviceToHost, s), "singular values");
    HIPCHK(hipMemcpyAsync(&hinfo, info, sizeof(int), hipMemcpyDeviceToHost, s), "singular values");
    HIPCHK(hipStreamSynchronize(s), "spectrum");
    if (hinfo) return c->fail(MLFFT_E_SINGULAR, "the sketch Y = A Omega is rank deficient (Y^H Y not positive definite)");
    return MLFFT_OK;
}
