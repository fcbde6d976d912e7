// Dense complex linear algebra on the device (kernels in dense.hip).  Matrices
// are column-major with a leading dimension; complex values are double2 (FP64)
// or float2 (FP32).
#pragma once
#include <hip/hip_runtime.h>

#include "common.h"

namespace mlfft {

// C = alpha A B + beta C for `batch` problems (element strides sA, sB, sC between
// them); A is M x K, B is K x N, C is M x N.  prec 0: complex128, 1: complex64
// (FP32 MFMA; alpha, beta applied in FP64 and rounded).  beta = 0 does not read C.
hipError_t dense_gemm(int prec, int M, int N, int K, double2 alpha, const void* A, long lda, long sA, const void* B,
                      long ldb, long sB, double2 beta, void* C, long ldc, long sC, int batch, hipStream_t s);

// C = alpha A^H B + beta C (complex128) with A stored K x M (lda >= K): the Gram products of
// the randomized range finder
hipError_t dense_gemm_ah(int M, int N, int K, double2 alpha, const double2* A, long lda, const double2* B, long ldb,
                         double2 beta, double2* C, long ldc, hipStream_t s);

// out = conj(x) over n complex128 values
hipError_t dense_conj(const double2* x, double2* out, size_t n, hipStream_t s);

// out[0 .. l) = square roots of the eigenvalues of L^{-1} M L^{-H} (descending) for l x l Hermitian
// G = L L^H and M, one workgroup (Cholesky, forward substitutions, `sweeps` round-robin Jacobi
// sweeps); G, M overwritten, X l x l scratch; *info = 1 if G is not positive definite.  l <= 1024.
hipError_t dense_herm_sqrt_eig(double2* G, double2* M, double2* X, int l, int sweeps, double* out, int* info,
                               hipStream_t s);

// LU with partial pivoting of the n x n matrix A in place (L unit lower, U upper,
// ipiv[k] = row interchanged with row k, absolute).  *info (device, cleared by
// the caller) receives the 1-based index of the first exactly zero pivot.
hipError_t dense_getrf(double2* A, long lda, int n, int* ipiv, int* info, hipStream_t s);

// B <- A^{-1} B for ncols columns, with A and ipiv from dense_getrf.
hipError_t dense_getrs(const double2* A, long lda, int n, const int* ipiv, double2* B, long ldb, int ncols,
                       hipStream_t s);

// *out = ||A||_1 (largest column sum of moduli) of the m x n matrix A; work holds n doubles.
hipError_t dense_norm1(const double2* A, long lda, int m, int n, double* work, double* out, hipStream_t s);

// out = alpha X + beta Y over an m x n block (Y may be NULL; out may alias X or Y exactly)
hipError_t dense_axpby2d(int prec, int m, int n, double2 alpha, const void* X, long ldx, double2 beta, const void* Y,
                         long ldy, void* out, long ldo, hipStream_t s);

// out (n x m) = A^T for the m x n matrix A (complex128; no conjugation)
hipError_t dense_transpose(const double2* A, long lda, int m, int n, double2* out, long ldo, hipStream_t s);

// A = the m x n identity (prec 0: complex128, 1: complex64)
hipError_t dense_identity(int prec, void* A, long lda, int m, int n, hipStream_t s);

// T^[1]_p for p = p0 .. p0 + np - 1, each a dense (Nx b) x (Nx b) column-major matrix,
// from the unique blocks R (library layout [p + Ny - 1][q + Nx - 1][m][n]).
hipError_t dense_level1(const double2* R, int Nx, int Ny, int b, int p0, int np, double2* T, hipStream_t s);

}  // namespace mlfft
