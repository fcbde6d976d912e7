/*
 * mlfft.h - C ABI of the MI355X MLFFT solver library.
 *
 * The library solves Z_A I = V for the two-level block-Toeplitz impedance
 * matrix Z_A of an Nx x Ny array of identical cells with b basis functions
 * each (Sec. II-A, eq. Tblock; Sec. III, "ZI = V"), using the multilevel FFT
 * product (Sec. II-C, eq. multL; Sec. III-A) inside restarted GMRES (Sec. III-C).
 *
 * Conventions shared by every entry point:
 *  - Every function returns an mlfft_status.  Negative values are errors and
 *    leave a message retrievable with mlfft_last_error(); MLFFT_NOT_CONVERGED
 *    (positive) means the call completed and its outputs are valid but some
 *    right-hand side missed its tolerance.  No C++ exception crosses the ABI.
 *  - Arguments are validated before any work is enqueued.
 *  - Complex numbers are interleaved (re, im): complex128 = two doubles,
 *    complex64 = two floats.
 *  - Vector layout (the paper's order, eq. xc2 and eq. ZIVvec): W columns,
 *    column w contiguous; inside a column the unknown of basis m of cell
 *    (iy, ix) is at ((iy * Nx) + ix) * b + m.
 *  - Device pointers are HIP device pointers of the context's device.  The
 *    caller owns every pointer it passes; the library never frees them.
 *  - Work is enqueued on the context's stream (the caller's stream, e.g. the
 *    PyTorch current stream).  Calls documented as asynchronous return before
 *    the work finishes; blocking calls synchronise the stream before returning.
 *  - A context is not thread safe; the caller serialises calls on it.
 *  - Every device buffer of the library (spectra, preconditioner, spectral and
 *    Krylov workspaces, network state) comes from the caller's allocator given
 *    to mlfft_create() and goes back to it; the library never calls hipMalloc.
 *    Buffers grow on demand and are kept for later calls; they are released by
 *    mlfft_drop_array() (an array's spectra and factors) and mlfft_destroy().
 *    An allocation the allocator refuses ends the call with MLFFT_E_NOMEM.
 */
#ifndef MLFFT_H
#define MLFFT_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mlfft_ctx_s* mlfft_ctx;

typedef enum {
    MLFFT_OK = 0,
    MLFFT_NOT_CONVERGED = 1,
    MLFFT_E_ARG = -1,        /* invalid argument (sizes, null pointers, non-finite input) */
    MLFFT_E_NOMEM = -2,      /* device allocation failed */
    MLFFT_E_HIP = -3,        /* a HIP runtime call or kernel launch failed */
    MLFFT_E_SINGULAR = -4,   /* a required inverse does not exist */
    MLFFT_E_STATE = -5       /* call not valid in the current state (e.g. unknown array id) */
} mlfft_status;

typedef enum {
    MLFFT_FP64 = 0,          /* complex128 data, FP64 FFTs and FP64 MFMA block product */
    MLFFT_FP32 = 1,          /* complex64 data, FP32 FFTs and FP32 MFMA block product */
    MLFFT_FP32_BF16GEMM = 2  /* complex64 data, FP32 FFTs, block product with bf16 inputs and FP32 accumulation */
} mlfft_prec;

/* Device allocator of the caller.  alloc_fn returns `bytes` bytes of device
 * memory of the context's device, aligned to at least 256 bytes, usable by work
 * enqueued on the context's stream, or NULL if it cannot (the library then
 * reports MLFFT_E_NOMEM); free_fn gives such a pointer back.  free_fn may be
 * called while work enqueued earlier on the context's stream still reads the
 * buffer: the allocator must not hand that memory to work that is not ordered
 * after it on that stream (a stream-ordered allocator, or a caching allocator
 * keyed by the stream such as PyTorch's, does this), or must synchronise the
 * stream first. */
typedef void* (*mlfft_alloc_fn)(size_t bytes, void* user);
typedef void (*mlfft_free_fn)(void* ptr, void* user);

/* Create a context on HIP device `device`, enqueueing on `hip_stream`
 * (a hipStream_t; NULL = the default stream), drawing all device memory from
 * alloc_fn / free_fn (both required; `user` is passed through to them).
 * *out receives the handle.  Sec. III-C hands GMRES a function for the
 * product and one for the preconditioner; a context holds both. */
mlfft_status mlfft_create(int device, void* hip_stream, mlfft_alloc_fn alloc_fn, mlfft_free_fn free_fn, void* user,
                          mlfft_ctx* out);

/* Free every device buffer the context owns and the context itself.  NULL is accepted. */
mlfft_status mlfft_destroy(mlfft_ctx ctx);

/* Message of the last error on this context; valid until the next call on it.
 * With ctx == NULL: the message of the last failed mlfft_create(). */
const char* mlfft_last_error(mlfft_ctx ctx);

/* Change the stream the context enqueues on. */
mlfft_status mlfft_set_stream(mlfft_ctx ctx, void* hip_stream);

/* Register (or replace) array `array_id` (>= 0) and build everything the
 * solver needs from its unique blocks.
 *
 * blocks: (2Ny-1) * (2Nx-1) * b * b complex128, layout [p+Ny-1][q+Nx-1][m][n],
 * where R_{p,q}[m][n] couples test basis m of cell (iy, ix) with source basis n
 * of cell (iy-p, ix-q) (T_ij = t_{i-j}, eq. T and eq. Tblock).  These are the
 * "unique blocks" of Z_A (Sec. II-C, storage (2N^[1]-1)(N^[0])^2 per level).
 * blocks_on_device: 0 = host pointer, 1 = device pointer.  The library copies
 * what it needs; the caller may free the blocks when the call returns.
 *
 * Built here (blocking; reported separately from solve time, like the paper's
 * "Con." split, Sec. V):
 *  - the block spectra G_hat(k) = 2-D DFT of the block grid embedded in the
 *    (2Ny) x (2Nx) circulant (eqs. cT1, circL1, circL2, multL), in FP64 with
 *    FP32 and bf16 copies;
 *  - the two-level Strang block-circulant preconditioner on the Ny x Nx torus
 *    and the FP64 inverse of each of its Nx*Ny frequency blocks, with FP32 and
 *    bf16 copies.  A frequency block whose reciprocal 1-norm condition number
 *    is below 1e-12 is replaced by the inverse of the self block R_{0,0}
 *    (the Kindt preconditioner of Sec. III-B); the count is reported by
 *    mlfft_array_info().  If R_{0,0} itself is singular the call fails with
 *    MLFFT_E_SINGULAR;
 *  - the inverse of R_{0,0} for the self-block preconditioner.
 * Limits: 1 <= Nx, Ny <= 32, 1 <= b <= 256.  Non-finite blocks: MLFFT_E_ARG. */
mlfft_status mlfft_set_blocks(mlfft_ctx ctx, int array_id, int Nx, int Ny, int b,
                              const void* blocks, int blocks_on_device);

/* Remove an array and free its buffers. */
mlfft_status mlfft_drop_array(mlfft_ctx ctx, int array_id);

/* Give array `array_id` the border blocks of the full impedance matrix
 *     Z = [[Z_A, Z_B^T], [Z_B, Z_C]]   (Sec. I, eq. Zblock):
 * Nc unknowns outside the Toeplitz part (the border of a connected array that the
 * mesh partition leaves outside the repeated cells), their coupling with the array
 * Z_B (Nc x N, N = Nx Ny b) and their self interaction Z_C (Nc x Nc), both row-major
 * complex128 (Z_B[i][(iy Nx + ix) b + m]), host (on_device = 0) or device pointers;
 * the library copies them.  From then on every vector of the array has N + Nc entries
 * per column, [x_A (the vector layout above), x_C], and every call works on the full Z:
 *  - mlfft_matvec multiplies blockwise (eq. ZIVblock): Z_A x_A by the MLFFT product,
 *    the border terms Z_B^T x_C, Z_B x_A and Z_C x_C as dense MFMA products;
 *  - preconditioners 1, 2 and 4 become P_X = blockdiag(P'_X, Z_C) (Sec. III-B), the
 *    border part applied with Z_C^{-1} (formed here, FP64 LU with partial pivoting);
 *    the learned correction (3) is not defined with a border (MLFFT_E_ARG);
 *  - mlfft_solve / mlfft_solve_batch run on the full system;
 *  - mlfft_direct_solve uses the Schur complement of Sec. III-E.
 * Nc = 0 removes the border.  Z_C with rcond < 1e-14: MLFFT_E_SINGULAR (no border is
 * kept).  Non-finite entries: MLFFT_E_ARG.  Blocking. */
mlfft_status mlfft_set_border(mlfft_ctx ctx, int array_id, int Nc, const void* ZB, const void* ZC, int on_device);

typedef struct {
    int Nx, Ny, b;
    int Px, Py;              /* matvec circulant grid, 2Nx x 2Ny */
    int pc_fallbacks;        /* preconditioner frequencies replaced by the self-block inverse */
    double pc_min_rcond;     /* smallest reciprocal condition number over the preconditioner blocks */
    size_t device_bytes;     /* device memory held for this array */
    int Nc;                  /* border unknowns (mlfft_set_border), 0 without a border */
} mlfft_array_info_t;

mlfft_status mlfft_array_info(mlfft_ctx ctx, int array_id, mlfft_array_info_t* out);

/* y = Z_A x for W columns (eq. multL): zero-pad every column to the
 * (2Ny) x (2Nx) grid (eq. xc2), blockwise 2-level FFT (eq. F2), per-frequency
 * b x b block product, inverse FFT, keep the first Ny x Nx cells.
 * x, y: device pointers, W columns in the vector layout; complex128 for
 * MLFFT_FP64, complex64 otherwise.  x and y must not overlap.
 * Asynchronous on the context's stream. */
mlfft_status mlfft_matvec(mlfft_ctx ctx, int array_id, int W, const void* x, void* y, mlfft_prec prec);

/* y = Z_A x exactly as mlfft_matvec (same kernels, same results), for callers
 * that cannot allocate device memory: code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation.  The two spectral workspaces
 * of the product come from a fixed array of 2 x 64 MiB in the library's own
 * device memory (every device the library runs on holds one from module load
 * until the process ends), never from the allocator: the call allocates
 * nothing on the device.  Limit: 4 Nx Ny b W x (16 bytes for MLFFT_FP64, 8
 * otherwise) must not exceed 64 MiB (e.g. W <= 163 at 10 x 10, b = 64 in FP64);
 * larger products return MLFFT_E_ARG before anything is enqueued.  Every call
 * on one device shares that device's array: calls that overlap in time on one
 * device (two contexts or streams running concurrently) race and give wrong
 * results; calls ordered on one stream are safe.  The array needs no clearing
 * (each product overwrites the workspace it reads).  Not profiled.  Argument
 * rules as for mlfft_matvec.  Asynchronous. */
mlfft_status mlfft_matvec_noalloc(mlfft_ctx ctx, int array_id, int W, const void* x, void* y, mlfft_prec prec);

/* y = alpha Z_A x + beta v for W columns: the MLFFT product of mlfft_matvec with
 * its result scaled and added to v in the inverse transform's epilogue (the true
 * residual V - Z_A I of Sec. III, "ZI = V", is alpha = -1, beta = 1).  v may be
 * NULL (then y = alpha Z_A x).  Layout and precision rules as for mlfft_matvec;
 * x, v and y must not overlap.  Non-finite alpha or beta: MLFFT_E_ARG.  Asynchronous. */
mlfft_status mlfft_matvec_axpby(mlfft_ctx ctx, int array_id, int W, double alpha, const void* x, double beta,
                                const void* v, void* y, mlfft_prec prec);

/* out = alpha x + beta y over n complex values (y may be NULL), with x and y of
 * precision in_prec and out of precision out_prec (MLFFT_FP64 = complex128,
 * MLFFT_FP32 = complex64; the combination is formed in FP64 and rounded once).
 * Forms the error x* - x_k and the precision casts of training pairs.  out may
 * be x or y itself when the precisions match; other overlaps: MLFFT_E_ARG.
 * Asynchronous. */
mlfft_status mlfft_axpby(mlfft_ctx ctx, size_t n, double alpha, const void* x, double beta, const void* y,
                         int in_prec, void* out, int out_prec);

/* z = P^{-1} r with P the preconditioner `kind`:
 *   1 = two-level Strang block circulant: z = IFFT2(S_hat(k)^{-1} FFT2(r)) on the
 *       Ny x Nx torus;
 *   2 = self-block (Kindt) preconditioner P'_K of Sec. III-B: every cell's
 *       b-vector multiplied by R_{0,0}^{-1};
 *   4 = row preconditioner P'_Z of Sec. III-B: every row of cells (Nx b unknowns)
 *       multiplied by (T^[1]_0)^{-1}, the inverse of the self interaction of one
 *       array row (eq. Tblock), as one dense product on MFMA (FP64 for MLFFT_FP64,
 *       FP32 otherwise).  The inverse is formed on first use (FP64 LU with partial
 *       pivoting, blocking; MLFFT_E_SINGULAR if its 1-norm rcond is below 1e-14).
 * Layout and precision rules as for mlfft_matvec.  Asynchronous. */
mlfft_status mlfft_precond_apply(mlfft_ctx ctx, int array_id, int kind, int W, const void* r, void* z,
                                 mlfft_prec prec);


/* ------------------------------------------------------------------ solve */

typedef struct {
    int restart;         /* GMRES restart length m, 1..31 (default 30) */
    int max_restarts;    /* restart cycles per inner solve (default 100) */
    double tol;          /* target true FP64 relative residual ||V_w - Z I_w|| / ||V_w|| per column (default 1e-6) */
    int inner_prec;      /* mlfft_prec of the inner GMRES (default MLFFT_FP32).  MLFFT_FP64 = plain FP64 GMRES:
                            the outer loop then only confirms the true residual */
    double inner_tol;    /* floor of the residual reduction asked of each FP32 / BF16 inner solve; every inner
                            solve aims at max(inner_tol, 0.3 * tol * ||V_w|| / ||r_w||).  0 (default) = automatic:
                            3e-7 for MLFFT_FP32, 1e-2 for MLFFT_FP32_BF16GEMM; ignored for MLFFT_FP64 */
    int max_outer;       /* FP64 refinement steps (default 10) */
    int precond;         /* 0 none, 1 block circulant (default), 2 self block (Kindt, P'_K), 3 learned correction of
                            the block-circulant output (flexible GMRES; needs a network, see mlfft_net_create),
                            4 row preconditioner P'_Z (see mlfft_precond_apply) */
    int orth;            /* 1 classical Gram-Schmidt, 2 classical Gram-Schmidt applied twice (default): the
                            second projection is formed from the FP64 Gram matrix of the stored basis, so
                            both read the basis twice per step; FP64 sums */
    int x0_given;        /* 1: I holds the initial guess on entry; 0: start from zero (default) */
    int record_history;  /* 1: fill info->history */
    int use_graph;       /* k in 1..8: run the Krylov steps (preconditioner, product,
                            orthogonalisation, rotation) k at a time as HIP graphs, captured the
                            second time their launch configuration occurs and replayed afterwards;
                            the host reads the column states once per graph instead of once per
                            step.  Solutions, iteration counts and residuals are identical to
                            use_graph = 0 (eager launches); with k > 1, steps after the last column
                            retires inside a graph are spent (and counted in matvecs_inner), so
                            k = 1 does the eager work with one launch per step.  Needs a context
                            stream other than the NULL stream (else the steps run eagerly).  Graphs
                            are dropped whenever a library buffer is reallocated.  Profiling does
                            not see captured launches.  MLFFT_E_ARG outside 0..8. */
    int mode;            /* 0 (default): one Krylov space per right-hand side (the paper's split
                            mode with all columns batched); 1: global GMRES (eq. ZIVvec), one
                            Krylov space for all W columns (of all arrays of a batch) with
                            Frobenius inner products; an inner solve aims at
                            ||R||_F <= f * tol * ||V||_F, and once that holds at
                            ||R||_F <= f * tol * min ||V_w|| over the columns still above tol.
                            The outer FP64 loop requires every column's own relres <= tol and
                            repeats the global inner solve until it holds; info->iters and info->history then report the
                            global iteration for every column.  MLFFT_E_ARG if the batch has
                            more than 2^31-1 unknowns in all. */
    int pc_bf16;         /* 1: an MLFFT_FP32 inner solve runs the per-frequency product of its
                            preconditioner (kinds 1, 2 and the block-circulant part of 3) with
                            bf16 inverse blocks and bf16-rounded vectors, FP32 accumulation (the
                            FFTs stay FP32).  Honoured only while the preconditioned directions
                            are stored (always for kind 3; for kinds 1 and 2 when the workspace
                            fits), since the solution is then formed from the very directions
                            the Arnoldi process saw; otherwise the product stays FP32.  The FP64
                            true residual still decides convergence.  0 (default): the product
                            runs in the inner precision.  Ignored for other inner precisions. */
} mlfft_solve_opts;

typedef struct {
    int* iters;          /* [W] inner GMRES iterations per column, or NULL (host, caller-owned) */
    int* outer;          /* [W] refinement steps that worked on the column, or NULL */
    double* relres;      /* [W] final true FP64 relative residual, or NULL */
    int* converged;      /* [W] 1 if relres <= tol, or NULL */
    double* history;     /* [history_len * W] residual estimate / ||V_w|| after each inner iteration
                            (row-major by iteration), or NULL */
    int history_len;     /* rows of history */
    int fallbacks;       /* out: learned-correction outputs replaced by the plain block-circulant output */
    int matvecs64;       /* out: FP64 MLFFT products used for true residuals */
    int matvecs_inner;   /* out: batched MLFFT products in the inner precision */
    int precond_applies; /* out: batched preconditioner applies */
    int net_applies;     /* out: batched network corrections */
    int pc_switched;     /* out: 1 if the solve turned the learned correction (precond 3) off and went on
                            with the plain block-circulant preconditioner, because a refinement step left
                            the FP64 true residual of the columns it solved above half of its previous
                            2-norm (each inner solve asks for a reduction of at least 0.3) */
} mlfft_solve_info;

/* Fill *opts with the defaults above. */
mlfft_status mlfft_solve_default_opts(mlfft_solve_opts* opts);

/* Solve Z_A I = V for the W columns of V (Sec. III, "ZI = V"; multiple right-hand
 * sides of Sec. III-C, eq. ZIVmat): restarted GMRES with the MLFFT matvec and the
 * chosen preconditioner, one Krylov space per column, FP64 iterative refinement
 * around an FP32 / BF16 inner solve.  V, I: device, complex128, W columns in the
 * vector layout.  opts == NULL uses the defaults; info may be NULL.
 * Blocking: returns when every column converged (MLFFT_OK) or the limits are
 * reached (MLFFT_NOT_CONVERGED, outputs valid).  Zero columns of V give zero
 * columns of I.  Non-finite residuals: MLFFT_E_ARG.  When V and I do not overlap
 * the solve reads V and builds the solution in I directly (no staging copies), so
 * after an error return I is unspecified; overlapping V and I (also V == I) are
 * staged through the workspace. */
mlfft_status mlfft_solve(mlfft_ctx ctx, int array_id, int W, const void* V, void* I,
                         const mlfft_solve_opts* opts, mlfft_solve_info* info);

/* The same for several arrays of different shapes in one batch: every MLFFT
 * product, preconditioner apply and Krylov step of the solve covers all arrays
 * in one grouped launch.  V[i], I[i]: device, complex128, W[i] columns of array
 * array_ids[i] (ids distinct).  info: NULL or one struct for the whole batch whose
 * per-column arrays are indexed by the concatenated column order.  The solve works
 * in V and I directly when the V[i] lie back to back in batch order in one range,
 * the I[i] likewise, and the two ranges do not overlap; otherwise V and I are
 * staged through the workspace. */
mlfft_status mlfft_solve_batch(mlfft_ctx ctx, int n_arrays, const int* array_ids, const int* W,
                               const void* const* V, void* const* I,
                               const mlfft_solve_opts* opts, mlfft_solve_info* info);

/* ------------------------------------------------------------------ direct solver and dense algebra */

/* Z_A I = V by the block Rybicki recursion on level 2 (Sec. III-D, eqs. xmpo, xi,
 * (with a border, mlfft_set_border: Z I = V by the Schur complement of Sec. III-E,
 * Z_A [U F] = [V_A Z_B^T] through the recursion, I_C = (Z_C - Z_B F)^{-1}(V_C - Z_B U),
 * I_A = U - F I_C; vectors of N + Nc entries per column)
 * GM1, HM1, HM, GH): the recursion runs over the Ny rows of the array, its blocks
 * are the dense level-1 matrices R_p = T^[1]_p (order Nx b, eq. Tblock) formed from
 * the unique blocks of mlfft_set_blocks, and all W right-hand sides are carried
 * along.  Every inverse of the recursion (R_0 and the sections D and E of each
 * order) is formed explicitly in FP64 (LU with partial pivoting) and its 1-norm
 * reciprocal condition number checked: below 1e-14 the call stops with
 * MLFFT_E_SINGULAR naming the section (the recursion needs every leading block
 * section to be invertible).  All products run as FP64 MFMA GEMMs.  V, I: device
 * complex128, W columns in the vector layout, not overlapping.  min_rcond and
 * flops (host, may be NULL) receive the smallest rcond met and the floating-point
 * operations executed (8 per complex multiply-add).  Device memory: about
 * (4 Ny + 3) (Nx b)^2 x 16 bytes for the duration of the call.  Blocking. */
mlfft_status mlfft_direct_solve(mlfft_ctx ctx, int array_id, int W, const void* V, void* I, double* min_rcond,
                                double* flops);

/* C = alpha A B + beta C for column-major complex matrices on the device
 * (A: M x K, B: K x N, C: M x N, leading dimensions lda >= M, ldb >= K, ldc >= M),
 * complex128 for MLFFT_FP64 (FP64 MFMA) or complex64 for MLFFT_FP32 (FP32 MFMA).
 * beta = 0 does not read C.  C must not overlap A or B.  Asynchronous.  The dense
 * product of the row preconditioner, the direct solver and the border blocks. */
mlfft_status mlfft_dense_gemm(mlfft_ctx ctx, int prec, int M, int N, int K, double alpha_re, double alpha_im,
                              const void* A, long lda, const void* B, long ldb, double beta_re, double beta_im, void* C,
                              long ldc);

/* C = alpha A^H B + beta C (complex128, FP64 MFMA) with A stored K x M (lda >= K),
 * B K x N (ldb >= K), C M x N (ldc >= M), column-major on the device; the Gram
 * products of mlfft_spectrum.  Asynchronous. */
mlfft_status mlfft_dense_gemm_ah(mlfft_ctx ctx, int M, int N, int K, double alpha_re, double alpha_im, const void* A,
                                 long lda, const void* B, long ldb, double beta_re, double beta_im, void* C, long ldc);

/* sigma (host, l values, descending) = square roots of the eigenvalues of the pencil
 * M v = lambda G v for Hermitian l x l G (positive definite) and M (device complex128,
 * column-major, both overwritten): Cholesky G = L L^H, T = L^{-1} M L^{-H}, cyclic
 * Jacobi on T in one workgroup (the last step of mlfft_spectrum).  1 <= l <= 1024.
 * G not positive definite: MLFFT_E_SINGULAR.  Blocking. */
mlfft_status mlfft_dense_gen_eig(mlfft_ctx ctx, int l, void* G, void* M, double* sigma);

/* B <- A^{-1} B for the n x n complex128 matrix A (device, column-major, overwritten
 * by its LU factors: blocked right-looking LU with partial pivoting, as LAPACK's
 * zgetrf / zgetrs) and ncols columns of B.  An exactly zero pivot gives
 * MLFFT_E_SINGULAR.  Blocking. */
mlfft_status mlfft_dense_solve(mlfft_ctx ctx, int n, void* A, long lda, void* B, long ldb, int ncols);

/* ------------------------------------------------------------------ spectrum diagnostics */

/* Approximate largest singular values of the preconditioned operator A = P^{-1} Z
 * (Sec. V, the spectra of P^{-1} Z for P = I, P_K and P_Z) by the randomized range
 * finder of Halko, Martinsson and Tropp with every product through the FP64 MLFFT
 * matvec and preconditioner: Y = A Omega, `power_iters` steps Y = A (A^H Y), then
 * with Y = Q R and C = A^H Y the matrix B = Q^H A has B B^H = R^{-H} C^H C R^{-1},
 * whose eigenvalues (Cholesky of Y^H Y and Jacobi on the device) are the squared
 * singular values returned.  kind: 0 (P = I, the spectrum of Z), 1 block circulant,
 * 2 P'_K, 4 P'_Z (with a border: P_X).  Omega: device complex128, l test vectors in
 * the vector layout (the caller draws them; 1 <= l <= 1024, l <= unknowns).
 * sigma: host, l doubles, descending.  The adjoint is applied as
 * A^H y = conj(Z P^{-1} conj(y)), which holds for complex-symmetric Z and P, i.e.
 * reciprocal blocks (R_{-p,-q} = R_{p,q}^T, the symmetric MoM form); for other
 * blocks the result is not the spectrum of A.  Without power steps the leading
 * values are accurate only when the spectrum decays; 1 or 2 steps sharpen them
 * (power_iters <= 8).  A rank-deficient sketch: MLFFT_E_SINGULAR.  Device memory:
 * 4 l N x 16 bytes.  Blocking. */
mlfft_status mlfft_spectrum(mlfft_ctx ctx, int array_id, int kind, int l, const void* Omega, int power_iters,
                            double* sigma);

/* ------------------------------------------------------------------ learned correction */
/*
 * A small convolutional network on the array grid corrects the output of the
 * block-circulant preconditioner (the paper asks for a preconditioner that
 * covers all neighbouring elements, Sec. V; the network is this library's
 * choice).  A column y (complex64, vector layout) is seen as an NHWC image of
 * Ny x Nx pixels with 2b real channels (channel 2m + part).  Normalisation:
 * s = ||y||, phi = arg of the entry of largest modulus, y_hat = y e^{-i phi}/s.
 * Network: four 3x3 convolutions, zero "same" padding, no bias,
 * 2b -> hidden -> hidden -> hidden -> 2b, ReLU after the first three; bf16
 * inputs and weights, FP32 accumulation.  Output z = s e^{i phi}(y_hat + Net(y_hat)).
 * Weights (FP32 master copy) are one flat array, layer by layer, each layer
 * [c_out][c_in][3][3] row-major.  One network per context.
 */

/* Create (or replace) the context's network for b basis functions per cell.
 * The first three layers start He-normal (standard deviation sqrt(2 / (9 c_in)))
 * from a counter-based generator (splitmix64 of (seed, weight index), Box-Muller);
 * the last layer starts at zero, so the correction starts as the identity.
 * seed = 0: every weight starts at zero. */
mlfft_status mlfft_net_create(mlfft_ctx ctx, int b, int hidden, unsigned seed);

/* Number of FP32 weights of the network (0 without a network). */
size_t mlfft_net_num_weights(mlfft_ctx ctx);

/* Copy n = mlfft_net_num_weights() FP32 weights from / to host memory.
 * Setting weights resets the Adam state.  Non-finite weights: MLFFT_E_ARG. */
mlfft_status mlfft_net_set_weights(mlfft_ctx ctx, const float* host, size_t n);
mlfft_status mlfft_net_get_weights(mlfft_ctx ctx, float* host, size_t n);

/* Raw network on W images: x, out device FP32 NHWC [W][H][Wd][2b] (x is rounded
 * to bf16 before the first convolution).  Asynchronous. */
mlfft_status mlfft_net_forward(mlfft_ctx ctx, int W, int H, int Wd, const void* x, void* out);

/* z = s e^{i phi}(y_hat + Net(y_hat)) for W columns of array array_id (whose b must
 * match the network); y, z device complex64 in the vector layout.  A column whose
 * result is not finite is replaced by y.  Asynchronous. */
mlfft_status mlfft_net_apply(mlfft_ctx ctx, int array_id, int W, const void* y, void* z);

/* Loss and weight gradients for W training pairs on an H x Wd grid:
 * y = block-circulant output P^{-1} r, e = the error it should become (device,
 * complex64, vector layout).  Loss = mean over pairs of
 * ||y_hat + Net(y_hat) - e_hat||^2 / ||e_hat||^2 with e_hat = e e^{-i phi}/s.
 * host_grads (may be NULL): mlfft_net_num_weights() floats, layout of the weights.
 * Blocking. */
mlfft_status mlfft_net_grads(mlfft_ctx ctx, int W, int H, int Wd, const void* y, const void* e,
                             float* host_grads, float* loss);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias corrected) on the loss
 * above with learning rate lr; *loss receives the loss before the step.  Blocking. */
mlfft_status mlfft_net_train_step(mlfft_ctx ctx, int W, int H, int Wd, const void* y, const void* e,
                                  float lr, float* loss);

/* ------------------------------------------------------------------ autotuning */

/* Time the candidate launch shapes of the MLFFT block product (waves per
 * workgroup x columns per LDS tile x product form: four real products, three
 * real products, three real products with a flat assignment of (frequency,
 * 16-row slice) items to eight- or four-wave workgroups) and of the 2-D FFTs (basis functions per
 * workgroup, for the MLFFT grid and the preconditioner torus) on array
 * array_id with W columns in precision prec, `reps` timed runs each, and keep
 * the fastest for the rest of the process (all contexts).  Blocking; overwrites
 * the context's spectral workspaces. */
mlfft_status mlfft_autotune(mlfft_ctx ctx, int array_id, int W, int prec, int reps);

/* Write the choices in force for array_id's shape, followed by the timings of
 * the last mlfft_autotune(), as text lines into buf (n bytes, truncated). */
mlfft_status mlfft_tune_report(mlfft_ctx ctx, int array_id, char* buf, size_t n);

/* Re-apply choices from text in the format of mlfft_tune_report(): lines
 * "gemm prec bp waves nt form" (form 0 four products, 1 three products, 2 three
 * products with the flat assignment, which takes prec 1 with waves 8 and nt 32
 * or 16, prec 1 with waves 4 and nt 16, or prec 0 with waves 4 and nt 16; form 4,
 * prec 1 with waves 8 and nt 16 or prec 0 with waves 4 and nt 16: the flat
 * assignment with X tiles loaded straight into LDS, in FP32 for even b only, else
 * the launch falls back to form 2; "gemm prec bp 0 0 0" restores the default
 * shape) and
 * "fftshape prec pad dir Nx Ny b cm half" (dir 0 forward, 1 inverse; cm the
 * m-chunk, 0 for the default rule; half 1 for the half-height tile of a padded
 * transform, 0 for the one-pass tile, -1 for the default), the older
 * "fftcm prec pad Nx Ny b cm" (both directions), and "gemmpc 2 bp waves nt form" for the bf16
 * preconditioner product with bp a multiple of 16 (forms 3 and 5, bp <= 208, 8
 * waves, 32-column tiles: each X tile staged once for all row slices of its
 * frequency, form 3 with the tiles of one frequency (or a column chunk of it) per
 * workgroup, form 5 with all (frequency, tile) items split evenly over the
 * workgroups, the default for bp in 112..208; form 2 with 8 waves and 32-column
 * tiles: the flat kernel, the default elsewhere; waves 0 restores the default),
 * "gemmpcwg n" for the number of workgroups a launch of form 3 or 5 aims at (form 3
 * splits the columns of a frequency to reach it, default 512; form 5 default: the
 * device's CU count); other lines are ignored.  MLFFT_E_ARG for a malformed gemm, gemmpc, gemmpcwg, fftshape or fftcm line. */
mlfft_status mlfft_tune_import(mlfft_ctx ctx, const char* text);

/* ------------------------------------------------------------------ profiling */

typedef struct {
    char name[32];       /* kernel group: mlfft_fwd_fft, block_gemm, mlfft_inv_fft, precond_fwd_fft, precond_gemm,
                            precond_inv_fft, arnoldi, net_forward, net_backward */
    int prec;            /* mlfft_prec of the launches */
    long launches;
    double ms;           /* summed launch durations (HIP events on the context's stream) */
    double bytes;        /* summed algorithmic bytes (minimum HBM traffic of the operation) */
    double flops;        /* summed algorithmic flops (block products: 8 b^2 W per frequency) */
} mlfft_kernel_stat;

/* Enable (1) or disable (0) per-launch timing of the hot kernels; either call
 * discards earlier records.  Enabling adds two event records per launch. */
mlfft_status mlfft_profile_enable(mlfft_ctx ctx, int enable);

/* Aggregate the records since the last mlfft_profile_enable() per (group, prec).
 * Writes at most max_out entries to out and the number of groups to *n_out.
 * Blocking (synchronises the stream). */
mlfft_status mlfft_profile_read(mlfft_ctx ctx, mlfft_kernel_stat* out, int max_out, int* n_out);

#ifdef __cplusplus
}
#endif

#endif /* MLFFT_H */
