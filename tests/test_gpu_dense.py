"""GPU parity of the dense paths: the MFMA complex GEMM and the LU solve (against NumPy),
the row preconditioner P'_Z (against the oracle's row_apply, Sec. III-B) and the block
Rybicki direct solver (against dense LU and the oracle's recursion, Sec. III-D).

Bars, per column: GEMM FP64 1e-13, FP32 1e-5 (one rounding per product term of a
K-term sum in FP32 relative to the column norm); LU solves 1e-10 on matrices of
condition number below 1e3; P'_Z FP64 1e-12, FP32 1e-5; Rybicki 1e-10 against LU
(the oracle's own bar for its recursion).
"""
import numpy as np
import pytest
import torch

from oracle import direct
from oracle import precond as opc
from oracle import toeplitz as tp
from paper_2506_20350_amd import abi, synth
from tests.gpu_util import ctx, relerr, to_dev, to_host  # noqa: F401

pytestmark = pytest.mark.gpu

DT = {abi.MLFFT_FP64: torch.complex128, abi.MLFFT_FP32: torch.complex64}


def crand(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def colmajor(A, ld, dtype):
    """A (rows x cols) into a device buffer in column-major order with leading dimension ld."""
    rows, cols = A.shape
    buf = np.zeros((cols, ld), np.complex128)
    buf[:, :rows] = A.T
    return torch.from_numpy(buf).to(dtype).cuda()


def from_colmajor(t, rows):
    return to_host(t)[:, :rows].T


@pytest.mark.parametrize("prec", [abi.MLFFT_FP64, abi.MLFFT_FP32])
@pytest.mark.parametrize("M,N,K,pad", [(1, 1, 1, 0), (37, 53, 19, 3), (64, 64, 64, 0), (130, 70, 200, 5),
                                       (300, 5, 1000, 1), (16, 200, 7, 0), (65, 65, 0, 2)])
def test_dense_gemm_matches_numpy(ctx, prec, M, N, K, pad):
    rng = np.random.default_rng(M * 7 + N * 3 + K)
    A, B, C = crand(rng, M, K), crand(rng, K, N), crand(rng, M, N)
    alpha, beta = 0.7 - 1.3j, -0.4 + 0.25j
    Ad, Bd, Cd = colmajor(A, M + pad, DT[prec]), colmajor(B, max(K, 1) + pad, DT[prec]), colmajor(C, M + pad, DT[prec])
    if prec == abi.MLFFT_FP32:
        A, B, C = (x.astype(np.complex64).astype(np.complex128) for x in (A, B, C))
    ctx.sync_stream()
    abi.mlfft_dense_gemm(ctx.h, prec, M, N, K, alpha, Ad.data_ptr(), M + pad, Bd.data_ptr(), max(K, 1) + pad, beta,
                         Cd.data_ptr(), M + pad)
    ref = alpha * (A @ B) + beta * C
    got = from_colmajor(Cd, M)
    assert relerr(got.T, ref.T) <= (1e-13 if prec == abi.MLFFT_FP64 else 1e-5)
    # the padding rows between columns are left alone
    if pad:
        assert np.all(to_host(Cd)[:, M:] == 0)


def test_dense_gemm_beta_zero_ignores_nan_output(ctx):
    rng = np.random.default_rng(3)
    A, B = crand(rng, 40, 30), crand(rng, 30, 20)
    Ad, Bd = colmajor(A, 40, torch.complex128), colmajor(B, 30, torch.complex128)
    Cd = torch.full((20, 40), complex(float("nan"), 0.0), dtype=torch.complex128, device="cuda")
    ctx.sync_stream()
    abi.mlfft_dense_gemm(ctx.h, abi.MLFFT_FP64, 40, 20, 30, 1.0, Ad.data_ptr(), 40, Bd.data_ptr(), 30, 0.0,
                         Cd.data_ptr(), 40)
    assert relerr(from_colmajor(Cd, 40).T, (A @ B).T) <= 1e-13


@pytest.mark.parametrize("M,N,K,pad", [(1, 1, 1, 0), (48, 48, 48, 0), (40, 40, 180000, 0), (70, 33, 129, 3),
                                       (130, 65, 17, 1)])
def test_dense_gemm_conj_transposed_matches_numpy(ctx, M, N, K, pad):
    rng = np.random.default_rng(M + 3 * N + K)
    A, B, C = crand(rng, K, M), crand(rng, K, N), crand(rng, M, N)
    alpha, beta = 1.1 + 0.2j, 0.5 - 0.5j
    Ad, Bd, Cd = (colmajor(A, K + pad, torch.complex128), colmajor(B, K + pad, torch.complex128),
                  colmajor(C, M + pad, torch.complex128))
    ctx.sync_stream()
    abi.mlfft_dense_gemm_ah(ctx.h, M, N, K, alpha, Ad.data_ptr(), K + pad, Bd.data_ptr(), K + pad, beta, Cd.data_ptr(),
                            M + pad)
    ref = alpha * (A.conj().T @ B) + beta * C
    assert relerr(from_colmajor(Cd, M).T, ref.T) <= 1e-13


@pytest.mark.parametrize("l", [1, 2, 7, 48, 64, 129, 256])
def test_generalised_hermitian_eigenvalues_match_numpy(ctx, l):
    """sqrt of the eigenvalues of M v = lambda G v (Cholesky + round-robin Jacobi in one workgroup)."""
    import scipy.linalg as sla
    rng = np.random.default_rng(l)
    Y = crand(rng, l + 5, l)
    G = Y.conj().T @ Y
    Cm = crand(rng, 2 * l, l)
    Mm = Cm.conj().T @ Cm
    Gd, Md = colmajor(G, l, torch.complex128), colmajor(Mm, l, torch.complex128)
    ctx.sync_stream()
    sv = abi.mlfft_dense_gen_eig(ctx.h, l, Gd.data_ptr(), Md.data_ptr())
    ref = np.sqrt(np.clip(np.sort(sla.eigh(Mm, G, eigvals_only=True))[::-1], 0, None))
    assert np.max(np.abs(sv - ref)) <= 1e-10 * ref[0]


@pytest.mark.parametrize("n,ncols", [(1, 1), (5, 3), (33, 7), (100, 40), (257, 9), (64, 1)])
def test_dense_solve_matches_numpy(ctx, n, ncols):
    rng = np.random.default_rng(n + ncols)
    A = crand(rng, n, n) + 2 * np.sqrt(n) * np.eye(n)
    # permute rows so that partial pivoting has to interchange them
    A = A[rng.permutation(n)]
    B = crand(rng, n, ncols)
    Ad, Bd = colmajor(A, n, torch.complex128), colmajor(B, n, torch.complex128)
    ctx.sync_stream()
    abi.mlfft_dense_solve(ctx.h, n, Ad.data_ptr(), n, Bd.data_ptr(), n, ncols)
    ref = np.linalg.solve(A, B)
    assert np.linalg.cond(A) < 1e3
    assert relerr(from_colmajor(Bd, n).T, ref.T) <= 1e-10


def test_dense_solve_reports_exactly_singular_matrix(ctx):
    n = 6
    A = np.eye(n, dtype=np.complex128)
    A[3] = A[1]                                   # two equal rows
    Ad, Bd = colmajor(A, n, torch.complex128), colmajor(np.ones((n, 1)), n, torch.complex128)
    ctx.sync_stream()
    with pytest.raises(abi.MlfftError) as e:
        abi.mlfft_dense_solve(ctx.h, n, Ad.data_ptr(), n, Bd.data_ptr(), n, 1)
    assert e.value.status == abi.MLFFT_E_SINGULAR


# ----------------------------------------------------------------- row preconditioner P'_Z

@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("Nx,Ny,b,W", [(4, 3, 6, 2), (1, 5, 7, 3), (7, 1, 5, 1), (10, 10, 24, 5), (30, 4, 16, 2)])
def test_row_preconditioner_matches_oracle(ctx, prec, Nx, Ny, b, W):
    blocks = synth.green_blocks(Nx, Ny, b, np.pi, seed=2)
    ctx.set_blocks(120, blocks)
    R = synth.random_vectors(Nx * Ny * b, W, seed=4)
    z = ctx.precond_apply(120, to_dev(R, torch.complex128 if prec == "fp64" else torch.complex64), kind=4, prec=prec)
    ref = opc.row_apply(blocks, R)
    assert relerr(to_host(z), ref) <= (1e-12 if prec == "fp64" else 1e-5)


@pytest.mark.parametrize("inner", ["fp64", "fp32"])
def test_solve_with_row_preconditioner_matches_lu(ctx, inner):
    Nx, Ny, b = 6, 5, 12
    blocks = synth.green_blocks(Nx, Ny, b, 0.8 * np.pi, seed=3)
    ctx.set_blocks(121, blocks)
    V = synth.port_rhs(Nx, Ny, b)
    I, info = ctx.solve(121, to_dev(V), tol=1e-10, inner_prec=inner, precond=4)
    assert info["status"] == abi.MLFFT_OK and np.all(info["relres"] <= 1e-10)
    assert relerr(to_host(I), direct.lu_solve(tp.dense_Z(blocks), V)) <= 1e-8


def test_row_preconditioner_takes_fewer_iterations_than_self_block(ctx):
    """Sec. V: P_Z includes the interactions along a row and converges in fewer iterations than
    P_K.  On a weakly loaded element (loading 1x, more iterations) per-column FP64 GMRES with
    P'_Z needs fewer iterations than with P'_K, in the split and in the global mode."""
    Nx, Ny, b = 8, 8, 16
    blocks = synth.green_blocks(Nx, Ny, b, np.pi, seed=0, alpha=1.0)
    ctx.set_blocks(122, blocks)
    V = to_dev(synth.port_rhs(Nx, Ny, b))
    its = {}
    for pc in (2, 4):
        for mode in (0, 1):
            _, info = ctx.solve(122, V, tol=1e-6, inner_prec="fp64", precond=pc, mode=mode)
            assert info["status"] == abi.MLFFT_OK
            its[pc, mode] = float(info["iters"].mean())
    print(f"\nmean iterations: P'_K split {its[2, 0]:.2f}, global {its[2, 1]:.2f}; "
          f"P'_Z split {its[4, 0]:.2f}, global {its[4, 1]:.2f}")
    assert its[4, 0] < its[2, 0] and its[4, 1] < its[2, 1]


# ----------------------------------------------------------------- block Rybicki

@pytest.mark.parametrize("Nx,Ny,b,kind", [(4, 4, 24, "green"), (3, 5, 8, "random"), (6, 6, 24, "green"),
                                          (5, 1, 6, "green"), (1, 6, 4, "random"), (9, 7, 10, "green")])
def test_direct_solve_matches_lu_and_oracle_recursion(ctx, Nx, Ny, b, kind):
    if kind == "green":
        blocks = synth.green_blocks(Nx, Ny, b, np.pi, seed=0)
    else:
        blocks = synth.random_blocks(Nx, Ny, b, seed=5)
        blocks[Ny - 1, Nx - 1] += 6 * np.sqrt(Nx * Ny * b) * np.eye(b)
    ctx.set_blocks(123, blocks)
    V = np.concatenate([synth.port_rhs(Nx, Ny, b), synth.random_vectors(Nx * Ny * b, 3, seed=1)])
    Vd = to_dev(V)
    I = torch.empty_like(Vd)
    ctx.sync_stream()
    rc, flops = abi.mlfft_direct_solve(ctx.h, 123, V.shape[0], Vd.data_ptr(), I.data_ptr())
    got = to_host(I)
    assert relerr(got, direct.lu_solve(tp.dense_Z(blocks), V)) <= 1e-10
    assert relerr(got, direct.rybicki_solve_array(blocks, V)) <= 1e-10
    assert 0 < rc <= 1 and flops > 0


def test_direct_solve_reports_a_singular_section(ctx):
    """R_0 is invertible but the order-1 section D = R_1 R_0^{-1} R_{-1} - R_0 vanishes: the
    recursion cannot continue (the oracle raises on the same blocks)."""
    b = 2
    A = np.array([[2.0, 0.5], [0.5, 1.0]], dtype=np.complex128)
    blocks = np.zeros((3, 1, b, b), dtype=np.complex128)          # Nx = 1, Ny = 2
    blocks[0, 0] = blocks[1, 0] = blocks[2, 0] = A
    with pytest.raises(direct.SingularSection):
        direct.rybicki_solve_array(blocks, np.ones((1, 2 * b)))
    ctx.set_blocks(124, blocks)
    Vd = to_dev(np.ones((1, 2 * b), np.complex128))
    I = torch.empty_like(Vd)
    ctx.sync_stream()
    with pytest.raises(abi.MlfftError) as e:
        abi.mlfft_direct_solve(ctx.h, 124, 1, Vd.data_ptr(), I.data_ptr())
    assert e.value.status == abi.MLFFT_E_SINGULAR and "order 1" in str(e.value)


def test_direct_solve_on_a_larger_array_matches_iterative_oracle(ctx):
    """14 x 12 array, b = 32 (level-1 blocks of order 448): all 168 port columns by the direct
    solver, sampled columns against the oracle's FP64 GMRES at 1e-12."""
    Nx, Ny, b = 14, 12, 32
    blocks = synth.green_blocks(Nx, Ny, b, 0.7 * np.pi, seed=4)
    ctx.set_blocks(125, blocks)
    V = synth.port_rhs(Nx, Ny, b)
    Vd = to_dev(V)
    I = torch.empty_like(Vd)
    ctx.sync_stream()
    abi.mlfft_direct_solve(ctx.h, 125, V.shape[0], Vd.data_ptr(), I.data_ptr())
    cols = [0, 13, 84, 167]
    from oracle import krylov
    Gh = tp.spectra(blocks, 2 * Ny, 2 * Nx)
    Sinv = opc.strang_inverse_spectrum(blocks)
    ref = np.array([r.x for r in krylov.gmres_columns(lambda X: tp.matvec_spectral(Gh, X, Nx, Ny), V[cols],
                                                       lambda X: opc.strang_apply(Sinv, X), tol=1e-12)])
    assert relerr(to_host(I)[cols], ref) <= 1e-10
    # and its residual through the library's own FP64 MLFFT product
    r = torch.empty_like(Vd)
    ctx.sync_stream()
    abi.mlfft_matvec_axpby(ctx.h, 125, V.shape[0], -1.0, I.data_ptr(), 1.0, Vd.data_ptr(), r.data_ptr(),
                           abi.MLFFT_FP64)
    assert np.max(np.linalg.norm(to_host(r), axis=1) / np.linalg.norm(V, axis=1)) <= 1e-12
