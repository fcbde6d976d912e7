"""GPU parity of the spectrum diagnostics (Sec. V): singular values of P^{-1} Z by the randomized
range finder through the MLFFT matvec, against the dense SVD (full sketches of small arrays) and
against the oracle's range finder with the same test matrix.

Bars: 1e-9 of the largest singular value (the eigenvalues come from a Cholesky of the sketch's
Gram matrix, which squares its condition number).
"""
import numpy as np
import pytest
import torch

from oracle import border, precond, spectrum
from oracle import toeplitz as tp
from paper_2506_20350_amd import abi, synth
from tests.gpu_util import ctx, to_dev  # noqa: F401

pytestmark = pytest.mark.gpu


def dense_pinv_z(blocks, kind, ZB=None, ZC=None):
    Nx, Ny, b = tp.shape_of(blocks)
    N = Nx * Ny * b
    if ZB is None:
        Z = tp.dense_Z(blocks)
        if kind == 0:
            return Z
        if kind == 1:
            return precond.strang_apply(precond.strang_inverse_spectrum(blocks), Z.T).T
        if kind == 2:
            return precond.kindt_apply(blocks, Z.T).T
        return precond.row_apply(blocks, Z.T).T
    Z = border.dense(blocks, ZB, ZC)
    return Z if kind == 0 else border.px_apply(kind, blocks, ZC, Z.T).T


def omega(n, l, seed):
    return synth.random_vectors(n, l, seed=seed)


@pytest.mark.parametrize("kind", [0, 1, 2, 4])
def test_full_sketch_equals_dense_svd(ctx, kind):
    Nx, Ny, b = 3, 4, 4
    blocks = synth.green_blocks(Nx, Ny, b, np.pi, seed=1, alpha=1.0)
    ctx.set_blocks(140, blocks)
    N = Nx * Ny * b
    sv = ctx.spectrum(140, to_dev(omega(N, N, seed=2)), kind, 1)
    ref = np.linalg.svd(dense_pinv_z(blocks, kind), compute_uv=False)
    assert np.max(np.abs(sv - ref)) <= 1e-9 * ref[0]


@pytest.mark.parametrize("kind,q", [(0, 0), (1, 1), (4, 2)])
def test_partial_sketch_matches_oracle_range_finder(ctx, kind, q):
    Nx, Ny, b = 8, 8, 16
    blocks = synth.green_blocks(Nx, Ny, b, 0.8 * np.pi, seed=3, alpha=1.0)
    ctx.set_blocks(141, blocks)
    N, l = Nx * Ny * b, 40
    Om = omega(N, l, seed=4)
    Gh = tp.spectra(blocks, 2 * Ny, 2 * Nx)
    Z = lambda X: tp.matvec_spectral(Gh, X, Nx, Ny)
    if kind == 0:
        P = lambda X: X
    elif kind == 1:
        Sinv = precond.strang_inverse_spectrum(blocks)
        P = lambda X: precond.strang_apply(Sinv, X)
    else:
        P = lambda X: precond.row_apply(blocks, X)
    A = lambda X: P(Z(X))
    # adjoint of the dense operator, assembled once (the oracle does not assume symmetry)
    Ad = A(np.eye(N)).T
    AH = lambda X: X @ Ad.conj()
    ref = spectrum.randomized_singular_values(A, AH, Om, q)
    sv = ctx.spectrum(141, to_dev(Om), kind, q)
    assert np.max(np.abs(sv - ref)) <= 1e-9 * ref[0]


@pytest.mark.parametrize("kind", [0, 1, 2])
def test_full_sketch_with_border_equals_dense_svd(ctx, kind):
    """(The test matrix is held by the caller while the library allocates its workspaces from the
    same PyTorch pool: a temporary freed at the call would hand its memory to the sketch.)"""
    Nx, Ny, b = 3, 3, 4
    blocks = synth.green_blocks(Nx, Ny, b, np.pi, seed=5)
    ZB, ZC = synth.border_blocks(Nx, Ny, b, np.pi, seed=5)
    ctx.set_blocks(142, blocks)
    ctx.set_border(142, ZB, ZC)
    n = Nx * Ny * b + ZC.shape[0]
    sv = ctx.spectrum(142, to_dev(omega(n, n, seed=6)), kind, 1)
    ref = np.linalg.svd(dense_pinv_z(blocks, kind, ZB, ZC), compute_uv=False)
    assert np.max(np.abs(sv - ref)) <= 1e-9 * ref[0]


def test_rank_deficient_sketch_is_reported(ctx):
    Nx, Ny, b = 3, 3, 4
    ctx.set_blocks(143, synth.green_blocks(Nx, Ny, b, np.pi, seed=7))
    Om = omega(Nx * Ny * b, 5, seed=8)
    Om[2] = 0.0
    with pytest.raises(abi.MlfftError) as e:
        ctx.spectrum(143, to_dev(Om), 1, 0)
    assert e.value.status == abi.MLFFT_E_SINGULAR
