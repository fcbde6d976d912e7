"""Pins of the oracle's randomized singular values (CPU only)."""
import numpy as np

from oracle import precond, spectrum
from oracle import toeplitz as tp
from paper_2506_20350_amd import synth


def crand(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def test_exact_for_a_matrix_of_rank_at_most_l():
    """A matrix of rank r <= l has its range captured exactly: the r singular values are exact."""
    rng = np.random.default_rng(0)
    n, r, l = 60, 7, 10
    M = crand(rng, n, r) @ crand(rng, r, n)
    A = lambda X: X @ M.T
    AH = lambda X: X @ M.conj()
    sv = spectrum.randomized_singular_values(A, AH, crand(rng, l, n))
    ref = np.linalg.svd(M, compute_uv=False)
    np.testing.assert_allclose(sv[:r], ref[:r], rtol=1e-10)
    assert np.all(sv[r:] <= 1e-10 * ref[0])


def test_full_sketch_gives_every_singular_value_of_the_preconditioned_array():
    """With l = N the sketch spans everything: all singular values of P^{-1} Z (block circulant P)."""
    Nx, Ny, b = 3, 3, 4
    blocks = synth.green_blocks(Nx, Ny, b, np.pi, seed=0, alpha=1.0)
    N = Nx * Ny * b
    Sinv = precond.strang_inverse_spectrum(blocks)
    Z = tp.dense_Z(blocks)
    A = lambda X: precond.strang_apply(Sinv, X @ Z.T)
    PinvZ = A(np.eye(N)).T                      # column j = P^{-1} Z e_j
    AH = lambda X: X @ PinvZ.conj()
    sv = spectrum.randomized_singular_values(A, AH, crand(np.random.default_rng(1), N, N), power_iters=1)
    np.testing.assert_allclose(sv, np.linalg.svd(PinvZ, compute_uv=False), rtol=1e-9)


def test_power_iterations_sharpen_the_leading_values():
    """Halko et al.: power steps raise the accuracy of the leading singular values on a slowly
    decaying spectrum; with one step the error of the largest falls well below the plain sketch's."""
    rng = np.random.default_rng(2)
    n, l = 200, 12
    U, _ = np.linalg.qr(crand(rng, n, n))
    V, _ = np.linalg.qr(crand(rng, n, n))
    s = 1.0 / np.arange(1, n + 1) ** 0.5
    M = (U * s) @ V.conj().T
    A = lambda X: X @ M.T
    AH = lambda X: X @ M.conj()
    Om = crand(rng, l, n)
    e0 = abs(spectrum.randomized_singular_values(A, AH, Om, 0)[0] - s[0])
    e2 = abs(spectrum.randomized_singular_values(A, AH, Om, 2)[0] - s[0])
    assert e2 < 0.2 * e0
