"""Pins of the oracle's embedding, blockwise DFTs and matvecs (CPU only).

Each test fixes the oracle to something outside itself: the paper's printed
worked example, the Kronecker definition of the blockwise DFT, brute-force
dense products, reciprocity and scipy's scalar Toeplitz routines.
"""
import os

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import toeplitz as tp
from paper_2506_20350_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def read_sections(path):
    sec, cur = {}, None
    for line in open(path):
        line = line.strip()
        if line.startswith("# section:"):
            cur = line.split(":", 1)[1].strip()
            sec[cur] = []
        elif line and not line.startswith("#"):
            sec[cur].append([int(v) for v in line.split()])
    return {k: np.array(v) for k, v in sec.items()}


def lag_values():
    # distinct integers per lag so that every entry names its lag exactly
    return {j: 100 + 7 * j for j in range(-4, 5)}


def test_worked_example_circulant_matches_paper():
    g = read_sections(os.path.join(GOLDEN, "circulant_n3.txt"))
    t = lag_values()
    inv = {v: k for k, v in t.items()}
    c1 = tp.circulant_first_column(t, 3)
    assert [inv[v] for v in c1] == list(g["c1"][0])
    C = tp.circulant(c1)
    lagsC = np.vectorize(inv.get)(C.astype(int))
    np.testing.assert_array_equal(lagsC, g["C"])
    T = tp.toeplitz_from_lags(t, 3)
    np.testing.assert_array_equal(np.vectorize(inv.get)(T), g["T"])
    np.testing.assert_array_equal(np.vectorize(inv.get)(C[3:, 3:].astype(int)), g["Tprime"])


@pytest.mark.parametrize("n,P", [(3, 5), (3, 6), (4, 8), (5, 16), (6, 11)])
def test_circulant_embedding_product(n, P):
    rng = np.random.default_rng(n * 31 + P)
    t = {j: complex(rng.standard_normal(), rng.standard_normal()) for j in range(-(n - 1), n)}
    T = tp.toeplitz_from_lags(t, n)
    C = tp.circulant(tp.circulant_first_column(t, n, P))
    np.testing.assert_array_equal(C[:n, :n], T)
    u = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    up = np.concatenate([u, np.zeros(P - n)])
    v = C @ up                                      # eq. circmult
    np.testing.assert_allclose(v[:n], T @ u, rtol=0, atol=1e-13)
    np.testing.assert_allclose(tp.circulant_matvec_dft(C[:, 0], up)[:n], T @ u, rtol=0, atol=1e-12)


def test_circulant_embedding_rejects_short_grid():
    with pytest.raises(ValueError):
        tp.circulant_first_column({0: 1, 1: 2, -1: 3}, 2, P=2)


@pytest.mark.parametrize("N2,N1,N0,W", [(2, 3, 2, 2), (4, 5, 3, 1), (3, 2, 4, 3), (1, 4, 2, 1)])
def test_multilevel_dft_is_kronecker_product(N2, N1, N0, W):
    rng = np.random.default_rng(N2 * 100 + N1 * 10 + N0)
    x = rng.standard_normal((N2 * N1 * N0, W)) + 1j * rng.standard_normal((N2 * N1 * N0, W))
    F2 = tp.kron_dft(N2, N1, N0)
    np.testing.assert_allclose(tp.multilevel_dft(x, N2, N1, N0), F2 @ x, rtol=0, atol=1e-12)
    F2i = tp.kron_dft(N2, N1, N0, inverse=True)
    np.testing.assert_allclose(tp.multilevel_dft(x, N2, N1, N0, inverse=True), F2i @ x, rtol=0, atol=1e-13)
    # the 2-level blockwise DFT equals a 2-D DFT over the two grid axes
    xg = x.reshape(N2, N1, N0, W)
    np.testing.assert_allclose(tp.multilevel_dft(x, N2, N1, N0).reshape(N2, N1, N0, W),
                               np.fft.fft2(xg, axes=(0, 1)), rtol=0, atol=1e-12)


@pytest.mark.parametrize("N1,N0", [(5, 3), (4, 1), (7, 2)])
def test_block_dft_1level_is_kronecker_product(N1, N0):
    rng = np.random.default_rng(N1 * 7 + N0)
    x = rng.standard_normal((N1 * N0, 2)) + 1j * rng.standard_normal((N1 * N0, 2))
    F1 = np.kron(tp.dft_matrix(N1), np.eye(N0))     # eq. F1
    np.testing.assert_allclose(tp.block_dft_1level(x, N0), F1 @ x, rtol=0, atol=1e-12)


SHAPES = [(1, 1, 3), (3, 1, 2), (1, 4, 2), (3, 2, 4), (4, 3, 5), (5, 5, 2), (2, 6, 3)]


@pytest.mark.parametrize("Nx,Ny,b", SHAPES)
def test_matvec_forms_agree_random_blocks(Nx, Ny, b):
    blocks = synth.random_blocks(Nx, Ny, b, seed=Nx * 100 + Ny * 10 + b)
    X = synth.random_vectors(Nx * Ny * b, 3, seed=7)
    Z = tp.dense_Z(blocks)
    yd = tp.matvec_dense(Z, X)
    scale = np.linalg.norm(yd)
    assert np.linalg.norm(tp.matvec_direct(blocks, X) - yd) <= 1e-13 * scale
    pairs = [(2 * Ny - 1, 2 * Nx - 1), (2 * Ny, 2 * Nx),
             (1 << (2 * Ny - 1).bit_length(), 1 << (2 * Nx - 1).bit_length()), (2 * Ny + 3, 2 * Nx + 1)]
    for Py, Px in pairs:
        assert np.linalg.norm(tp.matvec_fft(blocks, X, Py, Px) - yd) <= 1e-12 * scale, (Py, Px)
    assert np.linalg.norm(tp.matvec_mlfft_paper(blocks, X) - yd) <= 1e-12 * scale
    assert np.linalg.norm(tp.matvec_mlfft_paper(blocks, X, 2 * Ny, 2 * Nx) - yd) <= 1e-12 * scale


def test_dense_assembly_index_convention():
    # test cell (iy,ix) <- source cell (iy-p, ix-q) carries R_{p,q}
    Nx, Ny, b = 3, 2, 2
    blocks = synth.random_blocks(Nx, Ny, b, seed=3)
    Z = tp.dense_Z(blocks)
    iy, ix, jy, jx = 1, 0, 0, 2
    blk = Z[(iy * Nx + ix) * b:(iy * Nx + ix + 1) * b, (jy * Nx + jx) * b:(jy * Nx + jx + 1) * b]
    np.testing.assert_array_equal(blk, blocks[(iy - jy) + Ny - 1, (ix - jx) + Nx - 1])


def test_single_cell_reduces_to_self_block():
    blocks = synth.green_blocks(1, 1, 5, kd=np.pi, seed=2)
    np.testing.assert_array_equal(tp.dense_Z(blocks), blocks[0, 0])


@pytest.mark.parametrize("Nx", [1, 2, 5, 8])
def test_scalar_one_level_matches_scipy_toeplitz(Nx):
    rng = np.random.default_rng(Nx)
    blocks = (rng.standard_normal((1, 2 * Nx - 1, 1, 1)) + 1j * rng.standard_normal((1, 2 * Nx - 1, 1, 1)))
    col = blocks[0, Nx - 1:, 0, 0]                  # t_0 .. t_{Nx-1}
    row = blocks[0, Nx - 1::-1, 0, 0]               # t_0, t_{-1}, ..., t_{-(Nx-1)}
    np.testing.assert_array_equal(tp.dense_Z(blocks), sla.toeplitz(col, row))
    x = rng.standard_normal(Nx) + 1j * rng.standard_normal(Nx)
    ref = sla.matmul_toeplitz((col, row), x)
    got = tp.matvec_fft(blocks, x[None, :])[0]
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12 * np.linalg.norm(ref))


@pytest.mark.parametrize("Nx,Ny,b,kd", [(3, 2, 4, np.pi), (4, 4, 6, 2 * np.pi / 3), (2, 5, 3, np.pi / 2)])
def test_reciprocity_of_green_blocks(Nx, Ny, b, kd):
    blocks = synth.green_blocks(Nx, Ny, b, kd, seed=1)
    for p in range(-(Ny - 1), Ny):
        for q in range(-(Nx - 1), Nx):
            np.testing.assert_array_equal(tp.block(blocks, p, q), tp.block(blocks, -p, -q).T)
    Z = tp.dense_Z(blocks)
    np.testing.assert_array_equal(Z, Z.T)
    Py, Px = 2 * Ny, 2 * Nx
    Gh = tp.spectra(blocks, Py, Px)
    for ky in range(Py):
        for kx in range(Px):
            a = Gh[ky, kx]
            bt = Gh[(-ky) % Py, (-kx) % Px].T
            assert np.abs(a - bt).max() <= 1e-13 * np.abs(Gh).max()


def test_green_blocks_self_term_and_loading():
    b, kd = 6, np.pi
    blocks = synth.green_blocks(3, 3, b, kd, seed=4, alpha=0.0)
    lam = 2 * np.pi / kd
    a = 0.02 * lam
    d = np.diag(blocks[2, 2])
    ref = np.exp(-1j * kd * a) / (4 * np.pi * a)    # u_m . u_m = 1
    np.testing.assert_allclose(d, ref, rtol=1e-14)
    loaded = synth.green_blocks(3, 3, b, kd, seed=4, alpha=10.0)
    off = np.abs(blocks).copy()
    off[2, 2][np.diag_indices(b)] = 0
    np.testing.assert_allclose(np.diag(loaded[2, 2]) - d, 10.0 * off.max(), rtol=1e-14)
