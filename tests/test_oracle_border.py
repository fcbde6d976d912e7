"""Pins of the oracle's border-block parts (CPU only): eq. Zblock, eq. ZIVblock, Sec. III-E."""
import numpy as np
import pytest

from oracle import border, direct, precond
from oracle import toeplitz as tp
from paper_2506_20350_amd import synth


def relerr(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("Nx,Ny,b", [(3, 2, 4), (4, 4, 6), (1, 3, 5)])
def test_border_generator_is_reciprocal(Nx, Ny, b):
    blocks = synth.green_blocks(Nx, Ny, b, np.pi, seed=1)
    ZB, ZC = synth.border_blocks(Nx, Ny, b, np.pi, seed=1)
    assert ZB.shape == (2 * (Nx + Ny), Nx * Ny * b) and ZC.shape == (2 * (Nx + Ny),) * 2
    Z = border.dense(blocks, ZB, ZC)
    assert np.max(np.abs(Z - Z.T)) <= 1e-13 * np.max(np.abs(Z))


@pytest.mark.parametrize("Nx,Ny,b,W", [(3, 2, 4, 2), (4, 5, 3, 3), (2, 1, 7, 1)])
def test_blockwise_matvec_equals_dense(Nx, Ny, b, W):
    blocks = synth.green_blocks(Nx, Ny, b, 0.7 * np.pi, seed=2)
    ZB, ZC = synth.border_blocks(Nx, Ny, b, 0.7 * np.pi, seed=2, per_cell=2)
    X = synth.random_vectors(Nx * Ny * b + ZC.shape[0], W, seed=3)
    ref = X @ border.dense(blocks, ZB, ZC).T
    assert relerr(border.matvec(blocks, ZB, ZC, X), ref) <= 1e-13


@pytest.mark.parametrize("Nx,Ny,b", [(4, 4, 6), (3, 5, 4), (5, 1, 3)])
def test_schur_solve_equals_lu_of_the_full_matrix(Nx, Ny, b):
    blocks = synth.green_blocks(Nx, Ny, b, np.pi, seed=0)
    ZB, ZC = synth.border_blocks(Nx, Ny, b, np.pi, seed=0)
    N = Nx * Ny * b
    V = np.concatenate([synth.port_rhs(Nx, Ny, b), np.zeros((Nx * Ny, ZC.shape[0]))], axis=1)
    V = np.concatenate([V, synth.random_vectors(N + ZC.shape[0], 2, seed=4)])
    I = border.schur_solve(blocks, ZB, ZC, V)
    ref = direct.lu_solve(border.dense(blocks, ZB, ZC), V)
    assert relerr(I, ref) <= 1e-10


def test_schur_solve_without_border_coupling_splits_into_two_solves():
    Nx, Ny, b = 3, 3, 4
    blocks = synth.green_blocks(Nx, Ny, b, np.pi, seed=5)
    _, ZC = synth.border_blocks(Nx, Ny, b, np.pi, seed=5)
    ZB = np.zeros((ZC.shape[0], Nx * Ny * b), np.complex128)
    V = synth.random_vectors(Nx * Ny * b + ZC.shape[0], 2, seed=6)
    I = border.schur_solve(blocks, ZB, ZC, V)
    N = Nx * Ny * b
    assert relerr(I[:, :N], direct.lu_solve(tp.dense_Z(blocks), V[:, :N])) <= 1e-12
    assert relerr(I[:, N:], np.linalg.solve(ZC, V[:, N:].T).T) <= 1e-12


@pytest.mark.parametrize("kind", [1, 2, 4])
def test_px_apply_inverts_the_dense_block_diagonal(kind):
    Nx, Ny, b = 4, 3, 3
    blocks = synth.green_blocks(Nx, Ny, b, np.pi, seed=7)
    _, ZC = synth.border_blocks(Nx, Ny, b, np.pi, seed=7)
    N = Nx * Ny * b
    if kind == 1:
        PA = precond.strang_dense(blocks)
    elif kind == 2:
        PA = np.kron(np.eye(Nx * Ny), tp.block(blocks, 0, 0))
    else:
        PA = np.kron(np.eye(Ny), tp.level1_blocks(blocks)[0])
    P = np.block([[PA, np.zeros((N, ZC.shape[0]))], [np.zeros((ZC.shape[0], N)), ZC]])
    R = synth.random_vectors(N + ZC.shape[0], 2, seed=8)
    z = border.px_apply(kind, blocks, ZC, R)
    assert relerr(z @ P.T, R) <= 1e-12
