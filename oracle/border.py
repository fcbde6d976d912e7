"""The full impedance matrix with border blocks (Sec. I, eq. Zblock; Sec. III-E).

Oracle (test infrastructure only).  Z = [[Z_A, Z_B^T], [Z_B, Z_C]] with Z_A the
two-level block-Toeplitz part (unique blocks in the library layout), Z_B the
coupling of the Nc border unknowns with the array (Nc x N) and Z_C the border
self interaction (Nc x Nc).  Vectors are [x_A (N, paper order), x_C (Nc)],
one per row of a (W, N + Nc) array.
"""
from __future__ import annotations

import numpy as np

from . import direct, precond
from . import toeplitz as tp


def dense(blocks: np.ndarray, ZB: np.ndarray, ZC: np.ndarray) -> np.ndarray:
    """Z assembled from its four parts (eq. Zblock)."""
    ZA = tp.dense_Z(blocks)
    return np.block([[ZA, ZB.T], [ZB, ZC]])


def matvec(blocks: np.ndarray, ZB: np.ndarray, ZC: np.ndarray, X: np.ndarray) -> np.ndarray:
    """y = Z x blockwise (eq. ZIVblock): y_A = Z_A x_A + Z_B^T x_C with the FFT product of
    eq. multL for Z_A, y_C = Z_B x_A + Z_C x_C by plain products."""
    Nx, Ny, b = tp.shape_of(blocks)
    N = Nx * Ny * b
    XA, XC = X[:, :N], X[:, N:]
    YA = tp.matvec_fft(blocks, XA, 2 * Ny, 2 * Nx) + XC @ ZB
    YC = XA @ ZB.T + XC @ ZC.T
    return np.concatenate([YA, YC], axis=1)


def schur_solve(blocks: np.ndarray, ZB: np.ndarray, ZC: np.ndarray, V: np.ndarray) -> np.ndarray:
    """Z I = V with the border moved to the right-hand side (Sec. III-E): solve
    Z_A [U F] = [V_A Z_B^T] by the block Rybicki recursion, then
    I_C = (Z_C - Z_B F)^{-1} (V_C - Z_B U) and I_A = U - F I_C."""
    Nx, Ny, b = tp.shape_of(blocks)
    N = Nx * Ny * b
    VA, VC = V[:, :N], V[:, N:]
    W = V.shape[0]
    rhs = np.concatenate([VA, ZB], axis=0)          # rows: the W columns of V_A, then the Nc of Z_B^T
    UF = direct.rybicki_solve_array(blocks, rhs)
    U, F = UF[:W].T, UF[W:].T                         # N x W and N x Nc
    S = ZC - ZB @ F
    IC = np.linalg.solve(S, VC.T - ZB @ U)
    IA = U - F @ IC
    return np.concatenate([IA.T, IC.T], axis=1)


def px_apply(kind: int, blocks: np.ndarray, ZC: np.ndarray, R: np.ndarray) -> np.ndarray:
    """P_X^{-1} r with P_X = blockdiag(P'_X, Z_C) (Sec. III-B): the array part by the
    preconditioner `kind` (1 block circulant, 2 P'_K, 4 P'_Z), the border part by a solve
    with Z_C (its LU)."""
    Nx, Ny, b = tp.shape_of(blocks)
    N = Nx * Ny * b
    RA, RC = R[:, :N], R[:, N:]
    if kind == 1:
        ZA = precond.strang_apply(precond.strang_inverse_spectrum(blocks), RA)
    elif kind == 2:
        ZA = precond.kindt_apply(blocks, RA)
    elif kind == 4:
        ZA = precond.row_apply(blocks, RA)
    else:
        raise ValueError("kind must be 1, 2 or 4")
    ZCr = np.linalg.solve(ZC, RC.T).T
    return np.concatenate([ZA, ZCr], axis=1)
