"""Preconditioners for the MLFFT-accelerated iterative solve.

Oracle (test infrastructure only).

* Kindt self-block preconditioner P'_K (Sec. III-B): block diagonal with
  every diagonal block equal to the element self block R_{0,0}.
* Row preconditioner P'_Z (Sec. III-B): block diagonal with every diagonal
  block equal to the self interaction of one array row, T^[1]_0.
* Two-level block-circulant preconditioner (a reading; the paper asks for a
  preconditioner that covers all neighbouring elements, Sec. V, but does not
  define one).  The reading: the two-level Strang block circulant on the
  Ny x Nx torus.  Its first block column is S[py][qx] = R_{p,q}, with
  p = py if 2 py < Ny and p = py - Ny if 2 py > Ny (likewise for q); when
  2 py = Ny both lags +-Ny/2 exist and their blocks are averaged (and the four
  corner candidates when both axes sit at Ny/2, Nx/2).  The averaging keeps S
  complex symmetric, like Z_A.  S is diagonalised by the 2-D DFT on the
  Ny x Nx grid (eq. toeplitzmult in block form), so
  P^{-1} r = IFFT2( S_hat(k)^{-1} FFT2(r) ), one b x b inverse per frequency.
"""
from __future__ import annotations

import numpy as np

from .toeplitz import block, level1_blocks, shape_of


def strang_lag_weights(N: int) -> dict:
    """Lag -> weight of the Strang fold on an N-periodic axis.

    Lags |p| < N/2 keep weight 1; for even N the two lags +-N/2 share the
    position N/2 with weight 1/2 each.
    """
    w = {}
    for p in range(-(N - 1), N):
        if 2 * abs(p) < N:
            w[p] = 1.0
        elif 2 * abs(p) == N:
            w[p] = 0.5
    return w


def strang_blocks(blocks: np.ndarray) -> np.ndarray:
    """First block column of the two-level Strang block circulant, shape (Ny, Nx, b, b)."""
    Nx, Ny, b = shape_of(blocks)
    wy = strang_lag_weights(Ny)
    wx = strang_lag_weights(Nx)
    S = np.zeros((Ny, Nx, b, b), dtype=np.complex128)
    for p, cy in wy.items():
        for q, cx in wx.items():
            S[p % Ny, q % Nx] += cy * cx * block(blocks, p, q)
    return S


def strang_spectrum(blocks: np.ndarray) -> np.ndarray:
    """S_hat(ky, kx): 2-D DFT of the Strang first block column over its grid axes."""
    return np.fft.fft2(strang_blocks(blocks), axes=(0, 1))


def strang_inverse_spectrum(blocks: np.ndarray) -> np.ndarray:
    """S_hat(k)^{-1} for every frequency, shape (Ny, Nx, b, b)."""
    Sh = strang_spectrum(blocks)
    return np.linalg.inv(Sh)


def strang_apply(Sinv_hat: np.ndarray, Rv: np.ndarray) -> np.ndarray:
    """z = IFFT2(S_hat^{-1} FFT2(r)) for every column; Rv has shape (W, N)."""
    Ny, Nx, b, _ = Sinv_hat.shape
    W = Rv.shape[0]
    r = Rv.reshape(W, Ny, Nx, b)
    rh = np.fft.fft2(r, axes=(1, 2))
    zh = np.einsum('yxmn,wyxn->wyxm', Sinv_hat, rh)
    return np.fft.ifft2(zh, axes=(1, 2)).reshape(W, -1)


def strang_dense(blocks: np.ndarray) -> np.ndarray:
    """The Strang block circulant as an explicit N x N matrix (for tests)."""
    Nx, Ny, b = shape_of(blocks)
    S = strang_blocks(blocks)
    N = Nx * Ny * b
    P = np.empty((N, N), dtype=np.complex128)
    for iy in range(Ny):
        for ix in range(Nx):
            for jy in range(Ny):
                for jx in range(Nx):
                    P[(iy * Nx + ix) * b:(iy * Nx + ix + 1) * b,
                      (jy * Nx + jx) * b:(jy * Nx + jx + 1) * b] = S[(iy - jy) % Ny, (ix - jx) % Nx]
    return P


def kindt_apply(blocks: np.ndarray, Rv: np.ndarray) -> np.ndarray:
    """P'_K^{-1} r: solve with the self block R_{0,0} in every cell (Sec. III-B)."""
    Nx, Ny, b = shape_of(blocks)
    W = Rv.shape[0]
    r = Rv.reshape(W * Nx * Ny, b)
    z = np.linalg.solve(block(blocks, 0, 0), r.T).T
    return z.reshape(W, -1)


def row_apply(blocks: np.ndarray, Rv: np.ndarray) -> np.ndarray:
    """P'_Z^{-1} r: solve with the row self interaction T^[1]_0 in every row (Sec. III-B)."""
    Nx, Ny, b = shape_of(blocks)
    T0 = level1_blocks(blocks)[0]
    W = Rv.shape[0]
    r = Rv.reshape(W * Ny, Nx * b)
    z = np.linalg.solve(T0, r.T).T
    return z.reshape(W, -1)
