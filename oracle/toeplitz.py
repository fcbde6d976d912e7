"""Two-level block-Toeplitz Z_A, its circulant embedding and the MLFFT product.

Oracle (test infrastructure only).  Notation: Nx = N^[1] columns, Ny = N^[2]
rows, b = N^[0] basis functions per cell (Sec. II-A).  Unknown order inside a
column is ((iy*Nx)+ix)*b + m (Sec. II-C, eq. xc2: the vector is split into Ny
row sub-vectors of length Nx*b).  Blocks are stored as
blocks[p + Ny - 1, q + Nx - 1] = R_{p,q}, the coupling of a test cell
(iy, ix) with the source cell (iy - p, ix - q), following T_ij = t_{i-j}
(eq. T, eq. Tblock).  Right-hand sides are stored as rows of an array of
shape (W, N): X[w] is column w of the paper's matrix (vec of I_M, eq. ZIVvec).
"""
from __future__ import annotations

import numpy as np


# ---------------------------------------------------------------- scalar case

def toeplitz_from_lags(t: dict, n: int) -> np.ndarray:
    """n x n Toeplitz matrix with T[i, j] = t[i - j] (eq. T)."""
    T = np.empty((n, n), dtype=np.result_type(*[np.asarray(v) for v in t.values()]))
    for i in range(n):
        for j in range(n):
            T[i, j] = t[i - j]
    return T


def circulant_first_column(t: dict, n: int, P: int | None = None) -> np.ndarray:
    """First column c_1 of the circulant C(T) embedding an n x n Toeplitz T (eq. cT1).

    The column is [t_0, t_1, ..., t_{n-1}, t_{-(n-1)}, ..., t_{-1}]: the first
    column of T followed by its first row without the leading entry, in
    reverse order.  For P > 2n-1 zeros are inserted between the two parts,
    which keeps C(T)[:n, :n] = T (any P >= 2n-1 works).
    """
    if P is None:
        P = 2 * n - 1
    if P < 2 * n - 1:
        raise ValueError("circulant size must be at least 2n-1")
    c = np.zeros(P, dtype=np.result_type(*[np.asarray(v) for v in t.values()]))
    for j in range(n):
        c[j] = t[j]
    for j in range(1, n):
        c[P - j] = t[-j]
    return c


def circulant(c1: np.ndarray) -> np.ndarray:
    """Circulant matrix with first column c1: C[i, j] = c1[(i - j) mod P]."""
    P = len(c1)
    C = np.empty((P, P), dtype=c1.dtype)
    for i in range(P):
        for j in range(P):
            C[i, j] = c1[(i - j) % P]
    return C


def circulant_matvec_dft(c1: np.ndarray, u: np.ndarray) -> np.ndarray:
    """C u = F^{-1} diag(F c_1) F u (eq. toeplitzmult), with numpy's DFT."""
    return np.fft.ifft(np.fft.fft(c1) * np.fft.fft(u))


# ------------------------------------------------------------ block assembly

def shape_of(blocks: np.ndarray):
    """(Nx, Ny, b) of a block array of shape (2Ny-1, 2Nx-1, b, b)."""
    py, qx, b, b2 = blocks.shape
    if b != b2 or py % 2 == 0 or qx % 2 == 0:
        raise ValueError("blocks must have shape (2Ny-1, 2Nx-1, b, b)")
    return (qx + 1) // 2, (py + 1) // 2, b


def block(blocks: np.ndarray, p: int, q: int) -> np.ndarray:
    Nx, Ny, _ = shape_of(blocks)
    return blocks[p + Ny - 1, q + Nx - 1]


def dense_Z(blocks: np.ndarray) -> np.ndarray:
    """Full N x N Z_A (eq. Tblock with L = 2).

    Z[(iy*Nx+ix)*b + m, (jy*Nx+jx)*b + n] = R_{iy-jy, ix-jx}[m, n]: level 2
    (rows of the array) is the outer block-Toeplitz level with blocks
    T^[1]_{iy-jy}, each of which is a level-1 block-Toeplitz matrix over the
    columns with b x b blocks.
    """
    Nx, Ny, b = shape_of(blocks)
    N = Nx * Ny * b
    Z = np.empty((N, N), dtype=blocks.dtype)
    for iy in range(Ny):
        for ix in range(Nx):
            r0 = (iy * Nx + ix) * b
            for jy in range(Ny):
                for jx in range(Nx):
                    c0 = (jy * Nx + jx) * b
                    Z[r0:r0 + b, c0:c0 + b] = block(blocks, iy - jy, ix - jx)
    return Z


def level1_blocks(blocks: np.ndarray) -> dict:
    """Dense level-1 blocks T^[1]_p (Nx*b x Nx*b) for p in (-Ny, Ny).

    T^[1]_p[ix*b + m, jx*b + n] = R_{p, ix-jx}[m, n]; these are the blocks the
    Rybicki recursion works with ("fill in the lowest Toeplitz level", Sec. IV).
    """
    Nx, Ny, b = shape_of(blocks)
    out = {}
    for p in range(-(Ny - 1), Ny):
        T = np.empty((Nx * b, Nx * b), dtype=blocks.dtype)
        for ix in range(Nx):
            for jx in range(Nx):
                T[ix * b:(ix + 1) * b, jx * b:(jx + 1) * b] = block(blocks, p, ix - jx)
        out[p] = T
    return out


# ------------------------------------------------------------------ matvecs

def matvec_dense(Z: np.ndarray, X: np.ndarray) -> np.ndarray:
    """Y[w] = Z X[w] for every column w."""
    return (Z @ X.T).T


def matvec_direct(blocks: np.ndarray, X: np.ndarray) -> np.ndarray:
    """Direct block convolution y(iy,ix) = sum_{jy,jx} R_{iy-jy, ix-jx} x(jy,jx)."""
    Nx, Ny, b = shape_of(blocks)
    W = X.shape[0]
    x = X.reshape(W, Ny, Nx, b)
    y = np.zeros_like(x, dtype=np.result_type(blocks, X))
    for iy in range(Ny):
        for ix in range(Nx):
            acc = np.zeros((W, b), dtype=y.dtype)
            for jy in range(Ny):
                for jx in range(Nx):
                    acc += x[:, jy, jx, :] @ block(blocks, iy - jy, ix - jx).T
            y[:, iy, ix, :] = acc
    return y.reshape(W, -1)


def block_grid(blocks: np.ndarray, Py: int, Px: int) -> np.ndarray:
    """Two-level block-circulant first block column on a Py x Px grid.

    G[p mod Py, q mod Px] = R_{p,q} and zero elsewhere: the 2-D form of the
    first column of eq. cT1, built level by level as in eqs. circL1 and circL2.
    Needs Py >= 2Ny-1 and Px >= 2Nx-1.
    """
    Nx, Ny, b = shape_of(blocks)
    if Py < 2 * Ny - 1 or Px < 2 * Nx - 1:
        raise ValueError("grid too small for the circulant embedding")
    G = np.zeros((Py, Px, b, b), dtype=blocks.dtype)
    for p in range(-(Ny - 1), Ny):
        for q in range(-(Nx - 1), Nx):
            G[p % Py, q % Px] = block(blocks, p, q)
    return G


def spectra(blocks: np.ndarray, Py: int, Px: int) -> np.ndarray:
    """Block spectrum G_hat(ky, kx) = 2-D DFT of the block grid over its two grid axes.

    This is diag_{N^[0]}(F^[2] C_1^[2]) of eq. multL, one b x b block per
    frequency; returned with shape (Py, Px, b, b).
    """
    return np.fft.fft2(block_grid(blocks, Py, Px), axes=(0, 1))


def matvec_spectral(Gh: np.ndarray, X: np.ndarray, Nx: int, Ny: int) -> np.ndarray:
    """Z_A X from precomputed block spectra Gh (Py, Px, b, b) of eq. multL.

    Zero-pad every column to the Py x Px grid (eq. xc2), 2-D DFT over the grid
    axes, one b x b product per frequency, inverse DFT, keep Ny x Nx cells.
    """
    Py, Px, b, _ = Gh.shape
    W = X.shape[0]
    u = np.zeros((W, Py, Px, b), dtype=np.result_type(Gh, X))
    u[:, :Ny, :Nx, :] = X.reshape(W, Ny, Nx, b)
    uh = np.fft.fft2(u, axes=(1, 2))
    vh = np.einsum('yxmn,wyxn->wyxm', Gh, uh)
    v = np.fft.ifft2(vh, axes=(1, 2))
    return v[:, :Ny, :Nx, :].reshape(W, -1)


def matvec_fft(blocks: np.ndarray, X: np.ndarray, Py: int | None = None,
               Px: int | None = None) -> np.ndarray:
    """Z_A X via the blockwise 2-level FFT (eq. multL, L = 2).

    Zero-pad every column from Ny x Nx cells to Py x Px (eq. xc2), transform
    over the two grid axes, multiply each frequency's b-vector by its b x b
    spectrum block, transform back (1/(Py*Px) normalisation, as MATLAB's ifft)
    and keep the first Ny x Nx cells.  Any Py >= 2Ny-1, Px >= 2Nx-1 gives the
    same product.
    """
    Nx, Ny, b = shape_of(blocks)
    Py = 2 * Ny - 1 if Py is None else Py
    Px = 2 * Nx - 1 if Px is None else Px
    return matvec_spectral(spectra(blocks, Py, Px), X, Nx, Ny)


# ----------------------------------------------- blockwise multilevel DFTs

def dft_matrix(n: int, inverse: bool = False) -> np.ndarray:
    """F_n[j, k] = exp(-2 pi i jk/n) (forward) or its inverse F_n^{-1}."""
    j = np.arange(n)
    if inverse:
        return np.exp(2j * np.pi * np.outer(j, j) / n) / n
    return np.exp(-2j * np.pi * np.outer(j, j) / n)


def kron_dft(N2: int, N1: int, N0: int, inverse: bool = False) -> np.ndarray:
    """F^[2] = F_{N2} (x) F_{N1} (x) I_{N0} as an explicit matrix (eqs. F1, F2)."""
    return np.kron(dft_matrix(N2, inverse), np.kron(dft_matrix(N1, inverse), np.eye(N0)))


def block_dft_1level(x: np.ndarray, N0: int, inverse: bool = False) -> np.ndarray:
    """Blockwise DFT of a column block vector (Sec. III-A, App. A).

    x has shape (N1*N0, W).  For every offset r inside a block, the rows
    r, r+N0, r+2N0, ... form one sequence, transformed along its length, in
    every column.  This equals (F_{N1} (x) I_{N0}) x.
    """
    f = np.fft.ifft if inverse else np.fft.fft
    out = np.array(x, dtype=np.complex128, copy=True)
    for r in range(N0):
        out[r::N0, :] = f(x[r::N0, :], axis=0)
    return out


def multilevel_dft(x: np.ndarray, N2: int, N1: int, N0: int, inverse: bool = False) -> np.ndarray:
    """Two-level blockwise DFT of a column block vector (Sec. III-A, App. B).

    x has shape (N2*N1*N0, W).  Lower level: inside each of the N2 upper
    blocks (length N1*N0), for each offset r < N0, the N1 rows at stride N0
    are transformed.  Upper level: for each offset s < N1*N0, the N2 rows at
    stride N1*N0 are transformed.  Equals (F_{N2} (x) F_{N1} (x) I_{N0}) x.
    """
    f = np.fft.ifft if inverse else np.fft.fft
    out = np.array(x, dtype=np.complex128, copy=True)
    upper = N1 * N0
    for blk in range(N2):
        base = blk * upper
        for r in range(N0):
            idx = base + r + N0 * np.arange(N1)
            out[idx, :] = f(out[idx, :], axis=0)
    for s in range(upper):
        idx = s + upper * np.arange(N2)
        out[idx, :] = f(out[idx, :], axis=0)
    return out


def pad_two_level(X: np.ndarray, Nx: int, Ny: int, b: int, Px: int, Py: int) -> np.ndarray:
    """Padded vector u^[2] of eq. xc2 (generalised to any Px, Py).

    Each row sub-vector u_iy (length Nx*b) is followed by (Px - Nx)*b zeros,
    and (Py - Ny)*Px*b zeros close the vector.  Returns shape (Py*Px*b, W).
    """
    W = X.shape[0]
    u = np.zeros((Py * Px * b, W), dtype=np.complex128)
    for iy in range(Ny):
        src = X[:, iy * Nx * b:(iy + 1) * Nx * b].T
        u[iy * Px * b: iy * Px * b + Nx * b, :] = src
    return u


def extract_two_level(v: np.ndarray, Nx: int, Ny: int, b: int, Px: int) -> np.ndarray:
    """Take v_iy from positions iy*Px*b + [0, Nx*b) of v^[2] (Sec. II-C); shape (W, N)."""
    parts = [v[iy * Px * b: iy * Px * b + Nx * b, :] for iy in range(Ny)]
    return np.concatenate(parts, axis=0).T


def block_first_column(blocks: np.ndarray, Py: int, Px: int) -> np.ndarray:
    """C_1^[2] (eq. circL2) as a (Py*Px*b, b) block column.

    Block (ky_pos*Px + kx_pos) of the column is R_{p,q} with p = ky_pos (or
    ky_pos - Py for the wrapped, negative lags), likewise for q (eq. circL1).
    """
    G = block_grid(blocks, Py, Px)
    _, _, b = shape_of(blocks)
    return G.reshape(Py * Px * b, b)


def matvec_mlfft_paper(blocks: np.ndarray, X: np.ndarray, Py: int | None = None,
                       Px: int | None = None) -> np.ndarray:
    """Z_A X in the paper's own vector form (eq. multL with L = 2).

    v^[2] = (F^[2])^{-1} diag_{N0}(F^[2] C_1^[2]) F^[2] u^[2], with u^[2] the
    padded vector of eq. xc2, F^[2] applied blockwise by multilevel_dft, and
    the product extracted from v^[2] row sub-vector by row sub-vector.
    """
    Nx, Ny, b = shape_of(blocks)
    Py = 2 * Ny - 1 if Py is None else Py
    Px = 2 * Nx - 1 if Px is None else Px
    C1 = block_first_column(blocks, Py, Px)                 # (K*b, b)
    D = multilevel_dft(C1, Py, Px, b)                       # F^[2] C_1^[2]
    u = pad_two_level(X, Nx, Ny, b, Px, Py)                 # (K*b, W)
    uh = multilevel_dft(u, Py, Px, b)
    K = Py * Px
    vh = np.empty_like(uh)
    for k in range(K):                                      # diag_{N0}(...) product
        vh[k * b:(k + 1) * b, :] = D[k * b:(k + 1) * b, :] @ uh[k * b:(k + 1) * b, :]
    v = multilevel_dft(vh, Py, Px, b, inverse=True)
    return extract_two_level(v, Nx, Ny, b, Px)
