"""Seeded synthetic inputs: unique cell-coupling blocks and port excitations.

This module is input synthesis only.  It holds none of the solver's
arithmetic (no circulant embedding, FFT, block product or Krylov step) and is
shared, unchanged, by the CPU oracle's tests and by the GPU path's tests and
benchmark.  It stands in for the MoM construction step that fills the unique
sub-matrices of the array impedance matrix (Sec. IV, simulation step 3), whose
meshes and MoM code are not available.

Element model (a stand-in for an RWG element mesh):
  * unit cell spacing d = 1, wavenumber k = kd, wavelength 2*pi/kd,
    regularisation radius a = 0.02 wavelengths;
  * basis centres r_m = (s_m0, s_m1, 0) with s ~ U[0,1)^(b x 2), then basis
    directions u_m = g_m / |g_m| with g ~ N(0,1)^(b x 3), both drawn from
    numpy.random.default_rng(seed) in that order;
  * block R_{p,q}[m, n] couples test basis m of cell (iy, ix) with source
    basis n of cell (iy - p, ix - q):
        R_{p,q}[m, n] = (u_m . u_n) exp(-j k rho) / (4 pi rho),
        rho = | r_m - r_n + (q d, p d, 0) |,
    with rho := a for the self terms (p, q) = (0, 0), m = n;
  * diagonal loading: the real value alpha * M is added to the diagonal of
    R_{0,0}, where M is the largest |entry| over all blocks except the self
    terms (alpha = 10 unless stated).

Layout of the returned blocks: complex128 array of shape
(2 Ny - 1, 2 Nx - 1, b, b), index [p + Ny - 1, q + Nx - 1, m, n].

The symmetric form of the kernel makes Z complex symmetric, so the blocks obey
R_{-p,-q} = R_{p,q}^T (reciprocity, Sec. I, eq. Zblock).
"""
from __future__ import annotations

import math

import numpy as np


def element(b: int, seed: int):
    """Basis centres (b, 3) and unit directions (b, 3) of one element."""
    rng = np.random.default_rng(seed)
    s = rng.random((b, 2))
    g = rng.standard_normal((b, 3))
    r = np.zeros((b, 3))
    r[:, 0] = s[:, 0]
    r[:, 1] = s[:, 1]
    u = g / np.linalg.norm(g, axis=1, keepdims=True)
    return r, u


def green_blocks(Nx: int, Ny: int, b: int, kd: float, seed: int = 0,
                 alpha: float = 10.0, dtype=np.complex128) -> np.ndarray:
    """All (2Ny-1)(2Nx-1) unique b x b blocks of the two-level block-Toeplitz Z_A."""
    if Nx < 1 or Ny < 1 or b < 1:
        raise ValueError("Nx, Ny and b must be positive")
    r, u = element(b, seed)
    k = float(kd)
    lam = 2.0 * math.pi / k
    a = 0.02 * lam
    udot = u @ u.T                                   # (b, b)
    dr = r[:, None, :] - r[None, :, :]               # (b, b, 3): r_m - r_n
    qs = np.arange(-(Nx - 1), Nx, dtype=np.float64)  # lags q
    out = np.empty((2 * Ny - 1, 2 * Nx - 1, b, b), dtype=dtype)
    maxoff = 0.0
    for ip, p in enumerate(range(-(Ny - 1), Ny)):
        dx = dr[None, :, :, 0] + qs[:, None, None]   # (2Nx-1, b, b)
        dy = dr[None, :, :, 1] + float(p)
        dz = dr[None, :, :, 2]
        rho = np.sqrt(dx * dx + dy * dy + dz * dz)
        if p == 0:
            iq0 = Nx - 1
            rho[iq0][np.diag_indices(b)] = a
        blk = udot[None] * np.exp(-1j * k * rho) / (4.0 * math.pi * rho)
        mag = np.abs(blk)
        if p == 0:
            mag[Nx - 1][np.diag_indices(b)] = 0.0
        maxoff = max(maxoff, float(mag.max()))
        out[ip] = blk
    out[Ny - 1, Nx - 1][np.diag_indices(b)] += alpha * maxoff
    return out


def border_blocks(Nx: int, Ny: int, b: int, kd: float, seed: int = 0, per_cell: int = 1,
                  alpha: float = 10.0) -> tuple:
    """Border blocks Z_B (Nc x N) and Z_C (Nc x Nc) of the same element model (Sec. I, eq. Zblock).

    The border stands in for the shared-edge region of a connected array that the
    partition of the paper's mesh leaves outside the Toeplitz part: Nc =
    2 per_cell (Nx + Ny) basis functions just outside the array's perimeter
    (per_cell along every cell edge of the four sides, at a quarter cell from
    the outline), with positions and directions drawn from
    numpy.random.default_rng(seed + 7919) (offset along the side uniform in the
    cell, then a N(0,1)^3 direction), coupled to the array bases (cell (iy, ix),
    basis m at r_m + (ix, iy, 0)) and to each other by the same kernel as
    green_blocks.  Z_C's self terms use rho = a and get the real loading alpha
    times its largest off-diagonal magnitude.  Returns row-major complex128
    arrays: Z_B[i, (iy Nx + ix) b + m] and Z_C[i, j].
    """
    r, u = element(b, seed)
    rng = np.random.default_rng(seed + 7919)
    pos = []
    for side in range(4):
        n_edge = Nx if side < 2 else Ny
        for c in range(n_edge):
            for _ in range(per_cell):
                t = c + rng.random()
                if side == 0:
                    pos.append((t, -0.25))
                elif side == 1:
                    pos.append((t, Ny + 0.25))
                elif side == 2:
                    pos.append((-0.25, t))
                else:
                    pos.append((Nx + 0.25, t))
    Nc = len(pos)
    rc = np.zeros((Nc, 3))
    rc[:, :2] = np.array(pos)
    g = rng.standard_normal((Nc, 3))
    uc = g / np.linalg.norm(g, axis=1, keepdims=True)
    k = float(kd)
    a = 0.02 * (2.0 * math.pi / k)
    # array basis positions and directions in the vector order (iy Nx + ix) b + m
    iy, ix = np.meshgrid(np.arange(Ny), np.arange(Nx), indexing="ij")
    ra = (r[None, None, :, :] + np.stack([ix, iy, np.zeros_like(ix)], axis=-1)[:, :, None, :]).reshape(-1, 3)
    ua = np.broadcast_to(u, (Ny, Nx, b, 3)).reshape(-1, 3)
    rho_b = np.linalg.norm(rc[:, None, :] - ra[None, :, :], axis=-1)
    ZB = (uc @ ua.T) * np.exp(-1j * k * rho_b) / (4.0 * math.pi * rho_b)
    rho_c = np.linalg.norm(rc[:, None, :] - rc[None, :, :], axis=-1)
    rho_c[np.diag_indices(Nc)] = a
    ZC = (uc @ uc.T) * np.exp(-1j * k * rho_c) / (4.0 * math.pi * rho_c)
    off = np.abs(ZC).copy()
    off[np.diag_indices(Nc)] = 0.0
    ZC[np.diag_indices(Nc)] += alpha * float(off.max(initial=0.0))
    return ZB.astype(np.complex128), ZC.astype(np.complex128)


def port_rhs(Nx: int, Ny: int, b: int, cols=None, port: int = 0,
             dtype=np.complex128) -> np.ndarray:
    """Unit port excitations, one column per element (Sec. IV).

    Column w excites element w = iy*Nx + ix: entry ((iy*Nx+ix)*b + port) is 1,
    everything else 0.  Returned shape (W, Nx*Ny*b), column w contiguous.
    `cols` selects a subset of elements (default: all Nx*Ny).
    """
    if cols is None:
        cols = range(Nx * Ny)
    cols = list(cols)
    V = np.zeros((len(cols), Nx * Ny * b), dtype=dtype)
    for i, e in enumerate(cols):
        V[i, e * b + port] = 1.0
    return V


def centre_element(Nx: int, Ny: int) -> int:
    return (Ny // 2) * Nx + (Nx // 2)


def random_vectors(n: int, W: int, seed: int, dtype=np.complex128) -> np.ndarray:
    """Seeded complex Gaussian columns, shape (W, n)."""
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((W, n)) + 1j * rng.standard_normal((W, n))
    return x.astype(dtype)


def random_blocks(Nx: int, Ny: int, b: int, seed: int, dtype=np.complex128) -> np.ndarray:
    """Unstructured seeded complex blocks (no reciprocity), same layout as green_blocks."""
    rng = np.random.default_rng(seed)
    shp = (2 * Ny - 1, 2 * Nx - 1, b, b)
    return (rng.standard_normal(shp) + 1j * rng.standard_normal(shp)).astype(dtype)


def periodic_blocks(Nx: int, Ny: int, b: int, seed: int, loading: float = 4.0) -> np.ndarray:
    """Blocks of an operator that is exactly periodic on the Ny x Nx torus.

    A seeded set of b x b blocks C[py][qx] (py < Ny, qx < Nx) is drawn and the
    Toeplitz lags are filled as R_{p,q} = C[p mod Ny][q mod Nx].  The matrix
    built from such blocks is block circulant.  C[0][0] gets a diagonal
    loading so that the operator is comfortably invertible.
    """
    rng = np.random.default_rng(seed)
    C = (rng.standard_normal((Ny, Nx, b, b)) + 1j * rng.standard_normal((Ny, Nx, b, b))) / (b * Nx * Ny) ** 0.5
    C[0, 0] += loading * np.eye(b)
    out = np.empty((2 * Ny - 1, 2 * Nx - 1, b, b), dtype=np.complex128)
    for ip, p in enumerate(range(-(Ny - 1), Ny)):
        for iq, q in enumerate(range(-(Nx - 1), Nx)):
            out[ip, iq] = C[p % Ny, q % Nx]
    return out


def c4_arrays(count: int = 64, master_seed: int = 0):
    """Parameters of the uneven multi-array batch.

    Array i draws (Nx, Ny, b, kd) from the master stream: Nx, Ny uniform in
    [4, 24], b uniform in {24, 48, 64, 96}, kd uniform in [pi/2, pi]; its
    element seed is 1000 + i.
    """
    rng = np.random.default_rng(master_seed)
    out = []
    for i in range(count):
        Nx = int(rng.integers(4, 25))
        Ny = int(rng.integers(4, 25))
        b = int(rng.choice([24, 48, 64, 96]))
        kd = float(rng.uniform(math.pi / 2, math.pi))
        out.append(dict(Nx=Nx, Ny=Ny, b=b, kd=kd, seed=1000 + i))
    return out
