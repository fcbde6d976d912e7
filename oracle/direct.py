"""Direct references: dense LU and the block Rybicki recursion.

Oracle (test infrastructure only).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .toeplitz import level1_blocks, shape_of


def lu_solve(Z: np.ndarray, V: np.ndarray) -> np.ndarray:
    """I = Z^{-1} V with a dense LU (the analogue of mldivide, Sec. IV).

    V has shape (W, N) (one excitation per row); returns the same shape.
    """
    lu = sla.lu_factor(Z)
    return sla.lu_solve(lu, V.T).T


class SingularSection(np.linalg.LinAlgError):
    """A leading block section needed by the recursion is (numerically) singular."""


def _inv_checked(A: np.ndarray, what: str, rcond_min: float) -> np.ndarray:
    # The recursion needs every leading block section nonsingular; the paper
    # states it for invertible blocks, the bordering steps need more (our
    # reading): check the reciprocal condition number.
    c = np.linalg.cond(A, 1)
    if not np.isfinite(c) or 1.0 / c < rcond_min:
        raise SingularSection(f"{what} is singular (rcond {0.0 if not np.isfinite(c) else 1.0 / c:.2e})")
    return np.linalg.inv(A)


def rybicki_solve(R: dict, Y: list, rcond_min: float = 1e-14) -> list:
    """Solve sum_{j=1}^{n} R_{i-j} x_j = y_i (i = 1..n) with the block bordering recursion.

    Sec. III-D, eqs. xmpo, xi, GM1, HM1, HM and GH.  R maps a lag p in
    (-n, n) to a square block R_p (here the dense level-1 blocks of the
    array), Y is the list [y_1, ..., y_n] of right-hand-side blocks (each may
    have several columns).  Order-M solutions x^(M), together with the
    auxiliary block sequences G^(M) (solving sum_l R_{l-i} G_l = R_{-i}) and
    H^(M) (solving sum_l R_{i-l} H_l = R_i), are extended one block at a time;
    every update uses the order-M values, with the matrix products kept in the
    order the non-commuting blocks require.  Returns [x_1, ..., x_n].
    """
    n = len(Y)
    R0inv = _inv_checked(R[0], "R_0", rcond_min)
    x = [R0inv @ Y[0]]
    if n == 1:
        return x
    G = [None, R0inv @ R[-1]]            # 1-based: G[1]
    H = [None, R0inv @ R[1]]             # 1-based: H[1]
    for M in range(1, n):
        # eq. xmpo: the new last block of the solution
        D = sum(R[M + 1 - j] @ G[M + 1 - j] for j in range(1, M + 1)) - R[0]
        Dinv = _inv_checked(D, f"D at order {M}", rcond_min)
        rhs = sum(R[M + 1 - j] @ x[j - 1] for j in range(1, M + 1)) - Y[M]
        x_new = Dinv @ rhs
        # eq. xi: correct the earlier blocks
        x = [x[j - 1] - G[M + 1 - j] @ x_new for j in range(1, M + 1)] + [x_new]
        if M + 1 == n:
            break
        # eq. GM1
        E = sum(R[j - (M + 1)] @ H[M + 1 - j] for j in range(1, M + 1)) - R[0]
        Einv = _inv_checked(E, f"E at order {M}", rcond_min)
        G_new = Einv @ (sum(R[j - (M + 1)] @ G[j] for j in range(1, M + 1)) - R[-(M + 1)])
        # eq. HM1
        H_new = Dinv @ (sum(R[M + 1 - j] @ H[j] for j in range(1, M + 1)) - R[M + 1])
        # eqs. GH / HM, both from the order-M sequences
        G_old, H_old = G, H
        G = [None] + [G_old[j] - H_old[M + 1 - j] @ G_new for j in range(1, M + 1)] + [G_new]
        H = [None] + [H_old[j] - G_old[M + 1 - j] @ H_new for j in range(1, M + 1)] + [H_new]
    return x


def rybicki_solve_array(blocks: np.ndarray, V: np.ndarray, rcond_min: float = 1e-14) -> np.ndarray:
    """Solve Z_A I = V for a two-level array with the block Rybicki recursion on level 2.

    The recursion runs over the Ny array rows; its blocks are the dense
    level-1 blocks T^[1]_p of size Nx*b (Sec. III-D, last paragraph).  V has
    shape (W, N); returns the same shape.
    """
    Nx, Ny, b = shape_of(blocks)
    R = level1_blocks(blocks)
    L = Nx * b
    Y = [V[:, iy * L:(iy + 1) * L].T for iy in range(Ny)]
    xs = rybicki_solve(R, Y, rcond_min)
    return np.concatenate(xs, axis=0).T
