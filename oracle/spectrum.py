"""Singular values of the preconditioned operator P^{-1} Z by a randomized range finder.

Oracle (test infrastructure only).  Sec. V studies the spectrum of P^{-1} Z for
P = I, P_K and P_Z with the randomized methods of Halko, Martinsson and Tropp
("Finding structure with randomness", 2011), using the fast MLFFT product.  The
steps, with the test matrix Omega passed in (N x l, l = target rank plus
oversampling) so that both sides draw the same random numbers:

  1. Y = A Omega;
  2. q power steps, each Y = A (A^H Y) after orthonormalising Y (their
     Algorithm 4.4 without the intermediate re-orthonormalisation of A^H Y);
  3. Q = an orthonormal basis of range(Y) (QR);
  4. B = Q^H A (formed as (A^H Q)^H);
  5. the singular values of B approximate the l largest of A.

A is given by two callables, the product x -> A x and the adjoint product
y -> A^H y, each acting on the rows of a (l, N) array (one vector per row).
"""
from __future__ import annotations

import numpy as np


def randomized_singular_values(A, AH, Omega: np.ndarray, power_iters: int = 0) -> np.ndarray:
    """Approximate largest singular values (descending) of A; Omega has shape (l, N)."""
    Y = A(Omega)                                       # (l, N): rows are the vectors A omega_i
    for _ in range(power_iters):
        Q, _ = np.linalg.qr(Y.T)
        Y = A(AH(Q.T))
    Q, _ = np.linalg.qr(Y.T)                           # N x l orthonormal
    Bh = AH(Q.T)                                       # rows: A^H q_i, i.e. B^H = A^H Q column by column
    return np.linalg.svd(Bh.T, compute_uv=False)       # singular values of B^H equal those of B
