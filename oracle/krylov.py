"""Restarted GMRES / flexible GMRES, per right-hand side and global.

Oracle (test infrastructure only).  The paper passes GMRES a matvec handle
and a preconditioner handle (Sec. III-C) without stating restart, iteration
cap, initial guess or orthogonalisation.  Readings used here: restart m = 30,
x0 = 0, modified Gram-Schmidt, complex Givens rotations, right (or flexible)
preconditioning so that the minimised residual is the true one, and the stop
test  ||v - A x||_2 <= tol ||v||_2  per right-hand side, confirmed with the
true residual at every restart.  The paper's global (vectorised) variant,
eq. ZIVvec, is GMRES on vec(I_M) with the Frobenius inner product, which is
what `gmres_global` does.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class GmresResult:
    x: np.ndarray
    converged: bool
    iters: int
    relres: float
    history: list = field(default_factory=list)   # residual estimate / ||v|| after each iteration


def givens(a: complex, b: complex):
    """(cs, sn) with cs real such that [[cs, sn], [-conj(sn), cs]] @ [a, b] = [rho, 0]."""
    if b == 0:
        return 1.0, 0.0 + 0.0j
    if a == 0:
        return 0.0, np.conj(b) / abs(b)
    r = np.hypot(abs(a), abs(b))
    cs = abs(a) / r
    sn = (a / abs(a)) * np.conj(b) / r
    return cs, sn


def gmres(matvec, v: np.ndarray, precond=None, restart: int = 30, tol: float = 1e-8,
          max_restarts: int = 100, x0=None, flexible: bool = False) -> GmresResult:
    """Solve A x = v for one vector v (1-D), A given by `matvec`.

    `precond(r)` returns M^{-1} r (None: no preconditioner).  With
    `flexible=True` the preconditioned directions z_j are stored and the
    update is x += Z_m y (FGMRES); otherwise x += M^{-1}(V_m y).
    """
    n = v.shape[0]
    vnorm = np.linalg.norm(v)
    x = np.zeros(n, dtype=np.complex128) if x0 is None else np.array(x0, dtype=np.complex128)
    hist = []
    iters = 0
    if vnorm == 0:
        return GmresResult(np.zeros(n, dtype=np.complex128), True, 0, 0.0, hist)
    m = restart
    for _cycle in range(max_restarts + 1):
        r = v - matvec(x)
        beta = np.linalg.norm(r)
        relres = beta / vnorm
        if relres <= tol or _cycle == max_restarts:
            return GmresResult(x, relres <= tol, iters, relres, hist)
        V = np.zeros((m + 1, n), dtype=np.complex128)
        Zs = np.zeros((m, n), dtype=np.complex128) if (flexible and precond is not None) else None
        H = np.zeros((m + 1, m), dtype=np.complex128)
        cs = np.zeros(m)
        sn = np.zeros(m, dtype=np.complex128)
        g = np.zeros(m + 1, dtype=np.complex128)
        g[0] = beta
        V[0] = r / beta
        k = 0
        for j in range(m):
            z = V[j] if precond is None else precond(V[j])
            if Zs is not None:
                Zs[j] = z
            w = matvec(z)
            for i in range(j + 1):                         # modified Gram-Schmidt
                H[i, j] = np.vdot(V[i], w)
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            for i in range(j):                             # earlier rotations
                hi, hi1 = H[i, j], H[i + 1, j]
                H[i, j] = cs[i] * hi + sn[i] * hi1
                H[i + 1, j] = -np.conj(sn[i]) * hi + cs[i] * hi1
            cs[j], sn[j] = givens(H[j, j], H[j + 1, j])
            hj, hj1 = H[j, j], H[j + 1, j]
            H[j, j] = cs[j] * hj + sn[j] * hj1
            H[j + 1, j] = 0.0
            g[j + 1] = -np.conj(sn[j]) * g[j]
            g[j] = cs[j] * g[j]
            iters += 1
            k = j + 1
            est = abs(g[j + 1]) / vnorm
            hist.append(est)
            breakdown = np.linalg.norm(w) <= 1e-300
            if est <= tol or breakdown:
                break
            V[j + 1] = w / np.linalg.norm(w)
        y = np.linalg.solve(np.triu(H[:k, :k]), g[:k])
        if Zs is not None:
            x = x + y @ Zs[:k]
        elif precond is None:
            x = x + y @ V[:k]
        else:
            x = x + precond(y @ V[:k])
    raise AssertionError("unreachable")


def gmres_columns(matvec_cols, V: np.ndarray, precond_cols=None, **kw) -> list:
    """Per-RHS GMRES: one independent Krylov space per row of V (shape (W, N)).

    `matvec_cols(X)` and `precond_cols(X)` act on (k, N) arrays; they are
    called with single rows here.
    """
    out = []
    for w in range(V.shape[0]):
        mv = (lambda z: matvec_cols(z[None, :])[0])
        pc = None if precond_cols is None else (lambda z: precond_cols(z[None, :])[0])
        out.append(gmres(mv, V[w], pc, **kw))
    return out


def gmres_global(matvec_cols, V: np.ndarray, precond_cols=None, **kw) -> GmresResult:
    """Global (vectorised) GMRES on (I (x) A) vec(X) = vec(V) (eq. ZIVvec).

    One Krylov space for all columns together; inner products and norms are
    the Frobenius ones over all W columns.
    """
    W, N = V.shape
    mv = lambda z: matvec_cols(z.reshape(W, N)).reshape(-1)
    pc = None if precond_cols is None else (lambda z: precond_cols(z.reshape(W, N)).reshape(-1))
    res = gmres(mv, V.reshape(-1), pc, **kw)
    res.x = res.x.reshape(W, N)
    return res


def true_relres(matvec_cols, X: np.ndarray, V: np.ndarray) -> np.ndarray:
    """Per-column ||v_w - A x_w|| / ||v_w||."""
    R = V - matvec_cols(X)
    return np.linalg.norm(R, axis=1) / np.linalg.norm(V, axis=1)
