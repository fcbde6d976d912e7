"""How much of the block-circulant preconditioner's error a local correction can remove (CPU only).

The learned correction is a stack of four 3x3 convolutions, so its output at a
cell depends on the preconditioned residual in the 9x9 cells around it.  The
best such map that is linear is a least-squares problem on pairs
(yhat, ehat - yhat); its held-out loss bounds what the linear part of any
such network can reach.  At the element loading of the benchmark element
(10x the largest off-diagonal magnitude), the error left by the block-circulant
preconditioner comes from the wrap-around of the circulant across the array
edges, which no local map sees: the bound stays close to the identity's loss.
At a weak loading the bound is lower, which is where the trained network gains
iterations (tests/test_gpu_net.py).
"""
import numpy as np
import pytest

from oracle import krylov, precond
from oracle import net as onet
from oracle import toeplitz as tp
from paper_2506_20350_amd import synth


def _pairs(n, b, alpha, iters=4, nrand=16, seed=0):
    """(y_k, e_k) from the plain block-circulant GMRES iterates k = 0..iters-1 (as in training)."""
    blocks = synth.green_blocks(n, n, b, np.pi, seed=seed, alpha=alpha)
    mv = lambda X: tp.matvec_fft(blocks, X, 2 * n, 2 * n)
    Sinv = precond.strang_inverse_spectrum(blocks)
    pc = lambda X: precond.strang_apply(Sinv, X)
    V = np.concatenate([synth.port_rhs(n, n, b), synth.random_vectors(n * n * b, nrand, seed=seed + 7)])
    xs = np.array([r.x for r in krylov.gmres_columns(mv, V, pc, tol=1e-12)])
    Y, E = [], []
    for k in range(iters):
        xk = np.zeros_like(V) if k == 0 else np.array(
            [r.x for r in krylov.gmres_columns(mv, V, pc, tol=1e-14, restart=k, max_restarts=1)])
        Y.append(pc(V - mv(xk)))
        E.append(xs - xk)
    return np.concatenate(Y), np.concatenate(E)


def _local_linear_bound(n, b, alpha, radius=4):
    Y, E = _pairs(n, b, alpha)
    yh, s, ph = onet.normalise(Y)
    eh = E / (ph * s)[:, None]
    t = onet.complex_to_nhwc(yh, n, n, b)
    tg = onet.complex_to_nhwc(eh, n, n, b)
    D = tg - t
    S = t.shape[0]
    P = np.pad(t, ((0, 0), (radius, radius), (radius, radius), (0, 0)))
    k = 2 * radius + 1
    F = np.concatenate([P[:, i:i + n, j:j + n, :] for i in range(k) for j in range(k)], axis=3)
    F = F.reshape(S * n * n, -1)
    T = D.reshape(S * n * n, -1)
    held = np.arange(S) % 5 == 0               # every fifth pair is held out
    train = np.repeat(~held, n * n)
    Wls = np.linalg.lstsq(F[train], T[train], rcond=None)[0]
    den = np.sum(tg[held] ** 2)
    identity = np.sum(T[~train] ** 2) / den
    fitted = np.sum((T[~train] - F[~train] @ Wls) ** 2) / den
    return identity, fitted


def test_local_correction_bound_at_benchmark_loading():
    identity, fitted = _local_linear_bound(8, 8, alpha=10.0)
    assert identity < 1e-2                     # the block circulant is already close
    assert fitted > 0.75 * identity            # a 9x9 linear map removes less than a quarter of what is left


def test_local_correction_bound_at_weak_loading_is_lower():
    identity, fitted = _local_linear_bound(8, 8, alpha=1.0)
    assert fitted < 0.9 * identity
