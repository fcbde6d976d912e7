"""Training of the learned correction of the block-circulant preconditioner.

The training pairs come from the plain solver itself (block-circulant GMRES in
FP64 on a smaller array of the same element): for the k-th GMRES iterate x_k
of a right-hand side v, the residual is r_k = v - Z x_k and the error is
e_k = x* - x_k, where x* is the same system solved to 1e-12.  The exact
preconditioner would map r_k to e_k (Z e_k = r_k), so the network learns to
turn the block-circulant output y_k = P^{-1} r_k into e_k.  Every product,
preconditioner apply, solve, forward, backward and Adam step runs in
libmlfft.so; this module only sequences the calls and holds the pairs in
device tensors.
"""
from __future__ import annotations

import math
import time

import numpy as np
import torch

from . import abi, synth
from .api import Context


def make_pairs(ctx: Context, array_id: int, Nx: int, Ny: int, b: int, iters: int = 4, n_random: int = 64,
               seed: int = 0, log=None):
    """Pairs (y_k, e_k) as complex64 device tensors of shape (P, Nx*Ny*b) from GMRES iterates 0..iters-1.

    x* is the FP64 solve to 1e-12; x_k the k-step block-circulant GMRES iterate
    (x_0 = 0).  r_k = v - Z x_k is one fused product (mlfft_matvec_axpby),
    y_k = P^{-1} r_k the FP64 preconditioner, and the complex64 pairs are written
    by mlfft_axpby (y_k cast, e_k = x* - x_k formed and cast in one pass).
    """
    N = Nx * Ny * b
    V = synth.port_rhs(Nx, Ny, b)
    if n_random:
        V = np.concatenate([V, synth.random_vectors(N, n_random, seed=seed + 7)])
    Vd = torch.from_numpy(V).cuda()
    W = Vd.shape[0]
    xs, info = ctx.solve(array_id, Vd, tol=1e-12, inner_prec="fp64", precond=1, max_outer=4)
    Y = torch.empty((iters * W, N), dtype=torch.complex64, device=Vd.device)
    E = torch.empty_like(Y)
    rk = torch.empty_like(Vd)
    yk = torch.empty_like(Vd)
    xk = torch.zeros_like(Vd)
    for k in range(iters):
        if k > 0:
            xk, _ = ctx.solve(array_id, Vd, tol=1e-14, inner_prec="fp64", precond=1, restart=k, max_restarts=1,
                              max_outer=1)
        ctx.sync_stream()
        abi.mlfft_matvec_axpby(ctx.h, array_id, W, -1.0, xk.data_ptr(), 1.0, Vd.data_ptr(), rk.data_ptr(),
                               abi.MLFFT_FP64)
        ctx.precond_apply(array_id, rk, yk, kind=1)
        abi.mlfft_axpby(ctx.h, W * N, 1.0, yk.data_ptr(), 0.0, None, abi.MLFFT_FP64,
                        Y[k * W:(k + 1) * W].data_ptr(), abi.MLFFT_FP32)
        abi.mlfft_axpby(ctx.h, W * N, 1.0, xs.data_ptr(), -1.0, xk.data_ptr(), abi.MLFFT_FP64,
                        E[k * W:(k + 1) * W].data_ptr(), abi.MLFFT_FP32)
        if log:
            log(f"[learned] pairs from iterate {k}")
    return Y, E, info


def train(ctx: Context, Y: torch.Tensor, E: torch.Tensor, Nx: int, Ny: int, steps: int = 300, batch: int = 16,
          lr: float = 1e-3, seed: int = 0, holdout: int = 32, log=None):
    """Adam on random minibatches; returns (train loss history, validation loss before, after)."""
    P = Y.shape[0]
    g = torch.Generator(device="cpu").manual_seed(seed)
    perm = torch.randperm(P, generator=g)
    val = perm[:holdout].cuda()
    tr = perm[holdout:]
    Yv, Ev = Y[val].contiguous(), E[val].contiguous()
    _, v0 = abi.mlfft_net_grads(ctx.h, Yv.shape[0], Ny, Nx, Yv.data_ptr(), Ev.data_ptr(), want_grads=False)
    hist = []
    t0 = time.perf_counter()
    for s in range(steps):
        idx = tr[torch.randint(len(tr), (batch,), generator=g)].cuda()
        yb, eb = Y[idx].contiguous(), E[idx].contiguous()
        lr_s = lr * 0.5 * (1 + math.cos(math.pi * s / steps))        # cosine decay
        ctx.sync_stream()
        hist.append(abi.mlfft_net_train_step(ctx.h, batch, Ny, Nx, yb.data_ptr(), eb.data_ptr(), lr_s))
        if log and (s % 50 == 0 or s == steps - 1):
            log(f"[learned] step {s}: loss {hist[-1]:.4e} ({time.perf_counter() - t0:.1f} s)")
    _, v1 = abi.mlfft_net_grads(ctx.h, Yv.shape[0], Ny, Nx, Yv.data_ptr(), Ev.data_ptr(), want_grads=False)
    return hist, v0, v1


GATE = 0.98   # the correction is used only if it takes fewer than GATE x the plain iterations on held-out RHS


def iteration_gate(ctx: Context, array_id: int, N: int, n_rhs: int = 32, seed: int = 99, tol: float = 1e-6):
    """Mean FP32-inner iterations with the plain block circulant and with the learned correction on
    n_rhs held-out random right-hand sides of array `array_id` (the network must be loaded)."""
    V = torch.from_numpy(synth.random_vectors(N, n_rhs, seed=seed)).cuda()
    _, plain = ctx.solve(array_id, V, tol=tol, inner_prec="fp32", precond=1)
    _, lrn = ctx.solve(array_id, V, tol=tol, inner_prec="fp32", precond=3)
    return float(plain["iters"].mean()), float(lrn["iters"].mean())


def prepare(ctx: Context, cfg: dict, train_grid: int = 20, hidden: int = 64, steps: int = 300, log=None,
            array_id: int = 100, lr: float = 3e-4):
    """Build and train the network for the element of `cfg` (b, kd, seed) on a train_grid^2 array.

    The last layer starts at zero, so Adam's first steps move all its weights by
    about lr at once; at the benchmark's scale (a correction of a few percent of
    the preconditioner output) lr = 2e-3 overshoots and the network settles back
    near the identity, while 3e-4 keeps the held-out loss falling.

    The gate is the solver's own measure: the correction is enabled only if
    flexible GMRES with it needs fewer than GATE times the iterations of the
    plain block circulant on held-out right-hand sides of the training array.
    A lower held-out loss alone does not predict that (the network sees Krylov
    basis vectors in the solve, not the residuals it was trained on, and its
    output is a nonlinear function of them).  Returns a dict with the training
    record and the decision ("enabled"); when it is False the solver should use
    the plain preconditioner (the fallback) for this element.
    """
    b, kd, seed = cfg["b"], cfg["kd"], cfg["seed"]
    n = train_grid
    t0 = time.perf_counter()
    ctx.set_blocks(array_id, synth.green_blocks(n, n, b, kd, seed=seed))
    abi.mlfft_net_create(ctx.h, b, hidden, seed + 11)
    Y, E, _ = make_pairs(ctx, array_id, n, n, b, log=log)
    hist, v0, v1 = train(ctx, Y, E, n, n, steps=steps, lr=lr, log=log)
    del Y, E
    it_plain, it_lrn = iteration_gate(ctx, array_id, n * n * b)
    abi.mlfft_drop_array(ctx.h, array_id)
    torch.cuda.empty_cache()
    enabled = bool(it_lrn < GATE * it_plain)
    out = dict(train_grid=n, hidden=hidden, steps=steps, val_loss_before=v0, val_loss_after=v1,
               train_loss_last=hist[-1] if hist else None, heldout_iters_plain=it_plain,
               heldout_iters_learned=it_lrn, seconds=round(time.perf_counter() - t0, 2), enabled=enabled,
               gate=f"held-out iterations below {GATE} x plain")
    if log:
        log(f"[learned] validation loss {v0:.4e} -> {v1:.4e}; held-out iterations {it_lrn:.2f} learned vs "
            f"{it_plain:.2f} plain in {out['seconds']:.1f} s; correction "
            f"{'enabled' if enabled else 'not better than the plain preconditioner: fallback'}")
    return out
