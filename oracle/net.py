"""FP64 reference of the learned correction to the block-circulant preconditioner.

Oracle (test infrastructure only).  The paper proposes no network; it asks
for a preconditioner that covers the neighbouring elements (Sec. V).  The
learned correction is therefore a reading, stated here in full:

* A complex field on the array grid, y[w][iy][ix][m] (paper order of one
  column), is seen as a real tensor in NHWC layout with 2b channels, channel
  c = 2m + part (part 0 = real, 1 = imaginary).
* Normalisation per column: s = ||y||_2, phi = arg of the entry of largest
  modulus (first such entry), y_hat = y exp(-i phi) / s.
* Network: four 3x3 convolutions with zero "same" padding and no bias,
  channels 2b -> H -> H -> H -> 2b, ReLU after the first three:
      out[n,i,j,co] = sum_{ci,di,dj} w[co,ci,di,dj] x[n, i+di-1, j+dj-1, ci].
  The last layer starts at zero, so the untrained correction is the identity.
* Output: z = s exp(i phi) (y_hat + Net(y_hat)).
* Loss for a pair (y, e): ||y_hat + Net(y_hat) - e_hat||^2 / ||e_hat||^2
  with e_hat = e exp(-i phi) / s, averaged over the batch.
* Mixed precision: each convolution sees its weights and its input rounded
  to bfloat16 (round to nearest, ties to even); accumulation is exact here
  (FP64).  The backward pass differentiates that forward with the rounding
  taken as the identity (straight-through), using the rounded operands.
* Adam with beta1 = 0.9, beta2 = 0.999, eps = 1e-8 and bias correction.
"""
from __future__ import annotations

import numpy as np


# ------------------------------------------------------------- bfloat16

def bf16_round(x: np.ndarray) -> np.ndarray:
    """Round float values to the nearest bfloat16 (ties to even); returns float64.

    bfloat16 keeps the top 16 bits of an IEEE binary32 value; rounding adds
    0x7FFF plus the lowest kept bit before truncating, which is round to
    nearest with ties to even.  NaN stays NaN.
    """
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(np.isnan(f), np.nan, out)


# ------------------------------------------------------------- layout

def complex_to_nhwc(y: np.ndarray, Nx: int, Ny: int, b: int) -> np.ndarray:
    """(W, N) complex columns -> (W, Ny, Nx, 2b) real, channel 2m + part."""
    W = y.shape[0]
    c = y.reshape(W, Ny, Nx, b)
    out = np.empty((W, Ny, Nx, 2 * b))
    out[..., 0::2] = c.real
    out[..., 1::2] = c.imag
    return out


def nhwc_to_complex(t: np.ndarray) -> np.ndarray:
    W = t.shape[0]
    return (t[..., 0::2] + 1j * t[..., 1::2]).reshape(W, -1)


# ------------------------------------------------------------- convolutions

def conv3x3(x: np.ndarray, w: np.ndarray) -> np.ndarray:
    """x (n, H, W, Cin), w (Cout, Cin, 3, 3) -> (n, H, W, Cout); zero same padding."""
    n, H, Wd, Cin = x.shape
    Cout = w.shape[0]
    xp = np.zeros((n, H + 2, Wd + 2, Cin))
    xp[:, 1:H + 1, 1:Wd + 1, :] = x
    y = np.zeros((n, H, Wd, Cout))
    for di in range(3):
        for dj in range(3):
            y += xp[:, di:di + H, dj:dj + Wd, :] @ w[:, :, di, dj].T
    return y


def conv3x3_dgrad(g: np.ndarray, w: np.ndarray) -> np.ndarray:
    """Gradient of sum(g * conv3x3(x, w)) with respect to x."""
    n, H, Wd, Cout = g.shape
    Cin = w.shape[1]
    dxp = np.zeros((n, H + 2, Wd + 2, Cin))
    for di in range(3):
        for dj in range(3):
            dxp[:, di:di + H, dj:dj + Wd, :] += g @ w[:, :, di, dj]
    return dxp[:, 1:H + 1, 1:Wd + 1, :]


def conv3x3_wgrad(x: np.ndarray, g: np.ndarray) -> np.ndarray:
    """Gradient of sum(g * conv3x3(x, w)) with respect to w, shape (Cout, Cin, 3, 3)."""
    n, H, Wd, Cin = x.shape
    Cout = g.shape[3]
    xp = np.zeros((n, H + 2, Wd + 2, Cin))
    xp[:, 1:H + 1, 1:Wd + 1, :] = x
    dw = np.zeros((Cout, Cin, 3, 3))
    g2 = g.reshape(-1, Cout)
    for di in range(3):
        for dj in range(3):
            dw[:, :, di, dj] = g2.T @ xp[:, di:di + H, dj:dj + Wd, :].reshape(-1, Cin)
    return dw


# ------------------------------------------------------------- network

def init_weights(b: int, hidden: int, seed: int) -> list:
    """He-normal weights for the first three layers, zeros for the last one."""
    rng = np.random.default_rng(seed)
    chans = [2 * b, hidden, hidden, hidden, 2 * b]
    ws = []
    for l in range(4):
        cin, cout = chans[l], chans[l + 1]
        if l == 3:
            ws.append(np.zeros((cout, cin, 3, 3)))
        else:
            ws.append(rng.standard_normal((cout, cin, 3, 3)) * np.sqrt(2.0 / (9 * cin)))
    return ws


def net_forward(x: np.ndarray, ws: list, bf16: bool = True):
    """Forward pass; returns (output, cache) with cache = per-layer (conv input, pre-activation)."""
    cache = []
    a = x
    for l, w in enumerate(ws):
        wl = bf16_round(w) if bf16 else w
        al = bf16_round(a) if bf16 else a
        y = conv3x3(al, wl)
        cache.append((al, wl, y))
        a = np.maximum(y, 0.0) if l < len(ws) - 1 else y
    return a, cache


def net_backward(g_out: np.ndarray, cache: list) -> list:
    """Weight gradients given the gradient of the loss with respect to the net output."""
    grads = [None] * len(cache)
    g = g_out
    for l in range(len(cache) - 1, -1, -1):
        al, wl, y = cache[l]
        if l < len(cache) - 1:
            g = g * (y > 0)
        grads[l] = conv3x3_wgrad(al, g)
        if l > 0:
            g = conv3x3_dgrad(g, wl)
    return grads


def normalise(y: np.ndarray):
    """Per column: s = ||y||, phi = arg(y at the largest |y|), y_hat = y e^{-i phi}/s."""
    W = y.shape[0]
    s = np.linalg.norm(y, axis=1)
    idx = np.argmax(np.abs(y), axis=1)
    phase = np.exp(1j * np.angle(y[np.arange(W), idx]))
    safe = np.where(s > 0, s, 1.0)
    yh = y / (phase * safe)[:, None]
    return yh, s, phase


def learned_apply(y: np.ndarray, ws: list, Nx: int, Ny: int, b: int, bf16: bool = True) -> np.ndarray:
    """z = s e^{i phi} (y_hat + Net(y_hat)) for every column of y (shape (W, N))."""
    yh, s, phase = normalise(y)
    t = complex_to_nhwc(yh, Nx, Ny, b)
    out, _ = net_forward(t, ws, bf16)
    z = nhwc_to_complex(t + out)
    return z * (phase * s)[:, None]


def loss_and_grads(y: np.ndarray, e: np.ndarray, ws: list, Nx: int, Ny: int, b: int, bf16: bool = True):
    """Mean relative squared error of the corrected output against the target error e."""
    yh, s, phase = normalise(y)
    safe = np.where(s > 0, s, 1.0)
    eh = e / (phase * safe)[:, None]
    t = complex_to_nhwc(yh, Nx, Ny, b)
    tgt = complex_to_nhwc(eh, Nx, Ny, b)
    out, cache = net_forward(t, ws, bf16)
    diff = t + out - tgt
    den = np.sum(tgt * tgt, axis=(1, 2, 3))
    B = y.shape[0]
    loss = float(np.mean(np.sum(diff * diff, axis=(1, 2, 3)) / den))
    g_out = 2.0 * diff / den[:, None, None, None] / B
    return loss, net_backward(g_out, cache)


class Adam:
    """Adam with bias correction (beta1 = 0.9, beta2 = 0.999, eps = 1e-8)."""

    def __init__(self, ws: list, lr: float = 1e-3, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, beta1, beta2, eps
        self.m = [np.zeros_like(w) for w in ws]
        self.v = [np.zeros_like(w) for w in ws]
        self.t = 0

    def step(self, ws: list, grads: list) -> list:
        self.t += 1
        out = []
        for i, (w, g) in enumerate(zip(ws, grads)):
            self.m[i] = self.b1 * self.m[i] + (1 - self.b1) * g
            self.v[i] = self.b2 * self.v[i] + (1 - self.b2) * g * g
            mh = self.m[i] / (1 - self.b1 ** self.t)
            vh = self.v[i] / (1 - self.b2 ** self.t)
            out.append(w - self.lr * mh / (np.sqrt(vh) + self.eps))
        return out
