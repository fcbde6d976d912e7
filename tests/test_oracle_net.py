"""Pins of the oracle's learned-correction network (CPU only)."""
import numpy as np
import pytest
import scipy.signal as ss
import torch

from oracle import net


def test_bf16_round_ties_to_even_and_matches_torch():
    x = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, -1 - 2 ** -8, 3.14159, 1e-30, 65504.0, -0.0, 1 + 2 ** -9])
    got = net.bf16_round(x)
    assert got[1] == 1.0                       # tie -> even mantissa
    assert got[2] == 1 + 2 ** -6               # tie -> even mantissa (upwards)
    assert got[3] == -1.0
    assert got[8] == 1.0
    rng = np.random.default_rng(0)
    y = np.concatenate([x, rng.standard_normal(2000) * 10.0 ** rng.integers(-20, 20, 2000)])
    ref = torch.tensor(y, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(net.bf16_round(y), ref)


def test_conv_single_channel_matches_scipy_correlate():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((7, 5))
    w = rng.standard_normal((3, 3))
    got = net.conv3x3(x[None, :, :, None], w[None, None])[0, :, :, 0]
    np.testing.assert_allclose(got, ss.correlate2d(x, w, mode="same"), rtol=0, atol=1e-13)


def test_conv_multichannel_matches_torch_conv2d():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((2, 6, 4, 5))
    w = rng.standard_normal((3, 5, 3, 3))
    ref = torch.nn.functional.conv2d(torch.tensor(x).permute(0, 3, 1, 2), torch.tensor(w), padding=1)
    np.testing.assert_allclose(net.conv3x3(x, w), ref.permute(0, 2, 3, 1).numpy(), rtol=0, atol=1e-12)


def test_dgrad_and_wgrad_are_adjoints():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((3, 5, 6, 4))
    w = rng.standard_normal((7, 4, 3, 3))
    g = rng.standard_normal((3, 5, 6, 7))
    lhs = np.sum(net.conv3x3(x, w) * g)
    assert abs(lhs - np.sum(x * net.conv3x3_dgrad(g, w))) <= 1e-11 * abs(lhs)
    assert abs(lhs - np.sum(w * net.conv3x3_wgrad(x, g))) <= 1e-11 * abs(lhs)


def test_loss_gradient_matches_finite_differences():
    Nx, Ny, b, H = 3, 4, 2, 5
    rng = np.random.default_rng(4)
    ws = net.init_weights(b, H, seed=1)
    ws[3] = rng.standard_normal(ws[3].shape) * 0.1      # non-zero last layer for a real check
    y = rng.standard_normal((2, Nx * Ny * b)) + 1j * rng.standard_normal((2, Nx * Ny * b))
    e = rng.standard_normal((2, Nx * Ny * b)) + 1j * rng.standard_normal((2, Nx * Ny * b))
    loss, grads = net.loss_and_grads(y, e, ws, Nx, Ny, b, bf16=False)
    h = 1e-6
    for l in range(4):
        for idx in [(0, 0, 1, 1), (1, 1, 0, 2), (ws[l].shape[0] - 1, ws[l].shape[1] - 1, 2, 0)]:
            wp = [w.copy() for w in ws]
            wm = [w.copy() for w in ws]
            wp[l][idx] += h
            wm[l][idx] -= h
            lp, _ = net.loss_and_grads(y, e, wp, Nx, Ny, b, bf16=False)
            lm, _ = net.loss_and_grads(y, e, wm, Nx, Ny, b, bf16=False)
            fd = (lp - lm) / (2 * h)
            assert abs(fd - grads[l][idx]) <= 1e-6 * max(1.0, abs(fd)), (l, idx, fd, grads[l][idx])


def test_zero_last_layer_is_identity_correction():
    Nx, Ny, b = 4, 3, 3
    ws = net.init_weights(b, 8, seed=0)
    rng = np.random.default_rng(5)
    y = rng.standard_normal((3, Nx * Ny * b)) + 1j * rng.standard_normal((3, Nx * Ny * b))
    np.testing.assert_allclose(net.learned_apply(y, ws, Nx, Ny, b), y, rtol=1e-15, atol=1e-15)


def test_learned_apply_is_homogeneous():
    Nx, Ny, b = 3, 3, 2
    ws = net.init_weights(b, 6, seed=2)
    rng = np.random.default_rng(6)
    ws[3] = rng.standard_normal(ws[3].shape) * 0.2
    y = rng.standard_normal((2, Nx * Ny * b)) + 1j * rng.standard_normal((2, Nx * Ny * b))
    c = 3.7 * np.exp(0.9j)
    a = net.learned_apply(c * y, ws, Nx, Ny, b, bf16=False)
    np.testing.assert_allclose(a, c * net.learned_apply(y, ws, Nx, Ny, b, bf16=False), rtol=1e-12, atol=1e-12)


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(7)
    w = [rng.standard_normal((3, 2, 3, 3))]
    g = [rng.standard_normal((3, 2, 3, 3))]
    opt = net.Adam(w, lr=1e-3)
    w1 = opt.step(w, g)
    # first step: m_hat = g, v_hat = g^2, so the move is lr * g / (|g| + eps)
    np.testing.assert_allclose(w1[0], w[0] - 1e-3 * g[0] / (np.abs(g[0]) + 1e-8), rtol=1e-14, atol=1e-15)


@pytest.mark.parametrize("b", [1, 3])
def test_complex_nhwc_roundtrip(b):
    rng = np.random.default_rng(b)
    y = rng.standard_normal((2, 12 * b)) + 1j * rng.standard_normal((2, 12 * b))
    t = net.complex_to_nhwc(y, 4, 3, b)
    assert t.shape == (2, 3, 4, 2 * b)
    assert t[0, 0, 1, 0] == y[0, b].real and t[0, 0, 1, 1] == y[0, b].imag
    np.testing.assert_array_equal(net.nhwc_to_complex(t), y)


def test_adam_two_steps_closed_form():
    """Step 2 with gradients g1, g2: the bias-corrected moments are m_hat = (b1 g1 + g2) / (1 + b1)
    and v_hat = (b2 g1^2 + g2^2) / (1 + b2) (divide b1 (1 - b1) g1 + (1 - b1) g2 by 1 - b1^2)."""
    rng = np.random.default_rng(8)
    w = [rng.standard_normal((4, 3, 3, 3))]
    g1 = [rng.standard_normal(w[0].shape)]
    g2 = [rng.standard_normal(w[0].shape)]
    opt = net.Adam(w, lr=1e-3)
    w1 = opt.step(w, g1)
    w2 = opt.step(w1, g2)
    b1, b2 = 0.9, 0.999
    mh = (b1 * g1[0] + g2[0]) / (1 + b1)
    vh = (b2 * g1[0] ** 2 + g2[0] ** 2) / (1 + b2)
    np.testing.assert_allclose(w2[0], w1[0] - 1e-3 * mh / (np.sqrt(vh) + 1e-8), rtol=1e-13, atol=1e-15)


def test_adam_constant_gradient_moves_every_step_by_lr():
    """With a constant gradient g the bias-corrected moments are g and g^2 at every step t, so
    each step moves a weight by lr * g / (|g| + eps); a wrong power of beta in the correction fails."""
    rng = np.random.default_rng(9)
    w = [rng.standard_normal((2, 5))]
    g = [rng.standard_normal((2, 5))]
    opt = net.Adam(w, lr=2e-3)
    cur = w
    for t in range(1, 8):
        cur = opt.step(cur, g)
        np.testing.assert_allclose(cur[0], w[0] - t * 2e-3 * g[0] / (np.abs(g[0]) + 1e-8), rtol=0, atol=1e-14)
