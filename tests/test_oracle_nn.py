"""Pins of the network oracle (CPU only): brute force, a library correlation,
adjoint identities, finite-difference gradients and known BF16 roundings."""
import numpy as np
import pytest
import scipy.signal

from oracle import nn

RNG = np.random.Generator(np.random.PCG64(7))


def test_bf16_rounding_known_values():
    one = 1.0
    ulp = 2.0 ** -7  # BF16 spacing in [1, 2)
    assert nn.bf16(one) == one
    assert nn.bf16(one + ulp) == one + ulp
    assert nn.bf16(one + ulp / 2) == one              # tie -> even (1.0)
    assert nn.bf16(one + 3 * ulp / 2) == one + 2 * ulp  # tie -> even (1 + 2 ulp)
    assert nn.bf16(one + 0.7 * ulp) == one + ulp
    assert nn.bf16(-2.5) == -2.5 and nn.bf16(0.0) == 0.0
    x = RNG.standard_normal(1000)
    r = nn.bf16(x)
    assert np.all(np.abs(r - x) <= 2.0 ** -8 * np.abs(x) * (1 + 1e-6))


def test_conv_matches_brute_force():
    x = RNG.standard_normal((2, 4, 5, 3))
    w = RNG.standard_normal((9, 3, 2))
    y = nn.conv(x, w)
    B, H, W, _ = x.shape
    ref = np.zeros_like(y)
    for b in range(B):
        for i in range(H):
            for j in range(W):
                for t, (dy, dx) in enumerate(nn.TAPS):
                    ii, jj = i + dy, j + dx
                    if 0 <= ii < H and 0 <= jj < W:
                        ref[b, i, j] += x[b, ii, jj] @ w[t]
    np.testing.assert_allclose(y, ref, rtol=1e-13, atol=1e-13)


def test_conv_matches_scipy_correlate():
    x = RNG.standard_normal((1, 7, 6, 2))
    w = RNG.standard_normal((9, 2, 3))
    y = nn.conv(x, w)
    for o in range(3):
        ref = np.zeros((7, 6))
        for c in range(2):
            k = w[:, c, o].reshape(3, 3)
            ref += scipy.signal.correlate(x[0, :, :, c], k, mode="same")
        np.testing.assert_allclose(y[0, :, :, o], ref, rtol=1e-12, atol=1e-12)


def test_adjoints():
    x = RNG.standard_normal((2, 6, 5, 4))
    w = RNG.standard_normal((9, 4, 3))
    g = RNG.standard_normal((2, 6, 5, 3))
    lhs = float((nn.conv(x, w) * g).sum())
    assert float((x * nn.conv_adjoint(g, w)).sum()) == pytest.approx(lhs, rel=1e-12)
    assert float((w * nn.weight_grad(x, g)).sum()) == pytest.approx(lhs, rel=1e-12)


def test_gradients_match_finite_differences():
    params = nn.init_params(3)
    x = RNG.standard_normal((2, 10, 9, 4))
    t = RNG.standard_normal((2, 10, 9, 2))
    loss, grads = nn.loss_and_grads(params, x, t, rounding=False)
    h = 1e-6
    for l in range(3):
        for idx in [(0, 0, 0), (4, 1, 1), (8, 3 if l == 0 else 15, 1)]:
            pp = [p.copy() for p in params]
            pm = [p.copy() for p in params]
            pp[l][idx] += h
            pm[l][idx] -= h
            fd = (nn.loss_and_grads(pp, x, t, rounding=False)[0]
                  - nn.loss_and_grads(pm, x, t, rounding=False)[0]) / (2 * h)
            assert grads[l][idx] == pytest.approx(fd, rel=2e-5, abs=1e-10), (l, idx)


def test_loss_ignores_the_border():
    params = nn.init_params(4)
    x = RNG.standard_normal((1, 12, 12, 4))
    y, _ = nn.forward(params, x, rounding=False)
    t = y.copy()
    t[:, :nn.MARGIN] += 5.0  # differences only in the border
    loss, _ = nn.loss_and_grads(params, x, t, rounding=False)
    assert loss == 0.0


def test_adam_single_step_by_hand():
    w = [np.array([[[1.0]]])]
    g = [np.array([[[0.5]]])]
    state = [(np.zeros((1, 1, 1)), np.zeros((1, 1, 1)))]
    out = nn.adam_step(w, g, state, lr=0.1, step=1)
    # m = 0.05, v = 0.00025; bias-corrected m^ = 0.5, v^ = 0.25: step 0.1 * 0.5 / (0.5 + 1e-8)
    assert out[0][0, 0, 0] == pytest.approx(1.0 - 0.1 * 0.5 / (0.5 + 1e-8), rel=1e-15)
