"""CPU oracle of the learned preconditioner's network (test infrastructure only).

The network is a plain three-layer stack of 3x3 "same" convolutions with zero
padding: 4 -> 16 -> 16 -> 2 channels, ReLU after the first two layers, no
biases.  Inputs per interior node of a cos/sin plane pair are the pair's
residuals divided by their RMS, the normalised radius (r - r_in)/(r_out - r_in)
and the plane shift relative to the diagonal, lambda mu / (D0 + lambda mu);
outputs are the pair's corrections times diag / RMS.  (The paper has no such
network; the brief fixes its shape: 3 layers, 16 channels, 3x3, BF16 weights
with FP32 accumulation.)

Layouts: images (B, H, W, C) with C fastest; weights (9, Cin, Cout) with tap
t = (dy + 1) * 3 + (dx + 1), so that
    y[b, i, j, o] = sum_{t, c} x[b, i + dy, j + dx, c] * w[t, c, o]
(x = 0 outside the image).

With ``rounding=True`` every operand that the GPU feeds to its BF16 matrix
instructions is rounded to BF16 here too (round to nearest, ties to even, from
the FP32 value); accumulation is FP64.  So GPU and oracle compute the same
quantity and differ only by FP32 accumulation order.  With ``rounding=False``
everything is exact FP64 and the gradients are the exact derivatives of the
loss (pinned by finite differences).
"""
from __future__ import annotations

import numpy as np

TAPS = [(dy, dx) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]
SHAPES = ((4, 16), (16, 16), (16, 2))  # (Cin, Cout) of the three layers
MARGIN = 3  # receptive-field radius of three 3x3 layers: the loss skips this border


def bf16(x) -> np.ndarray:
    """Round to BF16 (nearest, ties to even) from the FP32 value; returns float64."""
    a = np.asarray(x, dtype=np.float32)
    bits = a.view(np.uint32).astype(np.uint64)
    bits = (bits + 0x7FFF + ((bits >> 16) & 1)) & 0xFFFF0000
    return bits.astype(np.uint32).view(np.float32).astype(np.float64)


def _r(x, rounding):
    return bf16(x) if rounding else np.asarray(x, dtype=np.float64)


def conv(x: np.ndarray, w: np.ndarray) -> np.ndarray:
    """3x3 'same' convolution (correlation) with zero padding, FP64."""
    B, H, W, _ = x.shape
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (0, 0)))
    y = np.zeros((B, H, W, w.shape[2]))
    for t, (dy, dx) in enumerate(TAPS):
        y += xp[:, 1 + dy:1 + dy + H, 1 + dx:1 + dx + W, :] @ w[t]
    return y


def conv_adjoint(dy: np.ndarray, w: np.ndarray) -> np.ndarray:
    """Adjoint of conv in x: dx[b, i, j, c] = sum_{t, o} dy[b, i - dy_t, j - dx_t, o] w[t, c, o]."""
    B, H, W, _ = dy.shape
    gp = np.pad(dy, ((0, 0), (1, 1), (1, 1), (0, 0)))
    dx = np.zeros((B, H, W, w.shape[1]))
    for t, (ey, ex) in enumerate(TAPS):
        dx += gp[:, 1 - ey:1 - ey + H, 1 - ex:1 - ex + W, :] @ w[t].T
    return dx


def weight_grad(x: np.ndarray, dy: np.ndarray) -> np.ndarray:
    """Gradient of <conv(x, w), dy> in w: dw[t, c, o] = sum_p x[p + off_t, c] dy[p, o]."""
    B, H, W, cin = x.shape
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (0, 0)))
    dw = np.zeros((9, cin, dy.shape[3]))
    for t, (ey, ex) in enumerate(TAPS):
        xs = xp[:, 1 + ey:1 + ey + H, 1 + ex:1 + ex + W, :].reshape(-1, cin)
        dw[t] = xs.T @ dy.reshape(-1, dy.shape[3])
    return dw


def init_params(seed: int = 2024) -> list[np.ndarray]:
    """He-normal initial weights (FP64 values; the GPU draws its own, see tests)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return [rng.standard_normal((9, ci, co)) * np.sqrt(2.0 / (9 * ci)) for ci, co in SHAPES]


def forward(params, x, rounding=True):
    """Returns (output, cache) with cache = the activations each layer consumed."""
    acts = []
    h = np.asarray(x, dtype=np.float64)
    for l, w in enumerate(params):
        a = _r(h, rounding)
        acts.append(a)
        h = conv(a, _r(w, rounding))
        if l < 2:
            h = np.maximum(h, 0.0)
    return h, acts


def inner_mask(H: int, W: int) -> np.ndarray:
    m = np.zeros((H, W))
    m[MARGIN:H - MARGIN, MARGIN:W - MARGIN] = 1.0
    return m


def loss_and_grads(params, x, target, rounding=True):
    """L = sum over inner pixels and channels of (y - t)^2 / (2 n), n = their count;
    gradients of L in the weights by back-propagation (BF16 operands as the GPU)."""
    y, acts = forward(params, x, rounding)
    B, H, W, C = y.shape
    m = inner_mask(H, W)[None, :, :, None]
    n = B * int(m.sum()) * C
    diff = (y - target) * m
    loss = float((diff ** 2).sum() / (2.0 * n))
    g = diff / n
    grads = [None, None, None]
    for l in (2, 1, 0):
        gr = _r(g, rounding)
        grads[l] = weight_grad(acts[l], gr)
        if l > 0:
            g = conv_adjoint(gr, _r(params[l], rounding))
            g = g * (acts[l] > 0.0)  # ReLU of the layer below (its output is acts[l])
    return loss, grads


def adam_step(params, grads, state, lr, step, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (bias-corrected) of FP64 master weights; `state` holds
    (m, v) per layer and is updated in place; step counts from 1."""
    out = []
    for l, (w, g) in enumerate(zip(params, grads)):
        m, v = state[l]
        m[:] = beta1 * m + (1.0 - beta1) * g
        v[:] = beta2 * v + (1.0 - beta2) * g * g
        mh = m / (1.0 - beta1 ** step)
        vh = v / (1.0 - beta2 ** step)
        out.append(w - lr * mh / (np.sqrt(vh) + eps))
    return out
