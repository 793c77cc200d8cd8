"""Plain FP64 U-Net used as a learned warm start of the scattering series.

TEST INFRASTRUCTURE ONLY (see ``oracle/lsop_oracle.py``).

The series of eq. (11) may start from any phi_0 (Section 2.2: the fixed point
does not depend on it).  A small convolutional network maps (velocity,
incident field, frequency) to an estimate of the scattered field
psi - psi0, and the estimate serves as phi_0.  This module is the reference
for the device network: forward pass, backward pass (every parameter
gradient), mean-squared loss and the bf16 rounding that the device applies to
the operands of its matrix products.

Layout: activations are [B][H][W][C] (channels fastest).  A 3x3 layer's
weights are [3][3][Ci][Co] (tap row, tap column, input channel, output
channel) and it computes the zero-padded cross-correlation
    y[b, i, j, o] = bias[o] + sum_{di, dj, c} x[b, i + di - 1, j + dj - 1, c] w[di, dj, c, o].
Topology for `levels` L and base width c (channels c 2^l at level l):
  encoder level l < L - 1: conv3x3 -> ReLU -> conv3x3 -> ReLU (the skip), then
  2x2 average pooling; level L - 1 (bottleneck): two conv3x3 + ReLU;
  decoder level l = L - 2 .. 0: nearest 2x upsampling of the level below,
  concatenation [upsampled, skip] along channels, two conv3x3 + ReLU;
  head: 1x1 convolution to the output channels, no activation.
Parameters are flattened layer by layer in that order, each layer as its
weights (C order) followed by its bias.
"""
from __future__ import annotations

import numpy as np


def bf16_round(a):
    """Round to the nearest bfloat16 (ties to even) through float32, returned as float64."""
    f = np.asarray(a, np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def conv3x3(x, w, b):
    """Zero-padded 3x3 cross-correlation, [B,H,W,Ci] x [3,3,Ci,Co] + [Co] -> [B,H,W,Co]."""
    B, H, W, _ = x.shape
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (0, 0)))
    y = np.zeros((B, H, W, w.shape[3]))
    for di in range(3):
        for dj in range(3):
            y += np.einsum("bhwc,co->bhwo", xp[:, di:di + H, dj:dj + W, :], w[di, dj], optimize=True)
    return y + b


def conv3x3_backward(x, w, dy):
    """Gradients (dx, dw, db) of conv3x3 for the output gradient dy."""
    B, H, W, _ = x.shape
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (0, 0)))
    dxp = np.zeros_like(xp)
    dw = np.zeros_like(w)
    for di in range(3):
        for dj in range(3):
            dxp[:, di:di + H, dj:dj + W, :] += np.einsum("bhwo,co->bhwc", dy, w[di, dj], optimize=True)
            dw[di, dj] = np.einsum("bhwc,bhwo->co", xp[:, di:di + H, dj:dj + W, :], dy, optimize=True)
    return dxp[:, 1:H + 1, 1:W + 1, :], dw, dy.sum(axis=(0, 1, 2))


def conv1x1(x, w, b):
    return np.einsum("bhwc,co->bhwo", x, w, optimize=True) + b


def conv1x1_backward(x, w, dy):
    return (np.einsum("bhwo,co->bhwc", dy, w, optimize=True), np.einsum("bhwc,bhwo->co", x, dy, optimize=True),
            dy.sum(axis=(0, 1, 2)))


def avgpool2(x):
    B, H, W, C = x.shape
    return x.reshape(B, H // 2, 2, W // 2, 2, C).mean(axis=(2, 4))


def avgpool2_backward(dy):
    return np.repeat(np.repeat(dy, 2, axis=1), 2, axis=2) / 4.0


def upsample2(x):
    return np.repeat(np.repeat(x, 2, axis=1), 2, axis=2)


def upsample2_backward(dy):
    B, H, W, C = dy.shape
    return dy.reshape(B, H // 2, 2, W // 2, 2, C).sum(axis=(2, 4))


def layer_shapes(levels=4, base=32, cin=4, cout=2):
    """[(name, kernel size, Ci, Co)] in parameter order."""
    out = []
    ch = [base << l for l in range(levels)]
    prev = cin
    for l in range(levels):
        out.append((f"e{l}a", 3, prev, ch[l]))
        out.append((f"e{l}b", 3, ch[l], ch[l]))
        prev = ch[l]
    for l in range(levels - 2, -1, -1):
        out.append((f"d{l}a", 3, ch[l + 1] + ch[l], ch[l]))
        out.append((f"d{l}b", 3, ch[l], ch[l]))
    out.append(("head", 1, ch[0], cout))
    return out


def param_count(levels=4, base=32, cin=4, cout=2):
    return sum(k * k * ci * co + co for _, k, ci, co in layer_shapes(levels, base, cin, cout))


class UNet:
    """FP64 reference network.  With bf16=True every operand of a convolution product (input activation and
    weights forward; output gradient, weights and input activation backward) is rounded to bfloat16 first, as
    the device's matrix cores take them; sums stay in FP64."""

    def __init__(self, params, levels=4, base=32, cin=4, cout=2, bf16=False):
        self.levels, self.base, self.cin, self.cout, self.bf16 = levels, base, cin, cout, bf16
        self.shapes = layer_shapes(levels, base, cin, cout)
        self.set_params(params)

    def set_params(self, flat):
        flat = np.asarray(flat, np.float64)
        assert flat.size == param_count(self.levels, self.base, self.cin, self.cout)
        self.w, self.b, at = {}, {}, 0
        for name, k, ci, co in self.shapes:
            n = k * k * ci * co
            self.w[name] = flat[at:at + n].reshape((k, k, ci, co) if k == 3 else (ci, co))
            self.b[name] = flat[at + n:at + n + co]
            at += n + co

    def _r(self, a):
        return bf16_round(a) if self.bf16 else a

    def _conv(self, name, x):
        w = self._r(self.w[name])
        return conv3x3(self._r(x), w, self.b[name]) if w.ndim == 4 else conv1x1(self._r(x), w, self.b[name])

    def forward(self, x):
        """Returns the output and keeps what the backward pass needs."""
        c = self.cache = {}
        h = np.asarray(x, np.float64)
        skips = []
        for l in range(self.levels):
            for part in "ab":
                name = f"e{l}{part}"
                c[name + ":in"] = h
                h = np.maximum(self._conv(name, h), 0.0)
                c[name + ":out"] = h
            if l < self.levels - 1:
                skips.append(h)
                h = avgpool2(h)
        for l in range(self.levels - 2, -1, -1):
            h = np.concatenate([upsample2(h), skips[l]], axis=3)
            for part in "ab":
                name = f"d{l}{part}"
                c[name + ":in"] = h
                h = np.maximum(self._conv(name, h), 0.0)
                c[name + ":out"] = h
        c["head:in"] = h
        return self._conv("head", h)

    def _conv_back(self, name, dy):
        # both products of the backward pass take bf16 operands (the output gradient too); the bias
        # gradient sums the unrounded output gradient
        x = self._r(self.cache[name + ":in"])
        w = self._r(self.w[name])
        dyr = self._r(dy)
        dx, dw, _ = conv3x3_backward(x, w, dyr) if w.ndim == 4 else conv1x1_backward(x, w, dyr)
        return dx, dw, dy.sum(axis=(0, 1, 2))

    def backward(self, dout):
        """Gradients of every parameter (flat, parameter order) for the output gradient dout."""
        g = {}
        dx, g["head:w"], g["head:b"] = self._conv_back("head", dout)
        skip_grads = {}
        d = dx
        for l in range(self.levels - 1):
            for part in "ba":
                name = f"d{l}{part}"
                d = d * (self.cache[name + ":out"] > 0)
                d, g[name + ":w"], g[name + ":b"] = self._conv_back(name, d)
            cu = self.base << (l + 1)
            skip_grads[l] = d[..., cu:]
            d = upsample2_backward(d[..., :cu])
        for l in range(self.levels - 1, -1, -1):
            if l < self.levels - 1:
                d = avgpool2_backward(d) + skip_grads[l]
            for part in "ba":
                name = f"e{l}{part}"
                d = d * (self.cache[name + ":out"] > 0)
                d, g[name + ":w"], g[name + ":b"] = self._conv_back(name, d)
        self.dx = d
        out = []
        for name, _, _, _ in self.shapes:
            out += [g[name + ":w"].ravel(), g[name + ":b"].ravel()]
        return np.concatenate(out)


def mse(out, target):
    """Mean squared error over all entries and its gradient with respect to out."""
    diff = np.asarray(out) - np.asarray(target)
    return float(np.mean(diff * diff)), 2.0 * diff / diff.size


def he_init(levels=4, base=32, cin=4, cout=2, seed=0):
    """He-normal weights (std sqrt(2 / fan_in)), zero biases, in parameter order."""
    rng = np.random.default_rng(seed)
    out = []
    for _, k, ci, co in layer_shapes(levels, base, cin, cout):
        out.append(rng.standard_normal(k * k * ci * co) * np.sqrt(2.0 / (k * k * ci)))
        out.append(np.zeros(co))
    return np.concatenate(out)


def adam_step(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba, ICLR 2015, Algorithm 1) in FP64.

    Moments m <- b1 m + (1 - b1) g and v <- b2 v + (1 - b2) g^2, bias-corrected
    by 1 - b1^t and 1 - b2^t (t = 1 at the first step), then
    p <- p - lr m_hat / (sqrt(v_hat) + eps).  Returns (p, m, v) as new arrays.
    """
    p, g = np.asarray(p, np.float64), np.asarray(g, np.float64)
    m = b1 * np.asarray(m, np.float64) + (1.0 - b1) * g
    v = b2 * np.asarray(v, np.float64) + (1.0 - b2) * g * g
    m_hat = m / (1.0 - b1 ** t)
    v_hat = v / (1.0 - b2 ** t)
    return p - lr * m_hat / (np.sqrt(v_hat) + eps), m, v
