"""Pins for the FP64 U-Net oracle (warm start of the series, Section 2.2): library correlation,
adjoint identities and finite differences."""
import numpy as np
import scipy.signal as ss

from oracle import unet as U


def rng(seed=0):
    return np.random.default_rng(seed)


def test_conv3x3_is_scipy_correlation():
    r = rng(1)
    x = r.standard_normal((2, 7, 9, 3))
    w = r.standard_normal((3, 3, 3, 4))
    b = r.standard_normal(4)
    y = U.conv3x3(x, w, b)
    for bb in range(2):
        for o in range(4):
            ref = sum(ss.correlate2d(x[bb, :, :, c], w[:, :, c, o], mode="same") for c in range(3)) + b[o]
            assert np.allclose(y[bb, :, :, o], ref, atol=1e-12)


def test_conv3x3_backward_adjoint_and_finite_differences():
    r = rng(2)
    x = r.standard_normal((2, 6, 5, 3))
    w = r.standard_normal((3, 3, 3, 4))
    b = r.standard_normal(4)
    g = r.standard_normal((2, 6, 5, 4))
    dx, dw, db = U.conv3x3_backward(x, w, g)
    # <conv(x) - b, g> is linear in x and in w: the backward pass is its exact adjoint
    lin = np.sum((U.conv3x3(x, w, b) - b) * g)
    assert abs(lin - np.sum(x * dx)) <= 1e-10 * abs(lin)
    assert abs(lin - np.sum(w * dw)) <= 1e-10 * abs(lin)
    assert np.allclose(db, g.sum(axis=(0, 1, 2)))


def test_pool_and_upsample_adjoints():
    r = rng(3)
    x = r.standard_normal((2, 8, 6, 3))
    y = r.standard_normal((2, 4, 3, 3))
    assert abs(np.sum(U.avgpool2(x) * y) - np.sum(x * U.avgpool2_backward(y))) < 1e-12
    assert abs(np.sum(U.upsample2(y) * x) - np.sum(y * U.upsample2_backward(x))) < 1e-12


def test_unet_gradient_matches_finite_differences():
    """Full network (3 levels, base 2) at 8x8: <grad L, d> equals the central difference of L along d."""
    r = rng(4)
    L, base = 3, 2
    theta = U.he_init(L, base, 4, 2, seed=5) + 0.05 * r.standard_normal(U.param_count(L, base))
    x = r.standard_normal((2, 8, 8, 4))
    t = r.standard_normal((2, 8, 8, 2))
    net = U.UNet(theta, L, base)
    loss, dout = U.mse(net.forward(x), t)
    grad = net.backward(dout)
    for k in range(3):
        d = r.standard_normal(theta.size)
        eps = 1e-6
        lp = U.mse(U.UNet(theta + eps * d, L, base).forward(x), t)[0]
        lm = U.mse(U.UNet(theta - eps * d, L, base).forward(x), t)[0]
        fd = (lp - lm) / (2 * eps)
        assert abs(fd - grad @ d) <= 1e-6 * max(abs(fd), 1e-8)


def test_unet_input_gradient_and_shapes():
    L, base = 4, 2
    assert U.param_count(L, base) == sum(k * k * ci * co + co for _, k, ci, co in U.layer_shapes(L, base))
    names = [s[0] for s in U.layer_shapes(L, base)]
    assert names == ["e0a", "e0b", "e1a", "e1b", "e2a", "e2b", "e3a", "e3b", "d2a", "d2b", "d1a", "d1b", "d0a",
                     "d0b", "head"]
    net = U.UNet(U.he_init(L, base), L, base)
    y = net.forward(np.ones((1, 16, 16, 4)))
    assert y.shape == (1, 16, 16, 2)


def test_bf16_rounding():
    one = 1.0
    assert U.bf16_round(one + 2.0 ** -8) == one                  # tie rounds to even (mantissa 0)
    assert U.bf16_round(one + 3 * 2.0 ** -8) == one + 2.0 ** -6  # tie rounds to even (up)
    assert U.bf16_round(one + 2.0 ** -7) == one + 2.0 ** -7      # representable
    assert U.bf16_round(-2.5) == -2.5
    x = rng(6).standard_normal(1000)
    assert np.all(np.abs(U.bf16_round(x) - x) <= (2.0 ** -8 + 2.0 ** -24) * np.abs(x))   # unit roundoff 2^-8


def _golden(name):
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", name)
    vals = {}
    for line in open(path):
        if line.strip() and not line.startswith("#"):
            k, v = line.split()[:2]
            vals[k] = float(v)
    return vals


def test_adam_two_steps_hand_worked():
    """Two steps on one parameter against the hand-worked values (moments, bias correction, update)."""
    g = _golden("adam_two_steps.txt")
    p, m, v = U.adam_step(np.array([1.0]), np.array([0.5]), np.zeros(1), np.zeros(1), 1, 0.1)
    for k, x in (("m1", m[0]), ("v1", v[0]), ("p1", p[0])):
        assert abs(x - g[k]) <= 1e-14 * abs(g[k]), k
    p, m, v = U.adam_step(p, np.array([-0.25]), m, v, 2, 0.1)
    for k, x in (("m2", m[0]), ("v2", v[0]), ("p2", p[0])):
        assert abs(x - g[k]) <= 1e-14 * abs(g[k]), k


def test_adam_constant_gradient_closed_form():
    """With a constant gradient g the bias-corrected moments are exactly g and g^2 at every step, so each
    step moves p by lr g / (|g| + eps): after t steps p = p0 - t lr g / (|g| + eps).  A missing or wrong bias
    correction breaks this at the first steps."""
    r = rng(7)
    g = r.standard_normal(50) * 10.0 ** r.uniform(-3, 2, 50)
    p0 = r.standard_normal(50)
    p, m, v = p0.copy(), np.zeros(50), np.zeros(50)
    for t in range(1, 8):
        p, m, v = U.adam_step(p, g, m, v, t, 0.01)
        assert np.allclose(p, p0 - t * 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-13)
