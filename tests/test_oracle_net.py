"""Pins of the warm-start network reference (oracle/net.py).

The convolution is checked against scipy's direct N-d correlation, the
backward pass against central finite differences of the loss, and Adam
against its closed-form first step.
"""

import numpy as np
import pytest
from scipy import signal

from oracle import net


def _conv_scipy(x, W, b, stride):
    """Direct correlation by scipy, one (co, ci) pair at a time."""
    co_n = W.shape[0]
    full = np.stack([sum(signal.correlate(np.pad(x[ci], 1), W[co, ci], mode="valid", method="direct")
                         for ci in range(x.shape[0])) + b[co] for co in range(co_n)])
    return full[:, ::stride, ::stride, ::stride]


@pytest.mark.parametrize("stride,shape", [(1, (5, 4, 6)), (2, (5, 4, 7)), (2, (6, 6, 6))])
def test_conv_matches_scipy(stride, shape):
    rng = np.random.default_rng(1)
    x = rng.normal(size=(3,) + shape)
    W = rng.normal(size=(4, 3, 3, 3, 3))
    b = rng.normal(size=4)
    got = net.conv3d(x, W, b, stride)
    assert got.shape == (4,) + tuple((n + stride - 1) // stride for n in shape)
    np.testing.assert_allclose(got, _conv_scipy(x, W, b, stride), rtol=1e-12, atol=1e-12)


def test_conv_single_tap_is_shift():
    """A kernel with one non-zero tap at (dz,dy,dx) shifts the input by tap-1
    with zero fill (the padding convention)."""
    x = np.arange(4 * 5 * 6, dtype=float).reshape(1, 4, 5, 6)
    W = np.zeros((1, 1, 3, 3, 3))
    W[0, 0, 2, 0, 1] = 1.0
    y = net.conv3d(x, W, np.zeros(1))
    ref = np.zeros_like(x)
    ref[0, :-1, 1:, :] = x[0, 1:, :-1, :]
    np.testing.assert_array_equal(y, ref)


def test_upsample_and_adjoint():
    rng = np.random.default_rng(2)
    a = rng.normal(size=(2, 3, 2, 4))
    up = net.upsample(a, (5, 4, 7))
    assert up[1, 4, 3, 6] == a[1, 2, 1, 3]
    assert up[0, 1, 0, 1] == a[0, 0, 0, 0]
    dy = rng.normal(size=up.shape)
    # <up(a), dy> == <a, up^T(dy)>
    np.testing.assert_allclose(np.sum(up * dy), np.sum(a * net.upsample_backward(dy, a.shape[1:])),
                               rtol=1e-12)


def test_conv_backward_adjoint():
    """<conv(x) - b, dy> == <x, dx> and == <W, dW> (the convolution is bilinear)."""
    rng = np.random.default_rng(3)
    for stride in (1, 2):
        x = rng.normal(size=(3, 5, 6, 5))
        W = rng.normal(size=(2, 3, 3, 3, 3))
        b = rng.normal(size=2)
        y = net.conv3d(x, W, b, stride)
        dy = rng.normal(size=y.shape)
        dx, dW, db = net.conv3d_backward(x, W, dy, stride)
        lin = np.sum((y - b[:, None, None, None]) * dy)
        np.testing.assert_allclose(lin, np.sum(x * dx), rtol=1e-11)
        np.testing.assert_allclose(lin, np.sum(W * dW), rtol=1e-11)
        np.testing.assert_allclose(db, dy.reshape(2, -1).sum(1), rtol=1e-12)


def test_network_gradient_finite_differences():
    rng = np.random.default_rng(4)
    p = net.init_params(rng, scale_head=1.0)
    for k in p:
        if k.endswith(".b"):
            p[k] = rng.normal(scale=0.1, size=p[k].shape)
    x = rng.normal(size=(8, 5, 6, 7))
    target = rng.normal(size=(3, 5, 6, 7))

    def loss_of(pp, xx):
        return net.mse_loss(net.forward(pp, xx)[0], target)[0]

    out, acts = net.forward(p, x)
    _, dout = net.mse_loss(out, target)
    g = net.backward(p, acts, dout)
    eps = 1e-6
    checked = 0
    for name in ["e0a.W", "e1a.W", "e2a.W", "e2.b", "u1.W", "d1.W", "u0.b", "d0.W", "head.W", "head.b"]:
        flat = p[name].reshape(-1)
        for idx in rng.choice(flat.size, size=3, replace=False):
            old = flat[idx]
            flat[idx] = old + eps
            lp = loss_of(p, x)
            flat[idx] = old - eps
            lm = loss_of(p, x)
            flat[idx] = old
            fd = (lp - lm) / (2 * eps)
            an = g[name].reshape(-1)[idx]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)), (name, idx, fd, an)
            checked += 1
    xf = x.reshape(-1)
    for idx in rng.choice(xf.size, size=5, replace=False):
        old = xf[idx]
        xf[idx] = old + eps
        lp = loss_of(p, x)
        xf[idx] = old - eps
        lm = loss_of(p, x)
        xf[idx] = old
        fd = (lp - lm) / (2 * eps)
        assert abs(fd - g["x"].reshape(-1)[idx]) <= 1e-6 * max(1.0, abs(fd))
    assert checked == 30


def test_adam_first_step_is_signed_lr():
    """With zero moments, the bias-corrected first step is lr * g / (|g| + eps)."""
    g = {"w": np.array([0.5, -2.0, 1e-3])}
    p = {"w": np.zeros(3)}
    m = {"w": np.zeros(3)}
    v = {"w": np.zeros(3)}
    p, m, v = net.adam_step(p, g, m, v, 1, lr=0.01, eps=0.0)
    np.testing.assert_allclose(p["w"], [-0.01, 0.01, -0.01], rtol=1e-12)


def test_training_reduces_loss():
    """A few Adam steps on one sample reduce the loss (sanity of the loop)."""
    rng = np.random.default_rng(5)
    p = net.init_params(rng)
    x = rng.normal(size=(8, 6, 6, 6))
    target = 0.5 * x[:3]
    m = {k: np.zeros_like(v) for k, v in p.items()}
    v = {k: np.zeros_like(val) for k, val in p.items()}
    losses = []
    for t in range(1, 21):
        out, a = net.forward(p, x)
        loss, dout = net.mse_loss(out, target)
        losses.append(loss)
        g = net.backward(p, a, dout)
        g.pop("x")
        p, m, v = net.adam_step(p, g, m, v, t)
    assert losses[-1] < 0.7 * losses[0]


def test_bf16_round():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -3.140625, 1e-3], np.float32)
    r = net.bf16_round(vals)
    # 1 + 2^-8 is a tie -> even (1.0); 1 + 3*2^-8 is a tie -> 1 + 2^-6 (even mantissa)
    assert r[0] == 1.0 and r[1] == 1.0 and r[2] == 1.0 + 2 ** -6
    assert r[3] == -3.140625
    assert abs(r[4] - 1e-3) <= 1e-3 * 2 ** -8


def _hand(name):
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "hand_examples.json")) as fh:
        return json.load(fh)[name]


def test_adam_three_steps_match_hand_computation():
    """Three Adam steps on one scalar with gradients 0.5, -2, 1e-3, worked out
    by hand (tests/golden/hand_examples.json): pins the moment recursions
    (m and v decayed and carried over) and both bias corrections, which the
    first step from zero moments cannot distinguish."""
    h = _hand("adam_three_steps")
    p = {"w": np.array([h["p0"]])}
    m = {"w": np.zeros(1)}
    v = {"w": np.zeros(1)}
    for t, g in enumerate(h["grads"], start=1):
        p, m, v = net.adam_step(p, {"w": np.array([g])}, m, v, t, lr=h["lr"], b1=h["beta1"],
                                b2=h["beta2"], eps=h["eps"])
        assert abs(m["w"][0] - h["m"][t - 1]) <= 1e-15
        assert abs(v["w"][0] - h["v"][t - 1]) <= 1e-17
        assert abs(p["w"][0] - h["p"][t - 1]) <= 1e-14, (t, p["w"][0], h["p"][t - 1])


def test_mse_loss_matches_hand_computation():
    """Loss normalisation: squared error summed over components, averaged over
    nodes (hand example in tests/golden/hand_examples.json)."""
    h = _hand("mse_two_nodes")
    target = np.array(h["target"])
    loss, dout = net.mse_loss(np.zeros_like(target), target)
    assert loss == h["loss"]
    np.testing.assert_array_equal(dout, np.array(h["dout"]))
