"""Pins for the learned scorer's CPU oracle: finite differences, closed forms
and symmetries, none of which retypes the oracle's formulas."""
import math

import numpy as np
import pytest

import oracle
from paper_2312_02063_amd import synth

NP = 312449
F3W, F3B = 312384, 312448


def test_param_count_and_layout():
    assert oracle.cnn_nparams() == NP
    shapes = synth.cnn_param_shapes()
    assert sum(int(np.prod(s)) for s in shapes) == NP


def test_delta_kernel_is_circular_shift():
    rng = np.random.default_rng(0)
    x = rng.normal(size=(2, 3, 16))
    for dx in range(5):
        w = np.zeros((3, 3, 5))
        for c in range(3):
            w[c, c, dx] = 1.0
        y = oracle.conv1d_circ(x, w, np.zeros(3))
        np.testing.assert_array_equal(y, np.roll(x, -(dx - 2), axis=2))


def test_conv_commutes_with_circular_shift():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(1, 4, 32))
    w = rng.normal(size=(6, 4, 5))
    b = rng.normal(size=6)
    y = oracle.conv1d_circ(x, w, b)
    for s in (1, 5, 31):
        ys = oracle.conv1d_circ(np.roll(x, s, axis=2), w, b)
        np.testing.assert_allclose(ys, np.roll(y, s, axis=2), atol=1e-12)


def test_maxpool_routing_by_hand():
    out, idx = oracle.maxpool2(np.array([1.0, 3.0, 2.0, 2.0, -1.0, -5.0, 0.0, 0.0]))
    assert list(out) == [3.0, 2.0, -1.0, 0.0]
    assert list(idx) == [1, 2, 4, 6]          # ties go to the first position


def test_bce_at_zero_logit():
    p = synth.cnn_init(7)
    p[F3W:F3B + 1] = 0.0                      # output layer off: logit 0 for every input
    x = np.random.default_rng(2).normal(size=(5, 256))
    y = np.array([0, 1, 1, 0, 1.0])
    loss, g = oracle.cnn_loss_grad(p, x, y)
    assert loss == pytest.approx(math.log(2.0), rel=1e-15)
    assert g[F3B] == pytest.approx(np.mean(0.5 - y), rel=1e-14)
    np.testing.assert_allclose(oracle.cnn_forward(p, x), 0.0)


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(3)
    p = synth.cnn_init(11)
    p += rng.normal(0, 0.01, p.size)          # non-zero biases
    x = rng.normal(size=(3, 256))
    y = np.array([1.0, 0.0, 1.0])
    _, g = oracle.cnn_loss_grad(p, x, y)
    bounds = [0, 96, 2688, 12992, 33536, 295936, 312384, NP]
    idx = np.concatenate([rng.choice(np.arange(a, b), size=min(20, b - a), replace=False)
                          for a, b in zip(bounds[:-1], bounds[1:])])
    h = 1e-6
    bad = 0
    for i in idx:
        pp = p.copy()
        pp[i] += h
        lp, _ = oracle.cnn_loss_grad(pp, x, y)
        pp[i] -= 2 * h
        lm, _ = oracle.cnn_loss_grad(pp, x, y)
        fd = (lp - lm) / (2 * h)
        if abs(fd - g[i]) > 1e-6 * max(1e-3, abs(g[i])) + 1e-10:
            bad += 1
    assert bad == 0


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(4)
    p = rng.normal(size=100)
    g = rng.normal(size=100)
    m = np.zeros(100)
    v = np.zeros(100)
    p0 = p.copy()
    oracle.adam(p, g, m, v, 1, lr=1e-3)
    np.testing.assert_allclose(p, p0 - 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    np.testing.assert_allclose(m, 0.1 * g, rtol=1e-15)
    np.testing.assert_allclose(v, 0.001 * g * g, rtol=1e-12)


def test_training_reduces_loss():
    # A few Adam steps on a separable toy set lower the loss.
    rng = np.random.default_rng(5)
    x = rng.normal(size=(8, 256))
    y = (np.arange(8) % 2).astype(float)
    x[y == 1, 100:110] -= 3.0
    p = synth.cnn_init(12)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    l0, _ = oracle.cnn_loss_grad(p, x, y)
    for step in range(1, 6):
        _, g = oracle.cnn_loss_grad(p, x, y)
        oracle.adam(p, g, m, v, step, lr=1e-3)
    l1, _ = oracle.cnn_loss_grad(p, x, y)
    assert l1 < l0


def _layout():
    """Offsets of the canonical parameter layout: conv l weight [Cout][Cin][5]
    then bias, then fc weight [out][in] then bias, in network order."""
    shapes = synth.cnn_param_shapes()
    offs, o = [], 0
    for s in shapes:
        offs.append(o)
        o += int(np.prod(s))
    return shapes, offs


def test_dense_head_closed_form():
    """Hand-set weights make the whole network a known piecewise-linear
    function of the input: every convolution passes channel 0 through its
    centre tap (other channels 0), so block 4 holds, in channel 0 only,
    M_p = max(0, max of x over positions 16p..16p+15); the fully connected
    layers then combine the M_p through ReLUs that are active for some inputs
    and not for others. A forward pass that flattened position-major, dropped
    a ReLU, or mixed up a layer's weights or biases gives another value."""
    shapes, offs = _layout()
    p = np.zeros(NP)

    def put(i, idx, v):
        a = p[offs[i]:offs[i] + int(np.prod(shapes[i]))].reshape(shapes[i])
        a[idx] = v

    for layer in range(4):                     # conv weights at even indices, biases odd
        put(2 * layer, (0, 0, 2), 1.0)
    # FC1 (params 8, 9): h1 = relu(W1 a + b1) over the channel-major flatten
    put(8, (0, slice(0, 16)), 1.0)
    put(9, 0, -20.0)
    put(8, (1, 0), 1.0)
    put(8, (1, 1), -1.0)
    put(8, (2, 0), -1.0)
    put(8, (2, 1), 1.0)
    put(8, (3, 5), 2.0)
    put(9, 3, -1.0)
    # FC2 (params 10, 11)
    put(10, (0, 0), 1.0)
    put(10, (0, 1), -2.0)
    put(11, 0, 0.5)
    put(10, (1, 2), 1.0)
    put(10, (1, 0), -1.0)
    put(10, (2, 3), 1.0)
    put(10, (2, 1), 1.0)
    # FC3 (params 12, 13)
    put(12, (0, 0), 1.5)
    put(12, (0, 1), -0.7)
    put(12, (0, 2), 0.25)
    put(13, 0, 0.1)

    rng = np.random.default_rng(21)
    x = rng.normal(size=(64, 256)) * rng.uniform(0.2, 2.0, size=(64, 1))
    relu = lambda v: np.maximum(v, 0.0)          # noqa: E731
    M = relu(x.reshape(64, 16, 16).max(axis=2))  # [input][p]
    h1 = np.stack([relu(M.sum(axis=1) - 20.0), relu(M[:, 0] - M[:, 1]), relu(M[:, 1] - M[:, 0]),
                   relu(2.0 * M[:, 5] - 1.0)], axis=1)
    h2 = np.stack([relu(h1[:, 0] - 2.0 * h1[:, 1] + 0.5), relu(h1[:, 2] - h1[:, 0]),
                   relu(h1[:, 3] + h1[:, 1])], axis=1)
    want = 1.5 * h2[:, 0] - 0.7 * h2[:, 1] + 0.25 * h2[:, 2] + 0.1
    # the inputs exercise both sides of every ReLU that decides the result
    assert (M.sum(axis=1) > 20).any() and (M.sum(axis=1) < 20).any()
    assert ((h1[:, 0] - 2 * h1[:, 1] + 0.5) < 0).any() and ((h1[:, 0] - 2 * h1[:, 1] + 0.5) > 0).any()
    assert ((h1[:, 2] - h1[:, 0]) < 0).any() and ((h1[:, 2] - h1[:, 0]) > 0).any()
    np.testing.assert_allclose(oracle.cnn_forward(p, x), want, rtol=1e-12, atol=1e-12)
