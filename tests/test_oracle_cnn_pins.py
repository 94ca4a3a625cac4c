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
