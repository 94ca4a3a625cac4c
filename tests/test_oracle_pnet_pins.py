"""Pins for the oracle of the paper's own network (Sec. 2.5, Fig. 5), each
against something other than the oracle's own loops:

* the circular convolution equals an FFT circular cross-correlation (numpy's
  FFT, a separate algorithm), and a delta kernel is np.roll's shift;
* hand-set weights make the whole forward pass a closed form written with
  numpy's reshape/roll/max, which fixes the row-major reshape of the input
  and of the pooled values, the pooling axis (positions, not channels),
  every ReLU, the hidden layer and the dropout scaling;
* the gradient agrees with central finite differences of the loss on a
  reduced network, with and without a dropout mask;
* a tie in a global max-pool routes the gradient to the first position;
* the full network has the parameter count of the stated readings.
"""
import numpy as np
import pytest

import oracle

SMALL = dict(S=4, F1=3, F2=16, F3=2, F4=5, K1=3, K2=3, H=4)


def _circ_xcorr_fft(x, w):
    """y[f] = sum_i xcorr_circ(x[i], w[f, i]) with the kernel centred, by FFT."""
    ci, S, _ = x.shape
    co, _, K, _ = w.shape
    p = (K - 1) // 2
    y = np.zeros((co, S, S))
    for f in range(co):
        for i in range(ci):
            ker = np.zeros((S, S))
            for u in range(K):
                for v in range(K):
                    ker[(u - p) % S, (v - p) % S] += w[f, i, u, v]
            # cross-correlation: y[r, c] = sum_{a, b} ker[a, b] x[r + a, c + b]
            y[f] += np.real(np.fft.ifft2(np.fft.fft2(x[i]) * np.conj(np.fft.fft2(ker))))
    return y


@pytest.mark.parametrize("ci,co,K,S", [(1, 3, 3, 16), (4, 2, 5, 16), (3, 2, 5, 4), (2, 3, 3, 5)])
def test_conv2d_circ_equals_fft_xcorr(ci, co, K, S):
    rng = np.random.default_rng(ci * 100 + co * 10 + K)
    x = rng.standard_normal((ci, S, S))
    w = rng.standard_normal((co, ci, K, K))
    b = rng.standard_normal(co)
    y = oracle.pnet_conv2d_circ(x, w, b)
    np.testing.assert_allclose(y, _circ_xcorr_fft(x, w) + b[:, None, None], rtol=0, atol=1e-11)


def test_delta_kernel_is_circular_shift():
    rng = np.random.default_rng(5)
    x = rng.standard_normal((1, 16, 16))
    for u, v in [(0, 0), (4, 1), (2, 2), (0, 4)]:
        w = np.zeros((1, 1, 5, 5))
        w[0, 0, u, v] = 1.0
        y = oracle.pnet_conv2d_circ(x, w, np.zeros(1))
        # y[r, c] = x[r + u - 2, c + v - 2]
        np.testing.assert_array_equal(y[0], np.roll(x[0], (2 - u, 2 - v), axis=(0, 1)))


def _hand_params():
    """Weights that turn the reduced network into a closed form."""
    c = SMALL
    p = np.zeros(oracle.pnet_nparams(c))
    n = oracle.pnet_split(p, c)
    n["w1"][0, 0, 1, 1] = 1.0          # a1[0] = relu(x)
    n["w1"][1, 0, 1, 1] = -1.0         # a1[1] = relu(-x)
    n["w1"][2, 0, 1, 2] = 1.0          # a1[2] = relu(right neighbour of x)
    n["b1"][2] = -0.25
    for f in range(16):                # z2[f] = (f+1) a1[0] - 0.5 a1[1] + (f % 3) a1[2](shifted down)
        n["w2"][f, 0, 1, 1] = f + 1.0
        n["w2"][f, 1, 1, 1] = -0.5
        n["w2"][f, 2, 0, 1] = float(f % 3)
        n["b2"][f] = -3.0 if f == 5 else 0.01 * f
    n["w3"][0, 0, 1, 1] = 1.0          # z3[0] = image + its right neighbour
    n["w3"][0, 0, 1, 2] = 1.0
    n["w3"][1, 0, 2, 1] = -1.0         # z3[1] = 2 - the lower neighbour
    n["b3"][1] = 2.0
    for f in range(5):                 # z4[f] = a3[0] (f=0..2 shifted) - (f - 2) a3[1]
        n["w4"][f, 0, 1, 1 + (f % 2)] = 1.0
        n["w4"][f, 1, 1, 1] = -(f - 2.0)
        n["b4"][f] = -0.5 * f
    n["w5"][:] = np.arange(20).reshape(4, 5) * 0.1 - 0.9
    n["b5"][:] = [0.3, -40.0, 0.0, 1.0]
    n["w6"][:] = [1.0, 2.0, -1.5, 0.25]
    n["b6"][0] = -0.125
    return p


def _closed_form(x, mask=None):
    relu = lambda a: np.maximum(a, 0.0)
    img = x.reshape(4, 4)                                   # row-major reshape of the input
    a0, a1 = relu(img), relu(-img)
    a2 = relu(np.roll(img, -1, axis=1) - 0.25)              # right neighbour
    g1 = np.empty(16)
    for f in range(16):
        b = -3.0 if f == 5 else 0.01 * f
        z = (f + 1) * a0 - 0.5 * a1 + (f % 3) * np.roll(a2, 1, axis=0) + b
        g1[f] = relu(z.max())                               # max over positions, then ReLU
    im2 = g1.reshape(4, 4)                                  # pooled values, row-major
    a3_0 = relu(im2 + np.roll(im2, -1, axis=1))
    a3_1 = relu(2.0 - np.roll(im2, -1, axis=0))
    g2 = np.empty(5)
    for f in range(5):
        sh = np.roll(a3_0, -(f % 2), axis=1)
        g2[f] = relu((sh - (f - 2.0) * a3_1 - 0.5 * f).max())
    W5 = np.arange(20).reshape(4, 5) * 0.1 - 0.9
    h = relu(W5 @ g2 + np.array([0.3, -40.0, 0.0, 1.0]))
    if mask is not None:
        h = h * mask
    return float(np.array([1.0, 2.0, -1.5, 0.25]) @ h - 0.125), g1, g2


def test_forward_closed_form_with_hand_set_weights():
    p = _hand_params()
    rng = np.random.default_rng(11)
    x = rng.standard_normal((6, 16))
    mask = np.where(rng.random((6, 4)) < 0.5, 0.0, 2.0)
    got = oracle.pnet_forward(p, x, SMALL)
    got_m = oracle.pnet_forward(p, x, SMALL, mask=mask)
    for b in range(6):
        want, g1, g2 = _closed_form(x[b])
        assert got[b] == pytest.approx(want, rel=1e-12, abs=1e-12)
        assert got_m[b] == pytest.approx(_closed_form(x[b], mask[b])[0], rel=1e-12, abs=1e-12)
        og1, og2, _ = oracle.pnet_features(p, x[b], SMALL)
        np.testing.assert_allclose(og1, g1, rtol=1e-13, atol=1e-13)
        np.testing.assert_allclose(og2, g2, rtol=1e-13, atol=1e-13)
    # a filter whose maximum is not positive pools to 0 (ReLU before the pool)
    assert np.all(og1 >= 0.0)


@pytest.mark.parametrize("with_mask", [False, True])
def test_gradient_matches_central_differences(with_mask):
    c = SMALL
    rng = np.random.default_rng(21 + with_mask)
    npar = oracle.pnet_nparams(c)
    p = rng.standard_normal(npar) * 0.5
    x = rng.standard_normal((3, 16))
    y = np.array([1.0, 0.0, 1.0])
    mask = np.where(rng.random((3, 4)) < 0.5, 0.0, 2.0) if with_mask else None
    loss, g = oracle.pnet_loss_grad(p, x, y, c, mask)
    assert np.isfinite(loss)
    idx = rng.choice(npar, 120, replace=False)
    h = 1e-6
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        lp, _ = oracle.pnet_loss_grad(pp, x, y, c, mask)
        lm, _ = oracle.pnet_loss_grad(pm, x, y, c, mask)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_pool_tie_routes_to_first_position():
    # identity network on a 4x4 image; conv1 is 3x3 with only its centre tap
    # set, so the gradient of its right-hand tap reads the right neighbour of
    # the position the first pool routed to
    c = dict(S=4, F1=1, F2=16, F3=1, F4=1, K1=3, K2=1, H=1)
    p = np.zeros(oracle.pnet_nparams(c))
    n = oracle.pnet_split(p, c)
    n["w1"][0, 0, 1, 1] = 1.0
    n["w2"][:, 0, 1, 1] = 1.0          # every z2[f] = relu(x)
    n["w3"][0, 0, 0, 0] = 1.0
    n["w4"][0, 0, 0, 0] = 1.0
    n["w5"][0, 0] = 1.0
    n["w6"][0] = 1.0
    x = np.zeros((1, 16))
    x[0, [3, 9]] = 2.0                 # tied maxima at (0, 3) and (2, 1)
    x[0, 0] = 0.5                      # right neighbour of (0, 3), wrapping round
    x[0, 10] = -0.7                    # right neighbour of (2, 1)
    _, g = oracle.pnet_loss_grad(p, x, np.array([0.0]), c)
    gs = oracle.pnet_split(g, c)
    sig = 1.0 / (1.0 + np.exp(-2.0))   # logit 2, label 0
    # the pooled image is all 2s, so the second pool routes to position 0:
    # only filter 0 of the first pool carries gradient
    np.testing.assert_allclose(gs["w2"][:, 0, 1, 1], [sig * 2.0] + [0.0] * 15, rtol=1e-12, atol=0)
    # and that filter routed to (0, 3), the first of the tied positions
    assert gs["w1"][0, 0, 1, 2] == pytest.approx(sig * 0.5, rel=1e-12)
    assert gs["w1"][0, 0, 1, 1] == pytest.approx(sig * 2.0, rel=1e-12)


def test_full_network_parameter_count():
    # conv 1x3x3x128 + 128x3x3x256 + 1x5x5x128 + 128x5x5x256 (+ biases), 256 -> 128 -> 1
    want = (128 * 9 + 128) + (256 * 128 * 9 + 256) + (128 * 25 + 128) + (256 * 128 * 25 + 256) \
        + (128 * 256 + 128) + (128 + 1)
    assert oracle.pnet_nparams() == want == 1_152_257
