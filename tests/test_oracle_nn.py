"""Pins of the oracle's learned-preconditioner network (FP64).

- impulse response: a unit input at one site and channel reproduces the
  weight column of every tap at the expected (periodically wrapped) site,
  fixing the tap convention out[x] = sum_d W[d] in[x + d];
- translation equivariance on the torus and linearity of a layer;
- positive homogeneity of the bias-free ReLU network;
- backward pass against central finite differences of the loss (with and
  without the skip term s x of M(x) = net(x) + s x);
- with all weights zero, M is exactly the scaled identity s x, and the loss
  of the target e = s x is zero;
- Adam's first step equals the closed form lr * g / (|g| + eps).
"""
import numpy as np
import pytest

from oracle import nn
from oracle.lattice import site_index

L = (4, 2, 2, 4)
V = 64


def test_impulse_response_fixes_tap_convention():
    rs = np.random.default_rng(0)
    W = rs.standard_normal((81, 5, 3))
    x0 = (1, 0, 1, 3)
    ci = 2
    a = np.zeros((1, V, 3))
    a[0, site_index(x0, L), ci] = 1.0
    out = nn.conv(a, W, L)
    for t, d in enumerate(nn.taps()):
        x = tuple((x0[m] - d[m]) % L[m] for m in range(4))
        # sites reached by several taps (extent-2 directions) sum their weights
        same = [t2 for t2, d2 in enumerate(nn.taps())
                if tuple((x0[m] - d2[m]) % L[m] for m in range(4)) == x]
        assert np.allclose(out[0, site_index(x, L)], W[same, :, ci].sum(axis=0))


def test_translation_equivariance_and_linearity():
    rs = np.random.default_rng(1)
    W = rs.standard_normal((81, 4, 6))
    a = rs.standard_normal((2, V, 6))
    b = rs.standard_normal((2, V, 6))
    d = (1, 1, 0, 3)
    assert np.allclose(nn.conv(nn.shift(a, L, d), W, L), nn.shift(nn.conv(a, W, L), L, d))
    assert np.allclose(nn.conv(2.0 * a - b, W, L), 2.0 * nn.conv(a, W, L) - nn.conv(b, W, L))


def test_network_positive_homogeneity():
    Ws = nn.init_weights(3)
    x = np.random.default_rng(2).standard_normal((1, V, 24))
    y1, _ = nn.forward(x, Ws, L)
    y2, _ = nn.forward(3.5 * x, Ws, L)
    assert np.allclose(y2, 3.5 * y1, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("skip", [0.0, 0.3])
def test_backward_matches_finite_differences(skip):
    rs = np.random.default_rng(4)
    Ws = nn.init_weights(5)
    x = rs.standard_normal((2, V, 24))
    e = rs.standard_normal((2, V, 24))
    loss, grads = nn.loss_and_grad(x, e, Ws, L, skip)
    h = 1e-6
    for l in range(3):
        for _ in range(6):
            idx = tuple(rs.integers(0, s) for s in Ws[l].shape)
            W0 = Ws[l][idx]
            Ws[l][idx] = W0 + h
            lp, _ = nn.loss_and_grad(x, e, Ws, L, skip)
            Ws[l][idx] = W0 - h
            lm, _ = nn.loss_and_grad(x, e, Ws, L, skip)
            Ws[l][idx] = W0
            fd = (lp - lm) / (2 * h)
            assert abs(fd - grads[l][idx]) <= 1e-6 * max(1.0, abs(fd)) + 1e-8, (l, idx, fd, grads[l][idx])


def test_zero_network_is_scaled_identity():
    rs = np.random.default_rng(9)
    Ws = [np.zeros_like(W) for W in nn.init_weights(1)]
    x = rs.standard_normal((3, V, 24))
    y, _ = nn.forward(x, Ws, L, skip=0.25)
    assert np.array_equal(y, 0.25 * x)
    loss, grads = nn.loss_and_grad(x, 0.25 * x, Ws, L, skip=0.25)
    assert loss == 0.0 and all(not g.any() for g in grads)


def test_adam_first_step_closed_form():
    W = [np.zeros((3, 2))]
    g = [np.array([[1.0, -2.0], [0.5, 0.0], [-3.0, 4.0]])]
    st = nn.adam_state(W)
    nn.adam_step(W, g, st, lr=0.01, eps=1e-8)
    assert np.allclose(W[0], -0.01 * g[0] / (np.abs(g[0]) + 1e-8))


def test_channel_packing_roundtrip():
    rs = np.random.default_rng(6)
    psi = rs.standard_normal((2, 12 * V)) + 1j * rs.standard_normal((2, 12 * V))
    ch = nn.spinor_to_channels(psi)
    assert ch.shape == (2, V, 24)
    assert np.allclose(ch[0, 3, 5], psi[0, 3 * 12 + 2].imag)
    assert np.allclose(nn.channels_to_spinor(ch), psi)
