"""Learned preconditioner of the solver: a small 4D convolutional network (oracle; FP64).

The paper leaves the linear solver open ("Solve Ay = z", Algorithm 1); the
build adds a learned right preconditioner M(r) ~ D^-1 r for FGMRES.  Network
(readings, listed with the design notes): three 4D convolutions with 3^4 taps
over the lattice, 24 -> 48 -> 48 -> 24 real channels (real and imaginary
parts of the 12 spin-colour components: channel 2c + part), ReLU after the
first two layers, no bias (so M is positively homogeneous: M(a r) = a M(r)
for a > 0), circular (periodic) padding on the 4D torus.

Layouts: activations [batch][V][C] with sites in lexicographic order (x
fastest); weights of a layer [81][Cout][Cin] with tap
d = (dx+1) + 3 (dy+1) + 9 (dz+1) + 27 (dt+1), so that
out[x][o] = sum_d sum_i W[d][o][i] in[x + d][i].

Loss: relative squared error sum_b ||M(r_b) - e_b||^2 / ||e_b||^2 / nbatch.
Optimiser: Adam (Kingma and Ba 2015) with bias correction.
"""
from __future__ import annotations

import numpy as np

CHANNELS = (24, 48, 48, 24)
NTAP = 81


def taps():
    """Tap offsets (dx, dy, dz, dt) in tap-index order."""
    out = []
    for t in range(NTAP):
        out.append((t % 3 - 1, (t // 3) % 3 - 1, (t // 9) % 3 - 1, (t // 27) % 3 - 1))
    return out


def shift(a: np.ndarray, L, d) -> np.ndarray:
    """b[..., x, :] = a[..., x + d, :] on the periodic lattice (a: [..., V, C])."""
    Lx, Ly, Lz, Lt = L
    lead = a.shape[:-2]
    C = a.shape[-1]
    g = a.reshape(lead + (Lt, Lz, Ly, Lx, C))
    n = len(lead)
    g = np.roll(g, shift=(-d[3], -d[2], -d[1], -d[0]), axis=(n, n + 1, n + 2, n + 3))
    return g.reshape(lead + (Lx * Ly * Lz * Lt, C))


def conv(a: np.ndarray, W: np.ndarray, L) -> np.ndarray:
    """One layer: out[b][x][o] = sum_d sum_i W[d][o][i] a[b][x + d][i]."""
    out = np.zeros(a.shape[:-1] + (W.shape[1],))
    for t, d in enumerate(taps()):
        out += shift(a, L, d) @ W[t].T
    return out


def conv_backward(a: np.ndarray, W: np.ndarray, gout: np.ndarray, L):
    """Gradients of sum(gout * conv(a, W)) with respect to a and W."""
    ga = np.zeros_like(a)
    gW = np.zeros_like(W)
    for t, d in enumerate(taps()):
        sa = shift(a, L, d)
        gW[t] = np.einsum("bxo,bxi->oi", gout, sa)
        # out[x] uses a[x + d]: the gradient flows back to site y = x + d
        ga += shift(gout @ W[t], L, (-d[0], -d[1], -d[2], -d[3]))
    return ga, gW


def init_weights(seed: int, scale: float = 1.0):
    """He-normal initial weights (fan-in 81 Cin), seeded."""
    rs = np.random.default_rng(seed)
    Ws = []
    for l in range(3):
        cin, cout = CHANNELS[l], CHANNELS[l + 1]
        std = scale * np.sqrt(2.0 / (NTAP * cin))
        Ws.append(rs.standard_normal((NTAP, cout, cin)) * std)
    return Ws


def forward(x: np.ndarray, Ws, L, skip: float = 0.0):
    """Preconditioner output M(x) = net(x) + skip * x and the activations
    needed by the backward pass.

    x: [batch][V][24].  Returns (y, cache) with cache = (x, h1, a1, h2, a2).
    skip = 1 / (4 + m), the inverse of the Wilson matrix's diagonal, makes M
    the point-Jacobi inverse plus a learned correction.
    """
    h1 = conv(x, Ws[0], L)
    a1 = np.maximum(h1, 0.0)
    h2 = conv(a1, Ws[1], L)
    a2 = np.maximum(h2, 0.0)
    y = conv(a2, Ws[2], L) + skip * x
    return y, (x, h1, a1, h2, a2)


def loss_and_grad(x: np.ndarray, e: np.ndarray, Ws, L, skip: float = 0.0):
    """Relative squared error of M(x) against e and its gradient with respect
    to the weights (the skip term has no weights)."""
    y, (x0, h1, a1, h2, a2) = forward(x, Ws, L, skip)
    diff = y - e
    en = np.sum(e * e, axis=(1, 2))
    nb = x.shape[0]
    loss = float(np.sum(np.sum(diff * diff, axis=(1, 2)) / en) / nb)
    gy = 2.0 * diff / en[:, None, None] / nb
    ga2, gW3 = conv_backward(a2, Ws[2], gy, L)
    gh2 = ga2 * (h2 > 0)
    ga1, gW2 = conv_backward(a1, Ws[1], gh2, L)
    gh1 = ga1 * (h1 > 0)
    _, gW1 = conv_backward(x0, Ws[0], gh1, L)
    return loss, [gW1, gW2, gW3]


def adam_step(Ws, grads, state, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update in place; state = dict(t, m, v)."""
    state["t"] += 1
    t = state["t"]
    for i, (W, g) in enumerate(zip(Ws, grads)):
        state["m"][i] = b1 * state["m"][i] + (1 - b1) * g
        state["v"][i] = b2 * state["v"][i] + (1 - b2) * g * g
        mh = state["m"][i] / (1 - b1 ** t)
        vh = state["v"][i] / (1 - b2 ** t)
        W -= lr * mh / (np.sqrt(vh) + eps)


def adam_state(Ws):
    return {"t": 0, "m": [np.zeros_like(W) for W in Ws], "v": [np.zeros_like(W) for W in Ws]}


def spinor_to_channels(psi: np.ndarray) -> np.ndarray:
    """Canonical complex spinors [batch][V*12] -> real channels [batch][V][24]."""
    b = psi.shape[0]
    z = psi.reshape(b, -1, 12)
    out = np.empty(z.shape[:2] + (24,))
    out[..., 0::2] = z.real
    out[..., 1::2] = z.imag
    return out


def channels_to_spinor(a: np.ndarray) -> np.ndarray:
    return (a[..., 0::2] + 1j * a[..., 1::2]).reshape(a.shape[0], -1)
