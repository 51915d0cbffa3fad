"""FP64 reference of the small network behind the learned block preconditioner.

Three affine layers with SiLU activations, x -> W3 a(W2 a(W1 x + b1) + b2) + b3,
a(z) = z / (1 + exp(-z)); hidden width 128.  The preconditioner loss for one (u-atom,
o-atom) block with gradient block g, target block G* (tight solve of Eq. precond) and
predicted elementwise scaling c = y[:E] is

    l = 1/2 || c * g - G* ||^2 / scale,

and the guess head y[E] is fitted to a per-block target w by 1/2 (y[E] - w)^2.  Adam
(Kingma and Ba, 2015) updates the parameters.  Plain NumPy, written for checking the GPU
training kernels, not for speed.
"""
from __future__ import annotations

import numpy as np


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


class MLP:
    def __init__(self, n_in: int, n_out: int, width: int = 128, seed: int = 0):
        rng = np.random.default_rng(seed)
        sizes = [n_in, width, width, n_out]
        self.params = []
        for a, b in zip(sizes[:-1], sizes[1:]):
            W = rng.standard_normal((a, b)) * np.sqrt(2.0 / a)
            self.params += [W, np.zeros(b)]

    # -- forward / backward ---------------------------------------------------------------
    def forward(self, X):
        W1, b1, W2, b2, W3, b3 = self.params
        z1 = X @ W1 + b1
        a1 = silu(z1)
        z2 = a1 @ W2 + b2
        a2 = silu(z2)
        y = a2 @ W3 + b3
        return y, (X, z1, a1, z2, a2)

    def backward(self, cache, dy):
        """Gradients of sum(dy * y) with respect to every parameter."""
        X, z1, a1, z2, a2 = cache
        W1, b1, W2, b2, W3, b3 = self.params
        gW3 = a2.T @ dy
        gb3 = dy.sum(0)
        d2 = (dy @ W3.T) * dsilu(z2)
        gW2 = a1.T @ d2
        gb2 = d2.sum(0)
        d1 = (d2 @ W2.T) * dsilu(z1)
        gW1 = X.T @ d1
        gb1 = d1.sum(0)
        return [gW1, gb1, gW2, gb2, gW3, gb3]


def precond_loss(y, g, gstar, w, E, scale=1.0):
    """Loss and dL/dy for the block-scaling head (y[:, :E]) and the guess head (y[:, E])."""
    c = y[:, :E]
    r = c * g - gstar
    lw = y[:, E] - w
    loss = 0.5 * np.sum(r * r) / scale + 0.5 * np.sum(lw * lw)
    dy = np.zeros_like(y)
    dy[:, :E] = r * g / scale
    dy[:, E] = lw
    return loss, dy


class Adam:
    def __init__(self, params, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps
        self.m = [np.zeros_like(p) for p in params]
        self.v = [np.zeros_like(p) for p in params]
        self.t = 0

    def step(self, params, grads):
        self.t += 1
        c1 = 1.0 - self.b1 ** self.t
        c2 = 1.0 - self.b2 ** self.t
        for p, g, m, v in zip(params, grads, self.m, self.v):
            m *= self.b1
            m += (1.0 - self.b1) * g
            v *= self.b2
            v += (1.0 - self.b2) * g * g
            p -= self.lr * (m / c1) / (np.sqrt(v / c2) + self.eps)
